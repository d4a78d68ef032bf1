// sfk_lane.h -- gfx950 per-lane device code of the linearized-implicit thermochemistry
// update of SFUMATO# (arXiv 2604.21438).
//
// One lane owns one cell.  A lane keeps the whole state (y_H2, y_e, E_th,
// T_d, E_IR, remaining time) in registers for all subcycles of its cell and
// touches HBM only to load it and to store the result.  Cells need from one
// to ~1e5 subcycles, so a wave does not wait for its slowest lane: lanes
// that finish store their cell and are refilled with new cells taken from a
// global work counter (one atomic per wave per refill, indices handed out
// with a ballot + mbcnt prefix), until the counter passes the end.
//
// Per subcycle (paper sections / equations):
//   - derived state: T_g from E_th and n_tot, y_H- = (k_H2/k_H3) y_e,
//     y_H+ = y_e + y_H-, y_H = 1 - 2 y_H2 - y_H+ - y_H-  (conservation);
//   - rate coefficients H0..H11 (Table "Chemical reactions") and heating /
//     cooling 1..13 (Table "Thermal processes") with their exact partial
//     derivatives w.r.t. (y_H2, y_e, T);
//   - subcycle h = f_chem / max(inverse timescales)  (Eqs.
//     timescale_of_dust, timescale_chemi, timescale_energy,
//     timestep_subcycle); dust "tightly coupled" while the dust would need
//     N_req >= N_cyc subcycles for the rest of the interval;
//   - chemistry + energy: (I - h J) du = h f, u = (y_H2, y_e, E/E_ref),
//     3x3 LU with partial pivoting in registers (Eq. eq_deq);
//   - renormalisation to H-nuclei and charge conservation;
//   - dust / IR / gas-grain: one Appendix C linear solve, or, when tightly
//     coupled, backward Euler reduced to one monotone convex equation in T_d
//     solved by Newton from the side where it is positive.
//
// Precision: the template parameter R is the type of the rate / source /
// Jacobian assembly (double for SFC_FP64, float for SFC_MIXED); abundance
// bookkeeping, the LU solves, the state update and the renormalisation are
// always binary64.  Heating and cooling are assembled as Q / (k_B n_H) in
// K/s so that every binary32 intermediate stays inside its normal range.
//
// Included by the plain step (sfk_li.hip) and the served drain
// (sfk_serve.hip); everything here has internal linkage.
#pragma once
#include "sfk.h"

#include <math.h>

namespace sfk {
namespace {

constexpr double KB = 1.380649e-16;
constexpr double MH = 1.67262192e-24;
constexpr double CL = 2.99792458e10;
constexpr double ARAD = 7.5657e-15;
constexpr double LN10 = 2.302585092994045684;
constexpr double RG = 5.83e-8;    // gas-grain coefficient (Appendix C)
constexpr double THIGH = 1000.0;
constexpr double TLOW = 75.0;
constexpr double EVK = 1.602176634e-12 / 1.380649e-16;  // eV / k_B [K]
constexpr double kSrcNoise = 64.0 * 2.220446049250313e-16;  // 64 ulps (dust timescale)

// ------------------------------------------------------------------ math
// 1/x for positive, finite, normal x: hardware estimate and two Newton
// steps (within an ulp; an IEEE divide costs about twice the instructions).
__device__ inline double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(x) for positive, finite, normal x: hardware 1/sqrt estimate, one
// coupled Newton step on (sqrt x, 1/(2 sqrt x)) and two residual
// corrections g += (x - g^2) h (Goldschmidt's iteration, Markstein's form);
// the library sqrt adds range scaling and special-value handling on top.
__device__ inline double fsqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

// e^x in binary64.  x = (n/512) ln2 + r with n = rint(512 x / ln2), the
// product n ln2/512 taken in two parts (the high part has 21 trailing zero
// bits, so it is exact for |n| < 2^21; every x whose result is neither 0
// nor infinite has |n| < 5.6e5); then e^x = 2^(n >> 9) 2^((n & 511)/512) e^r
// with |r| <= ln2/1024, e^r - 1 = r + r^2 (1/2 + r/6 + r^2/24) (truncation
// below 2e-18 relative), and 2^(j/512) (each the nearest binary64, from
// sfk_exp_table.h) read from a table staged in LDS by each kernel
// (stage_tables).  Within one ulp of e^x; 0 below the binary64 range,
// infinity above it.  About 14 VALU instructions and one LDS read against
// ~21 for the library routine, whose wider reduction interval needs a
// degree-11 polynomial.
#include "sfk_exp_table.h"
__shared__ double lds_exp2j512[512];

// ln x in binary64 for positive normal x.  x = m 2^e with m in [0.5, 1);
// c_j = 1/2 + j/256 is the node nearest m (j = 0..128), and with
// i_j = RN(1/c_j), ln x = e ln2 - ln i_j + ln(1 + r), r = m i_j - 1 exact
// to one rounding and |r| <= 1/256, ln(1 + r) by its series to r^7
// (truncation below 2e-18 relative).  -ln i_j is tabulated in high
// precision as a part on the 2^-32 grid plus a remainder, like ln 2, so
// e ln2 + (-ln i_j) is exact in binary64: ln 1 = 0 exactly and results near
// 1 keep their relative accuracy.  Within one ulp; ~21 VALU instructions
// and two LDS reads against ~50 for the library's double-double routine.
__constant__ double kLogTab[129][4] = {
    {0x1.0000000000000p+1, -0x1.62e42ff000000p-1, 0x1.718432a1b0e26p-35, 0.0},
    {0x1.fc07f01fc07f0p+0, -0x1.5ee82aa200000p-1, -0x1.064800e033692p-35, 0.0},
    {0x1.f81f81f81f820p+0, -0x1.5af405c400000p-1, 0x1.36c3fb38a7de7p-34, 0.0},
    {0x1.f44659e4a4271p+0, -0x1.5707a26c00000p-1, 0x1.1ce67e7400cd0p-35, 0.0},
    {0x1.f07c1f07c1f08p+0, -0x1.5322e26800000p-1, -0x1.9e15dcc45d257p-35, 0.0},
    {0x1.ecc07b301ecc0p+0, -0x1.4f45a83600000p-1, 0x1.6c79d145b64eep-35, 0.0},
    {0x1.e9131abf0b767p+0, -0x1.4b6fd6fa00000p-1, 0x1.1e7c175d42567p-34, 0.0},
    {0x1.e573ac901e574p+0, -0x1.47a1527e00000p-1, -0x1.145a742a0d654p-34, 0.0},
    {0x1.e1e1e1e1e1e1ep+0, -0x1.43d9ff3000000p-1, 0x1.b70ed427a4083p-35, 0.0},
    {0x1.de5d6e3f8868ap+0, -0x1.4019c21200000p-1, -0x1.72a4b31b3c3cep-35, 0.0},
    {0x1.dae6076b981dbp+0, -0x1.3c6080c400000p-1, 0x1.2809581b3e7f1p-34, 0.0},
    {0x1.d77b654b82c34p+0, -0x1.38ae217200000p-1, 0x1.a2460feaed55ap-35, 0.0},
    {0x1.d41d41d41d41dp+0, -0x1.35028ada00000p-1, 0x1.39bd4301ab606p-36, 0.0},
    {0x1.d0cb58f6ec074p+0, -0x1.315da44400000p-1, 0x1.7f2ea4278b41ep-34, 0.0},
    {0x1.cd85689039b0bp+0, -0x1.2dbf557c00000p-1, 0x1.e417a06507b9ep-34, 0.0},
    {0x1.ca4b3055ee191p+0, -0x1.2a2786d000000p-1, -0x1.d820da17cf2f1p-34, 0.0},
    {0x1.c71c71c71c71cp+0, -0x1.2696211400000p-1, 0x1.648dc0f882913p-34, 0.0},
    {0x1.c3f8f01c3f8f0p+0, -0x1.230b0d8c00000p-1, 0x1.43683fcc8dbcdp-37, 0.0},
    {0x1.c0e070381c0e0p+0, -0x1.1f8635fc00000p-1, -0x1.859616f4d8060p-35, 0.0},
    {0x1.bdd2b899406f7p+0, -0x1.1c07849a00000p-1, -0x1.cc00daa6f76b8p-34, 0.0},
    {0x1.bacf914c1bad0p+0, -0x1.188ee41000000p-1, 0x1.b86b23b10754cp-34, 0.0},
    {0x1.b7d6c3dda338bp+0, -0x1.151c3f7000000p-1, 0x1.ad3dc16f45276p-34, 0.0},
    {0x1.b4e81b4e81b4fp+0, -0x1.11af823c00000p-1, -0x1.d6aa0be111889p-35, 0.0},
    {0x1.b2036406c80d9p+0, -0x1.0e48986200000p-1, 0x1.c663d6a7f87ffp-34, 0.0},
    {0x1.af286bca1af28p+0, -0x1.0ae76e2e00000p-1, 0x1.f560c79477818p-34, 0.0},
    {0x1.ac5701ac5701bp+0, -0x1.078bf05400000p-1, 0x1.8752f4fb7c241p-34, 0.0},
    {0x1.a98ef606a63bep+0, -0x1.04360be800000p-1, 0x1.3f8a4f2ff3caap-34, 0.0},
    {0x1.a6d01a6d01a6dp+0, -0x1.00e5ae5c00000p-1, 0x1.bf0a9e11d8b94p-34, 0.0},
    {0x1.a41a41a41a41ap+0, -0x1.fb358af800000p-2, 0x1.6ddf1c0b87d37p-36, 0.0},
    {0x1.a16d3f97a4b02p+0, -0x1.f4aa7ee000000p-2, -0x1.8c96e32b780a5p-37, 0.0},
    {0x1.9ec8e951033d9p+0, -0x1.ee2a156c00000p-2, 0x1.7d83692e96e3fp-35, 0.0},
    {0x1.9c2d14ee4a102p+0, -0x1.e7b42c3c00000p-2, -0x1.dad744df591a8p-34, 0.0},
    {0x1.999999999999ap+0, -0x1.e148a1a400000p-2, 0x1.8d9316b207323p-34, 0.0},
    {0x1.970e4f80cb872p+0, -0x1.dae7548400000p-2, -0x1.92c290a53e474p-35, 0.0},
    {0x1.948b0fcd6e9e0p+0, -0x1.d490246c00000p-2, -0x1.efa6a75fd34edp-34, 0.0},
    {0x1.920fb49d0e229p+0, -0x1.ce42f18000000p-2, -0x1.91d0eb798270bp-36, 0.0},
    {0x1.8f9c18f9c18fap+0, -0x1.c7ff9c7400000p-2, -0x1.55327111f56dbp-36, 0.0},
    {0x1.8d3018d3018d3p+0, -0x1.c1c6069400000p-2, 0x1.7189cfc00b8f4p-40, 0.0},
    {0x1.8acb90f6bf3aap+0, -0x1.bb9611b800000p-2, -0x1.c5f7f6fd0299ap-39, 0.0},
    {0x1.886e5f0abb04ap+0, -0x1.b56fa04400000p-2, -0x1.8a429a94b6106p-36, 0.0},
    {0x1.8618618618618p+0, -0x1.af52952400000p-2, -0x1.19b9eceab622fp-35, 0.0},
    {0x1.83c977ab2beddp+0, -0x1.a93ed3c800000p-2, -0x1.5b3c60657d4efp-35, 0.0},
    {0x1.8181818181818p+0, -0x1.a334402400000p-2, 0x1.b058777500c51p-34, 0.0},
    {0x1.7f405fd017f40p+0, -0x1.9d32bea000000p-2, -0x1.5ed3a0c3de5e8p-34, 0.0},
    {0x1.7d05f417d05f4p+0, -0x1.973a343000000p-2, -0x1.356ad8ec5afd2p-34, 0.0},
    {0x1.7ad2208e0ecc3p+0, -0x1.914a863400000p-2, -0x1.bf688b0ad119dp-34, 0.0},
    {0x1.78a4c8178a4c8p+0, -0x1.8b639a8800000p-2, -0x1.65be8c786863fp-35, 0.0},
    {0x1.767dce434a9b1p+0, -0x1.8585577800000p-2, 0x1.2340556199991p-34, 0.0},
    {0x1.745d1745d1746p+0, -0x1.7fafa3bc00000p-2, -0x1.8151c6de6fdb5p-34, 0.0},
    {0x1.724287f46debcp+0, -0x1.79e2668800000p-2, 0x1.8261402d102e9p-37, 0.0},
    {0x1.702e05c0b8170p+0, -0x1.741d876c00000p-2, -0x1.9eec384a4ee30p-36, 0.0},
    {0x1.6e1f76b4337c7p+0, -0x1.6e60ee6c00000p-2, 0x1.0e68d55a83dddp-34, 0.0},
    {0x1.6c16c16c16c17p+0, -0x1.68ac83e800000p-2, -0x1.c6a14ca64eaddp-34, 0.0},
    {0x1.6a13cd1537290p+0, -0x1.630030b400000p-2, 0x1.54ede11f398d7p-36, 0.0},
    {0x1.6816816816817p+0, -0x1.5d5bddf400000p-2, -0x1.95f310eafbaddp-34, 0.0},
    {0x1.661ec6a5122f9p+0, -0x1.57bf753c00000p-2, -0x1.1a3f5b5bdcba8p-35, 0.0},
    {0x1.642c8590b2164p+0, -0x1.522ae07400000p-2, 0x1.d70a2c7bf4d9cp-36, 0.0},
    {0x1.623fa77016240p+0, -0x1.4c9e09e000000p-2, -0x1.72c3ceedc9ea5p-34, 0.0},
    {0x1.6058160581606p+0, -0x1.4718dc2800000p-2, 0x1.c77c7138259f6p-35, 0.0},
    {0x1.5e75bb8d015e7p+0, -0x1.419b423c00000p-2, -0x1.5e8c615b76487p-34, 0.0},
    {0x1.5c9882b931057p+0, -0x1.3c25277400000p-2, 0x1.99cf975693f28p-35, 0.0},
    {0x1.5ac056b015ac0p+0, -0x1.36b6776c00000p-2, 0x1.eeea1324f0e88p-38, 0.0},
    {0x1.58ed2308158edp+0, -0x1.314f1e1c00000p-2, -0x1.35ce348a59bd8p-34, 0.0},
    {0x1.571ed3c506b3ap+0, -0x1.2bef07cc00000p-2, -0x1.c9354b7494a01p-34, 0.0},
    {0x1.5555555555555p+0, -0x1.2696211400000p-2, 0x1.648dd0f882913p-35, 0.0},
    {0x1.5390948f40febp+0, -0x1.214456d000000p-2, -0x1.d71a9d5eba46cp-35, 0.0},
    {0x1.51d07eae2f815p+0, -0x1.1bf9963400000p-2, -0x1.a6b9485aa28f8p-34, 0.0},
    {0x1.5015015015015p+0, -0x1.16b5ccbc00000p-2, 0x1.3048caa410b5dp-34, 0.0},
    {0x1.4e5e0a72f0539p+0, -0x1.1178e82400000p-2, 0x1.81b8591cc74bep-34, 0.0},
    {0x1.4cab88725af6ep+0, -0x1.0c42d67800000p-2, 0x1.e9d1e569d3863p-34, 0.0},
    {0x1.4afd6a052bf5bp+0, -0x1.0713860400000p-2, -0x1.ab0c7f6d8b76ap-35, 0.0},
    {0x1.49539e3b2d067p+0, -0x1.01eae56400000p-2, 0x1.9396ec4c1485fp-34, 0.0},
    {0x1.47ae147ae147bp+0, -0x1.f991c6c800000p-3, -0x1.9d9bd1ecca0cep-34, 0.0},
    {0x1.460cbc7f5cf9ap+0, -0x1.ef5ade5000000p-3, 0x1.1800d688ab2dep-34, 0.0},
    {0x1.446f86562d9fbp+0, -0x1.e530f00000000p-3, 0x1.8efed7dd89fbep-35, 0.0},
    {0x1.42d6625d51f87p+0, -0x1.db13db1000000p-3, 0x1.5bb5fb15ee2b6p-34, 0.0},
    {0x1.4141414141414p+0, -0x1.d1037f2800000p-3, 0x1.aa18527e75b6fp-35, 0.0},
    {0x1.3fb013fb013fbp+0, -0x1.c6ffbc7000000p-3, 0x1.fe11ed72c5963p-36, 0.0},
    {0x1.3e22cbce4a902p+0, -0x1.bd08738000000p-3, -0x1.dec54f774d57ep-34, 0.0},
    {0x1.3c995a47babe7p+0, -0x1.b31d857800000p-3, 0x1.218e2886a7567p-34, 0.0},
    {0x1.3b13b13b13b14p+0, -0x1.a93ed3c800000p-3, -0x1.5b3cade57d4efp-36, 0.0},
    {0x1.3991c2c187f63p+0, -0x1.9f6c407000000p-3, -0x1.12cc556b432c1p-36, 0.0},
    {0x1.3813813813814p+0, -0x1.95a5add000000p-3, 0x1.1fcfb3af4ebe0p-36, 0.0},
    {0x1.3698df3de0748p+0, -0x1.8beafeb000000p-3, -0x1.c7f47755aa8b7p-34, 0.0},
    {0x1.3521cfb2b78c1p+0, -0x1.823c165800000p-3, 0x1.72e1fd24659cep-34, 0.0},
    {0x1.33ae45b57bcb2p+0, -0x1.7898d85800000p-3, 0x1.dd9c5f9070914p-34, 0.0},
    {0x1.323e34a2b10bfp+0, -0x1.6f0128b800000p-3, 0x1.52a8e26f2ce11p-36, 0.0},
    {0x1.30d190130d190p+0, -0x1.6574ebe800000p-3, -0x1.82672e2cb0f0cp-36, 0.0},
    {0x1.2f684bda12f68p+0, -0x1.5bf406b800000p-3, 0x1.5e128023eb68ap-34, 0.0},
    {0x1.2e025c04b8097p+0, -0x1.527e5e4800000p-3, -0x1.0dac6791cad30p-34, 0.0},
    {0x1.2c9fb4d812ca0p+0, -0x1.4913d83000000p-3, -0x1.9dab16f2a9fb7p-34, 0.0},
    {0x1.2b404ad012b40p+0, -0x1.3fb45a5800000p-3, -0x1.928c989e06573p-35, 0.0},
    {0x1.29e4129e4129ep+0, -0x1.365fcb0000000p-3, -0x1.590146fa8234bp-35, 0.0},
    {0x1.288b01288b013p+0, -0x1.2d1610c800000p-3, -0x1.a04f43b32e06dp-37, 0.0},
    {0x1.27350b8812735p+0, -0x1.23d712a800000p-3, 0x1.b1eff55c702c2p-34, 0.0},
    {0x1.25e22708092f1p+0, -0x1.1aa2b7e000000p-3, -0x1.1fb94adc88713p-34, 0.0},
    {0x1.2492492492492p+0, -0x1.1178e82000000p-3, -0x1.3f23cef19c5a1p-34, 0.0},
    {0x1.23456789abcdfp+0, -0x1.08598b5800000p-3, -0x1.e3a0680a3fd9cp-35, 0.0},
    {0x1.21fb78121fb78p+0, -0x1.fe8913a000000p-4, 0x1.2154db593e843p-35, 0.0},
    {0x1.20b470c67c0d9p+0, -0x1.ec73983000000p-4, -0x1.4224cf75019bap-37, 0.0},
    {0x1.1f7047dc11f70p+0, -0x1.da72764000000p-4, 0x1.eee586bfe058fp-34, 0.0},
    {0x1.1e2ef3b3fb874p+0, -0x1.c885802000000p-4, 0x1.0ed3815c734aap-34, 0.0},
    {0x1.1cf06ada2811dp+0, -0x1.b6ac88e000000p-4, 0x1.4a938d002bf77p-34, 0.0},
    {0x1.1bb4a4046ed29p+0, -0x1.a4e7641000000p-4, 0x1.390f219b5ca20p-34, 0.0},
    {0x1.1a7b9611a7b96p+0, -0x1.9335e5d000000p-4, -0x1.65261eb8757a9p-34, 0.0},
    {0x1.19453808ca29cp+0, -0x1.8197e2f000000p-4, -0x1.038fbf6e7cb80p-34, 0.0},
    {0x1.1811811811812p+0, -0x1.700d30b000000p-4, 0x1.53f17cb92b311p-36, 0.0},
    {0x1.16e0689427379p+0, -0x1.5e95a4e000000p-4, 0x1.a1b8cd4c78ba4p-34, 0.0},
    {0x1.15b1e5f75270dp+0, -0x1.4d3115d000000p-4, -0x1.03f560ed3e859p-35, 0.0},
    {0x1.1485f0e0acd3bp+0, -0x1.3bdf5a8000000p-4, 0x1.708d0f056892cp-35, 0.0},
    {0x1.135c81135c811p+0, -0x1.2aa04a4000000p-4, -0x1.1c5e85aea2c73p-34, 0.0},
    {0x1.12358e75d3033p+0, -0x1.1973bd1000000p-4, -0x1.1955828553e4cp-34, 0.0},
    {0x1.1111111111111p+0, -0x1.08598b6000000p-4, 0x1.8717e9dd70099p-34, 0.0},
    {0x1.0fef010fef011p+0, -0x1.eea31c0000000p-5, -0x1.ae1ef41b036c5p-39, 0.0},
    {0x1.0ecf56be69c90p+0, -0x1.ccb73ce000000p-5, 0x1.126983c91f60ap-36, 0.0},
    {0x1.0db20a88f4696p+0, -0x1.aaef2d0000000p-5, -0x1.f62210b46a777p-34, 0.0},
    {0x1.0c9714fbcda3bp+0, -0x1.894aa14000000p-5, -0x1.3f66956a2fa5ep-34, 0.0},
    {0x1.0b7e6ec259dc8p+0, -0x1.67c94f2000000p-5, -0x1.a976ca8209f33p-34, 0.0},
    {0x1.0a6810a6810a7p+0, -0x1.466aed4000000p-5, -0x1.6f1fc66452101p-36, 0.0},
    {0x1.0953f39010954p+0, -0x1.252f330000000p-5, 0x1.cb9eff947f792p-35, 0.0},
    {0x1.0842108421084p+0, -0x1.0415d8a000000p-5, 0x1.8bbbf8fe8c38ap-37, 0.0},
    {0x1.073260a47f7c6p+0, -0x1.c63d2ec000000p-6, -0x1.4aad70c7f3d66p-38, 0.0},
    {0x1.0624dd2f1a9fcp+0, -0x1.8492528000000p-6, -0x1.919589173697dp-35, 0.0},
    {0x1.05197f7d73404p+0, -0x1.432a924000000p-6, -0x1.980cbb9cc9432p-34, 0.0},
    {0x1.0410410410410p+0, -0x1.0205658000000p-6, -0x1.26b06e93e4742p-35, 0.0},
    {0x1.03091b51f5e1ap+0, -0x1.82448a0000000p-7, -0x1.c45141904b161p-34, 0.0},
    {0x1.0204081020408p+0, -0x1.0101578000000p-7, 0x1.3b90cb6b999d3p-34, 0.0},
    {0x1.0101010101010p+0, -0x1.0080560000000p-8, 0x1.a9dd36a0699c7p-34, 0.0},
    {0x1.0000000000000p+0, 0x0.0p+0, 0x0.0p+0, 0.0}};
__shared__ __attribute__((aligned(32))) double lds_logtab[129][4];

// Every kernel that evaluates the per-lane code calls this first, with all
// threads of the block (it ends with a barrier).
__device__ inline void stage_tables() {
  for (unsigned i = threadIdx.x; i < 512u; i += blockDim.x) lds_exp2j512[i] = kExp2j512[i];
  for (unsigned i = threadIdx.x; i < 129u * 4u; i += blockDim.x)
    (&lds_logtab[0][0])[i] = (&kLogTab[0][0])[i];
  __syncthreads();
}

__device__ inline double fexp(double x) {
  const double n = __builtin_rint(x * 738.6598609351493);  // 512 / ln2
  double r = fma(-n, 0x1.62e42fee00000p-10, x);
  r = fma(-n, 0x1.a39ef35793c76p-42, r);
  const double p = fma(fma(r, 1.0 / 24.0, 1.0 / 6.0), r, 0.5);
  const double q = fma(r * r, p, r);
  const int ni = int(n);
  const double t = lds_exp2j512[ni & 511];
  return __builtin_ldexp(fma(t, q, t), ni >> 9);
}

__device__ inline double flog(double x) {
  const double m = __builtin_amdgcn_frexp_mant(x);
  const int e = __builtin_amdgcn_frexp_exp(x);
  const int j = int(__builtin_rint(fma(m, 256.0, -128.0)));
  const double* t = lds_logtab[j];
  const double r = fma(m, t[0], -1.0);
  double q = fma(r, 1.0 / 7.0, -1.0 / 6.0);
  q = fma(r, q, 1.0 / 5.0);
  q = fma(r, q, -0.25);
  q = fma(r, q, 1.0 / 3.0);
  q = fma(r, q, -0.5);
  const double p = fma(r * r, q, r);
  const double de = double(e);
  const double hi = fma(de, 0x1.62e42ff000000p-1, t[1]);  // ln 2 on the 2^-32 grid
  const double lo = fma(de, -0x1.718432a1b0e26p-35, t[2]);
  return hi + (lo + p);
}

template <class R>
struct Mth;
template <>
struct Mth<double> {
  __device__ static double ea(double x) { return fexp(x); }
  __device__ static double ex(double x) { return fexp(x); }
  __device__ static double lg(double x) { return flog(x); }
  // every root and quotient in the assembly has a positive, normal argument
  // (temperatures are clamped to [1, 1e8] K or floored at T_CMB)
  __device__ static double sq(double x) { return fsqrt(x); }
  __device__ static double dv(double a, double b) { return a * frcp(b); }
};
template <>
struct Mth<float> {
  // e^x for a binary64 argument: the range reduction x log2(e) = n + f,
  // |f| <= 1/2, is done in binary64 so that large arguments (theta/T up to
  // ~1e4) lose nothing; 2^f comes from the hardware v_exp_f32 (about one
  // binary32 ulp), the result is scaled by 2^n (flushing to zero below the
  // binary32 range).
  __device__ static float ea(double x) {
    const double t = x * 1.4426950408889634;
    const double n = rint(fmax(fmin(t, 256.0), -256.0));
    const float r = __builtin_amdgcn_exp2f(float(t - n));
    return __builtin_amdgcn_ldexpf(r, int(n));
  }
  // hardware transcendental unit: v_exp_f32 / v_log_f32 are base 2
  __device__ static float ex(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
  __device__ static float lg(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }
  __device__ static float sq(float x) { return __builtin_amdgcn_sqrtf(x); }
  __device__ static float dv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
};

// Value with partials w.r.t. (y_H2, y_e, T).  The mask M says which
// partials can be non-zero (kDA: d/dy_H2, kDE: d/dy_e, kDT: d/dT); the
// others are exactly zero by construction (y_H2 does not depend on y_e,
// a rate coefficient depends on T only, ...).  The operators compute only
// the partials in the result's mask, so the structural zeros are neither
// multiplied nor added: IEEE arithmetic does not let the compiler drop
// x * 0 or x + 0 * y on its own.  Absent partials hold an exact 0.
constexpr unsigned kDA = 1u, kDE = 2u, kDT = 4u, kDAll = 7u;
template <class R, unsigned M>
struct D {
  R v, a, e, t;
};
template <class R>
using G = D<R, kDAll>;  // all partials
template <class R, unsigned M>
__device__ inline G<R> dense(D<R, M> x) {
  return {x.v, x.a, x.e, x.t};
}
// function of T only
template <class R>
struct TF {
  R v, t;
};

template <unsigned B, unsigned M1, unsigned M2, class R>
__device__ inline R p_add(R x, R y) {
  if constexpr ((M1 & B) && (M2 & B)) return x + y;
  else if constexpr ((M1 & B) != 0) return x;
  else if constexpr ((M2 & B) != 0) return y;
  else return R(0);
}
template <unsigned B, unsigned M1, unsigned M2, class R>
__device__ inline R p_sub(R x, R y) {
  if constexpr ((M1 & B) && (M2 & B)) return x - y;
  else if constexpr ((M1 & B) != 0) return x;
  else if constexpr ((M2 & B) != 0) return -y;
  else return R(0);
}
// partial of a product: x' y + x y'
template <unsigned B, unsigned M1, unsigned M2, class R>
__device__ inline R p_mul(R xp, R yv, R xv, R yp) {
  if constexpr ((M1 & B) && (M2 & B)) return xp * yv + xv * yp;
  else if constexpr ((M1 & B) != 0) return xp * yv;
  else if constexpr ((M2 & B) != 0) return xv * yp;
  else return R(0);
}
template <unsigned B, unsigned M, class R>
__device__ inline R p_scale(R s, R xp) {
  if constexpr ((M & B) != 0) return s * xp;
  else return R(0);
}

template <class R, unsigned M1, unsigned M2>
__device__ inline D<R, M1 | M2> operator+(D<R, M1> x, D<R, M2> y) {
  return {x.v + y.v, p_add<kDA, M1, M2>(x.a, y.a), p_add<kDE, M1, M2>(x.e, y.e),
          p_add<kDT, M1, M2>(x.t, y.t)};
}
template <class R, unsigned M1, unsigned M2>
__device__ inline D<R, M1 | M2> operator-(D<R, M1> x, D<R, M2> y) {
  return {x.v - y.v, p_sub<kDA, M1, M2>(x.a, y.a), p_sub<kDE, M1, M2>(x.e, y.e),
          p_sub<kDT, M1, M2>(x.t, y.t)};
}
template <class R, unsigned M1, unsigned M2>
__device__ inline D<R, M1 | M2> operator*(D<R, M1> x, D<R, M2> y) {
  return {x.v * y.v, p_mul<kDA, M1, M2>(x.a, y.v, x.v, y.a),
          p_mul<kDE, M1, M2>(x.e, y.v, x.v, y.e), p_mul<kDT, M1, M2>(x.t, y.v, x.v, y.t)};
}
template <class R, unsigned M>
__device__ inline D<R, M> operator*(R s, D<R, M> x) {
  return {s * x.v, p_scale<kDA, M>(s, x.a), p_scale<kDE, M>(s, x.e), p_scale<kDT, M>(s, x.t)};
}
template <class R, unsigned M>
__device__ inline D<R, M | kDT> operator*(TF<R> k, D<R, M> x) {
  return {k.v * x.v, p_scale<kDA, M>(k.v, x.a), p_scale<kDE, M>(k.v, x.e),
          p_mul<kDT, kDT, M>(k.t, x.v, k.v, x.t)};
}
// quotient: partials (x' - q y') / y
template <unsigned B, unsigned M1, unsigned M2, class R>
__device__ inline R p_quot(R xp, R q, R yp, R iy) {
  if constexpr ((M1 & B) && (M2 & B)) return (xp - q * yp) * iy;
  else if constexpr ((M1 & B) != 0) return xp * iy;
  else if constexpr ((M2 & B) != 0) return -(q * yp) * iy;
  else return R(0);
}
template <class R, unsigned M1, unsigned M2>
__device__ inline D<R, M1 | M2> quot(D<R, M1> x, D<R, M2> y) {
  using Mt = Mth<R>;
  const R iy = Mt::dv(R(1), y.v);
  const R q = x.v * iy;
  return {q, p_quot<kDA, M1, M2>(x.a, q, y.a, iy), p_quot<kDE, M1, M2>(x.e, q, y.e, iy),
          p_quot<kDT, M1, M2>(x.t, q, y.t, iy)};
}

// ------------------------------------------------------------------ rates
// k_H2 (H + e -> H- + photon) and k_H3 (H- + H -> H2 + e), Table
// "Chemical reactions"; powers of T through one shared ln T.
// k_H3 fit: exponents a_i, coefficients c_i, and c_i a_i (for dk/dT)
__constant__ double kH3[3][6] = {
    {0.098493, 0.5561, 2.1826, 1.0461, 3.0424, 3.7741},
    {1.0, 0.32852, 2.771e-7, 6.191e-3, 8.9712e-11, 3.2576e-14},
    {0.098493, 0.32852 * 0.5561, 2.771e-7 * 2.1826, 6.191e-3 * 1.0461, 8.9712e-11 * 3.0424,
     3.2576e-14 * 3.7741}};

template <class R>
__device__ inline void k2k3(double T, double lnT, double iT, TF<R>& k2, TF<R>& k3) {
  using M = Mth<R>;
  k2.v = M::ea(-41.11005943727161 + 0.928 * lnT - T * (1.0 / 16200.0));  // ln 1.4e-18
  k2.t = k2.v * R(0.928 * iT - 1.0 / 16200.0);
  // N = T^a0 + c1 T^a1 + c2 T^a2 and D = 1 + c3 T^a3 + c4 T^a4 + c5 T^a5:
  // the six powers are independent exponentials, unrolled so that their
  // dependent FMA chains overlap (the kernel's register peak lies elsewhere)
  R N = R(0), dN = R(0), D = R(1), dD = R(0);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const R p = M::ea(kH3[0][i] * lnT);
    if (i < 3) {
      N = N + R(kH3[1][i]) * p;
      dN = dN + R(kH3[2][i]) * p;
    } else {
      D = D + R(kH3[1][i]) * p;
      dD = dD + R(kH3[2][i]) * p;
    }
  }
  const R iN = M::dv(R(1), N), iD = M::dv(R(1), D);
  k3.v = R(1.35e-9) * N * iD;
  k3.t = k3.v * (dN * iN - dD * iD) * R(iT);
}

template <class R>
struct Chem {
  double f[3];   // R_H2, R_e [1/s], Q/(k_B n_H) [K/s]
  R J[3][3];     // d f_i / d (y_H2, y_e, T) at fixed others
  R ratio;       // k_H2 / k_H3 (steady-state y_H- / y_e)
};

// Accumulator of a net source (R_H2, R_e, Q): value in binary64 in both
// precisions, partials in R.  A net source near balance is a small
// difference of large formation and destruction (heating and cooling)
// terms; summed in binary32 its relative error would be eps_32 times
// gross / net, and the step-size control, which divides abundances and
// energy by these net sources, would follow that rounding noise.
template <class R>
struct Acc {
  double v;
  R a, e, t;
};

// Per-cell constants that do not change during a call.
struct CellK {
  double n, fd, rho;
  double k9, k10, k11;  // photo / CR rates
  double g4;            // photoelectric heating / (k_B n) [K/s] (pe_mode 0), G0 (pe_mode 1)
  double euv;           // dust UV absorption [erg/g/s]
  double ikn, irho;     // 1 / (k_B n), 1 / rho
  double rho_kn;        // rho / (k_B n)
};

// A += s * (k * x), k a function of T only; the accumulator's mask holds x's
template <class R, unsigned MA, unsigned M>
__device__ inline void acc(D<R, MA>& A, R s, TF<R> k, D<R, M> x) {
  static_assert((M | kDT | MA) == MA, "accumulator lacks a partial of the term");
  const R kv = s * k.v, kt = s * k.t;
  A.v = A.v + kv * x.v;
  if constexpr ((M & kDA) != 0) A.a = A.a + kv * x.a;
  if constexpr ((M & kDE) != 0) A.e = A.e + kv * x.e;
  if constexpr ((M & kDT) != 0) A.t = A.t + (kt * x.v + kv * x.t);
  else A.t = A.t + kt * x.v;
}
// the same into a net-source accumulator: each term rounded in R, the sum
// in binary64 (for R = double the arithmetic of the overload above)
template <class R, unsigned M>
__device__ inline void acc(Acc<R>& A, R s, TF<R> k, D<R, M> x) {
  const R kv = s * k.v, kt = s * k.t;
  A.v = A.v + double(kv) * double(x.v);
  if constexpr ((M & kDA) != 0) A.a = A.a + kv * x.a;
  if constexpr ((M & kDE) != 0) A.e = A.e + kv * x.e;
  if constexpr ((M & kDT) != 0) A.t = A.t + (kt * x.v + kv * x.t);
  else A.t = A.t + kt * x.v;
}

// Chemistry and gas heating/cooling with partials; T_d frozen.  Each rate
// coefficient is evaluated once and all of its contributions (reaction
// rate and the heating / cooling it drives) are added to the three
// accumulators at once.  Temperature, 1/T, ln T, the fit polynomials and
// every exponent argument are binary64 in both precisions; R is the type
// of the exponentials' results and of the products and partials.  kS
// compiles in the pieces beside the solver that the network can switch on
// (H2 self-shielding, grain-charge photoelectric heating); without it their
// branches, and the registers they hold, are gone.
template <class R, bool kS>
__device__ void assemble(const Net& nt, const Par& pr, double y2d, double yed, double Td_,
                         double Tin, const CellK& ck, Chem<R>& out) {
  using M = Mth<R>;
  double Tc = Tin;
  R clampT = R(1);
  if (Tc < 1.0) { Tc = 1.0; clampT = R(0); }
  if (Tc > 1.0e8) { Tc = 1.0e8; clampT = R(0); }
  const double T64 = Tc;
  const double iT64 = frcp(Tc);
  const double lnT64 = flog(Tc);
  const R T = R(T64);
  const R n = R(ck.n);
  const R iT = R(iT64);
  // every half-integer power of T below comes from one root and one
  // reciprocal: T^1/2, T^-1/2, T^-1/4 = (T^-1/2)^1/2
  const R sT = M::sq(T);
  const R rsT = M::dv(R(1), sT);

  // ---- steady-state H- and the abundances (values in binary64) ----
  R ratio = R(0), dratio = R(0);
  TF<R> k2, k3;  // k3 is used again by Gamma_1 below
  {
    k2k3<R>(T64, lnT64, iT64, k2, k3);
    k2.v *= R(nt.rm[2]);
    k2.t *= R(nt.rm[2]);
    if (nt.rm[3] > 0.0) {
      const R i3 = M::dv(R(1), R(nt.rm[3]) * k3.v);
      ratio = k2.v * i3;
      dratio = (k2.t - ratio * R(nt.rm[3]) * k3.t) * i3;
    }
  }
  out.ratio = ratio;
  const double rd = double(ratio);
  const double yhm_d = rd * yed;
  const double yhp_d = yed + yhm_d;
  const double yh_d = 1.0 - 2.0 * y2d - yhp_d - yhm_d;
  const R ye = R(yed);
  const D<R, kDA> Y2{R(y2d), R(1), R(0), R(0)};
  const D<R, kDE> YE{ye, R(0), R(1), R(0)};
  const D<R, kDE | kDT> YHM{R(yhm_d), R(0), ratio, dratio * ye};
  const D<R, kDE | kDT> YHP{R(yhp_d), R(0), R(1) + ratio, dratio * ye};
  const G<R> YH{R(yh_d), R(-2), R(-1) - R(2) * ratio, R(-2) * dratio * ye};
  const auto HE = YH * YE;

  Acc<R> rh2{0.0, R(0), R(0), R(0)}, re = rh2, q = rh2;
  const R evn = R(EVK) * n;  // eV / k_B * n_H

  // H2 (through the H- channel, H3): net H2 formation k_H2 n y_H y_e;
  // Lambda_8, H- free-bound cooling k_B T k_H2 n(H) n(e)
  acc(rh2, n, k2, HE);
  acc(q, -R(nt.pm[7]) * n, TF<R>{T * k2.v, k2.v + T * k2.t}, HE);

  // H0 collisional ionisation (fit in ln T[eV]) and Lambda_5
  {
    const double x = lnT64 - 9.359149794498732;  // ln(k_B / eV)
    const double c[9] = {-32.71396786, 13.536556, -5.73932875, 1.563154998, -0.2877056,
                         3.48255977e-2, -2.63197617e-3, 1.11954395e-4, -2.03914985e-6};
    double P = c[8], dP = 8.0 * c[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) P = P * x + c[i];
#pragma unroll
    for (int i = 7; i >= 1; --i) dP = dP * x + double(i) * c[i];
    TF<R> k0;
    k0.v = R(nt.rm[0]) * M::ea(P);
    k0.t = k0.v * R(dP * iT64);
    acc(re, n, k0, HE);
    acc(q, -R(nt.pm[4] * 13.6) * evn, k0, HE);
  }
  // H1 radiative recombination
  {
    const R w = M::ea(0.407 * (11.654320855151537 - lnT64));  // ln 115188
    const double L = -31.22350007575617 + 1.5 * (12.662275226919286 - lnT64) -
                     2.242 * double(M::lg(R(1) + w));  // ln 2.753e-14, ln 315614
    TF<R> k1;
    k1.v = R(nt.rm[1]) * M::ea(L);
    k1.t = k1.v * iT * (R(-1.5) + R(2.242 * 0.407) * w * M::dv(R(1), R(1) + w));
    acc(re, -n, k1, YHP * YE);
  }
  // Gamma_1 factor f = (1 + n_cr/n_H)^-1 = n D / (n D + 1e6 T^-1/2)
  G<R> f;
  {
    const double e1x = 400.0 * iT64;
    const R e1 = M::ea(-e1x * e1x);
    const double iT12 = frcp(T64 + 1200.0);
    const R e2 = M::ea(-12000.0 * iT12);
    G<R> nD{R(0), R(0), R(0), R(0)};
    acc(nD, R(1.6) * n, TF<R>{e1, e1 * R(2.0 * e1x * e1x * iT64)}, YH);
    acc(nD, R(1.4) * n, TF<R>{e2, e2 * R(12000.0 * iT12 * iT12)}, Y2);
    const R g = R(1e6) * rsT;
    const G<R> den{nD.v + g, nD.a, nD.e, nD.t - R(0.5) * g * iT};
    f = quot(nD, den);
  }
  const R g1 = R(nt.pm[0]) * evn;  // Gamma_1 prefactor
  // H3 in Gamma_1: 3.73 eV per H2 formed through H-
  {
    const TF<R> k3m{k3.v * R(nt.rm[3]), k3.t * R(nt.rm[3])};
    acc(q, g1 * R(3.73), k3m, f * (YH * YHM));
  }
  const auto H2H = Y2 * YH;
  const auto H22 = Y2 * Y2;
  // H4 collisional dissociation by H (stand-in rate) and Lambda_6 (part)
  {
    TF<R> k4;
    k4.v = R(nt.rm[4] * nt.k4_pre) * M::ea(-nt.k4_theta * iT64);
    k4.t = k4.v * R(nt.k4_theta * iT64 * iT64);
    acc(rh2, -n, k4, H2H);
    acc(q, -R(nt.pm[5] * 4.48) * evn, k4, H2H);
  }
  // H5 three-body formation, H6 = H5/8, and Gamma_1 (4.48 eV per H2)
  {
    const R t50 = rsT;
    const R t25 = M::sq(rsT);
    const TF<R> k5{R(6.0e-32) * t25 + R(2.0e-31) * t50,
                   (R(-0.25 * 6.0e-32) * t25 - R(0.5 * 2.0e-31) * t50) * iT};
    const auto HH = YH * YH;
    const auto HHH = HH * YH;
    acc(rh2, R(nt.rm[5]) * n * n, k5, HHH);
    acc(rh2, R(nt.rm[6] * 0.125) * n * n, k5, HH * Y2);
    acc(q, g1 * R(4.48) * n * R(nt.rm[5]), k5, f * HHH);
  }
  // H7 collisional dissociation by H2: k_high^(1-a) k_low^a in ln space
  {
    const double lnkl = -22.860336491462885 - 6.95e4 * iT64;  // ln 1.18e-10
    const double dlnkl = 6.95e4 * iT64 * iT64;
    const R eb = M::ea(-6000.0 * iT64);
    // ln(1 - e^(-6000/T)): the plain log of 1 - eb is as accurate in
    // absolute terms (all that enters ln k) as log1p, at a third of the cost
    const double lnkh = -16.325735015736566 - 0.5 * lnT64 - 5.2e4 * iT64 +
                        double(M::lg(R(1) - eb));  // ln 8.125e-8
    const double ebd = double(eb);
    const double dlnkh = -0.5 * iT64 + 5.2e4 * iT64 * iT64 -
                         ebd * 6000.0 * iT64 * iT64 * frcp(1.0 - ebd);
    const double t = lnT64 * (1.0 / LN10) - 4.0;
    const R ncr = M::ea(LN10 * (4.845 - 1.3 * t + 1.62 * t * t));
    const double a = double(ncr * M::dv(R(1), ncr + n));
    const double da = a * (1.0 - a) * (-1.3 + 3.24 * t) * iT64;
    TF<R> k7;
    k7.v = R(nt.rm[7]) * M::ea((1.0 - a) * lnkh + a * lnkl);
    k7.t = k7.v * R((1.0 - a) * dlnkh + a * dlnkl + (lnkl - lnkh) * da);
    acc(rh2, -n, k7, H22);
    acc(q, -R(nt.pm[5] * 4.48) * evn, k7, H22);
  }
  // H8 formation on grains (T_d frozen) and Gamma_1 (0.2 + 4.2 f eV)
  {
    const R Td = R(Td_);
    const R fa = M::dv(R(1), R(1) + M::ea(750.0 * (1.0 / 75.0 - frcp(Td_))));
    const R s = M::sq(T + Td);
    const R D = R(1) + R(0.04) * s + R(2e-3) * T + R(8e-6) * T * T;
    const R iD = M::dv(R(1), D);
    TF<R> k8;
    k8.v = R(nt.rm[8] * 6.0e-17 * 0.057735026918962574) * sT * fa * R(ck.fd) * iD;  // 300^-1/2
    k8.t = k8.v * (R(0.5) * iT - (R(0.02) * M::dv(R(1), s) + R(2e-3) + R(1.6e-5) * T) * iD);
    acc(rh2, n, k8, YH);
    const G<R> fc{R(0.2) + R(4.2) * f.v, R(4.2) * f.a, R(4.2) * f.e, R(4.2) * f.t};
    acc(q, g1, k8, fc * YH);
  }
  // H9, H10, H11 (photo / cosmic-ray rates of the cell) and Gamma_2..4
  {
    const R k9 = R(ck.k9), k10 = R(ck.k10), k11 = R(ck.k11);
    acc(re, k9 + k11, TF<R>{R(1), R(0)}, YH);
    acc(q, R(nt.pm[1] * nt.g2k) * k9, TF<R>{R(1), R(0)}, YH);
    if (kS && nt.shield_mode == 1) {
      // H2 self-shielding (stand-in, the fit of Draine & Bertoldi 1996):
      // f = 0.965 / (1 + x/b5)^2 + 0.035 / s exp(-8.5e-4 s), s = sqrt(1 + x),
      // x = y_H2 sh_k sqrt(n_H T) (local column of shield_len Jeans lengths)
      const double xk = pr.sh_k * fsqrt(ck.n * T64);  // dx / dy_H2
      const double x = y2d * xk;
      const R iu = M::dv(R(1), R(1) + R(x / nt.sh_b5));
      const R sq = M::sq(R(1) + R(x));
      const R isq = M::dv(R(1), sq);
      const R ex = M::ea(-8.5e-4 * double(sq));
      const R f = R(0.965) * iu * iu + R(0.035) * isq * ex;
      const R dfdx = R(-2.0 * 0.965 / nt.sh_b5) * iu * iu * iu +
                     R(0.5 * 0.035) * ex * isq * (-(isq * isq) - R(8.5e-4) * isq);
      const D<R, kDA | kDT> fsh{f, dfdx * R(xk), R(0), dfdx * R(x) * R(0.5) * iT};
      const auto S2 = fsh * Y2;
      acc(rh2, -k10, TF<R>{R(1), R(0)}, S2);
      acc(q, R(nt.pm[2] * nt.g3k) * k10, TF<R>{R(1), R(0)}, S2);
    } else {
      acc(rh2, -k10, TF<R>{R(1), R(0)}, Y2);
      acc(q, R(nt.pm[2] * nt.g3k) * k10, TF<R>{R(1), R(0)}, Y2);
    }
    if (!kS || nt.pe_mode != 1) {
      q.v = q.v + ck.g4;
    } else if (ck.g4 > 0.0) {
      // photoelectric heating with grain charging and the cooling by
      // electron recombination on grains (stand-in: Bakes & Tielens 1994 in
      // the form of Wolfire et al. 2003), psi = G0 sqrt(T) / n_e with n_e
      // floored at y_abs n_H; per k_B n_H
      const bool floored = yed < pr.y_abs;
      const double lnpsi = flog(ck.g4) + 0.5 * lnT64 - flog((floored ? pr.y_abs : yed) * ck.n);
      const R psi = M::ea(lnpsi);
      const R ipsi = M::ea(-lnpsi);
      const R dpsi_e = floored ? R(0) : -psi * M::dv(R(1), ye);  // d psi / d y_e
      const R dpsi_t = R(0.5) * psi * iT;
      const R p73 = M::ea(0.73 * lnpsi);
      const R ia = M::dv(R(1), R(1) + R(4e-3) * p73);
      const R tt = M::ea(0.7 * (lnT64 - 9.210340371976184));  // (T / 1e4)^0.7
      const R ib = M::dv(R(1), R(1) + R(2e-4) * psi);
      const R eps = R(0.0487) * ia + R(0.0365) * tt * ib;
      const R deps = R(-0.0487 * 4e-3 * 0.73) * p73 * ipsi * ia * ia -
                     R(0.0365 * 2e-4) * tt * ib * ib;  // d eps / d psi
      const R deps_t = R(0.0365 * 0.7) * tt * iT * ib;
      const R ch = R(nt.pe_ch * ck.g4 * ck.fd);
      const R beta = R(0.735) * M::ea(-0.068 * lnT64);
      const R pb = M::ea(double(beta) * lnpsi);
      const R t94 = M::ea(0.94 * lnT64);
      const R cr = R(nt.pe_cr * ck.n * ck.fd);
      const R rec = cr * ye * t94 * pb;
      const R rec_e = cr * t94 * pb * (floored ? R(1) : R(1) - beta);
      const R rec_t = rec * (R(0.94) * iT - R(0.068) * beta * iT * R(lnpsi) + beta * R(0.5) * iT);
      q.v = q.v + (double(ch * eps) - double(rec));
      q.e = q.e + (ch * deps * dpsi_e - rec_e);
      q.t = q.t + (ch * (deps * dpsi_t + deps_t) - rec_t);
    }
  }
  // Lambda_7, recombination cooling fit in log10 T (10^P / k_B)
  {
    const double l = lnT64 * (1.0 / LN10);
    const double c[6] = {-25.87, 0.4958, -0.1052, 0.04264, -9.165e-3, 5.491e-4};
    double P = c[5], dP = 5.0 * c[5];
#pragma unroll
    for (int i = 4; i >= 0; --i) P = P * l + c[i];
#pragma unroll
    for (int i = 4; i >= 1; --i) dP = dP * l + double(i) * c[i];
    const R v = M::ea(LN10 * P + 36.51880780943216);  // - ln k_B
    acc(q, -R(nt.pm[6]) * n, TF<R>{v, v * R(dP * iT64)}, YHP * YE);
  }
  // Lambda_9 (H excitation, partner n(H)) and Lambda_10 (He+, all He ionised)
  {
    const R s5 = R(0.0031622776601683794) * sT;  // (T / 1e5)^1/2
    const R ds5 = R(0.5) * s5 * iT;
    const R i5 = M::dv(R(1), R(1) + s5);
    const R v9 = R(7.5e-19 / KB) * M::ea(-118348.0 * iT64) * i5;
    acc(q, -R(nt.pm[8]) * n, TF<R>{v9, v9 * (R(118348.0 * iT64 * iT64) - ds5 * i5)}, HE);
    const R v10 = R(5.54e-17 / KB) * M::ea(-0.397 * lnT64 - 473638.0 * iT64) * i5;
    acc(q, -R(nt.pm[9] * pr.y_he) * n,
        TF<R>{v10, v10 * (R(-0.397 * iT64 + 473638.0 * iT64 * iT64) - ds5 * i5)}, YE);
  }
  // Lambda_11, free-free with the piecewise Gaunt factor
  {
    const R l = R(lnT64 * (1.0 / LN10));
    R gff, dg;
    if (T64 < 3.2e5) {
      gff = R(0.79464) + R(0.1243) * l;
      dg = R(0.1243 / LN10) * iT;
    } else {
      gff = R(2.13164) - R(0.1240) * l;
      dg = R(-0.1240 / LN10) * iT;
    }
    acc(q, -R(nt.pm[10]) * n,
        TF<R>{R(1.426e-27 / KB) * sT * gff,
              R(1.426e-27 / KB) * (R(0.5) * gff * rsT + sT * dg)},
        YHP * YE);
  }
  // Lambda_12, Compton cooling off the CMB
  {
    const R cc = R(pr.compton);
    acc(q, R(-1), TF<R>{R(double(cc) * (T64 - pr.t_cmb)), cc}, YE);
  }
  // Lambda_13, line cooling: two-level coolants (stand-in)
  {
    const R s100 = R(10) * rsT;  // (100 / T)^1/2
    const G<R> ncoll = n * (YH + Y2);
    D<R, kDE | kDT> nel{R(0), R(0), R(0), R(0)};
    acc(nel, n, TF<R>{s100, R(-0.5) * s100 * iT}, YE);
    const R xo = R(nt.x_o * ck.fd);
    const R m13 = -R(nt.pm[12]);
    // kept rolled: five interleaved copies of this body cost ~130 VGPRs
#pragma unroll 1
    for (int j = 0; j < 5; ++j) {
      G<R> emit;
      if (j == 0) emit = dense(Y2);
      else if (j == 1) emit = G<R>{R(nt.x_c * ck.fd), R(0), R(0), R(0)};
      else if (j == 2) emit = G<R>{xo * (R(1) - YHP.v), R(0), -xo * YHP.e, -xo * YHP.t};
      else if (j == 3) emit = dense((xo * R(1.0 - nt.f_oiii)) * YHP);
      else emit = dense((xo * R(nt.f_oiii)) * YHP);
      const double tul = nt.l_tul[j];
      const R b = M::ea(-tul * iT64);
      const G<R> cul = R(nt.l_qn[j]) * ncoll + R(nt.l_qe[j]) * nel;
      G<R> clu{R(0), R(0), R(0), R(0)};
      acc(clu, R(nt.l_g[j]), TF<R>{b, b * R(tul * iT64 * iT64)}, cul);
      G<R> den = clu + cul;
      den.v = den.v + R(nt.l_a[j]);
      const G<R> frac = quot(clu, den);
      const G<R> e = emit * frac;
      const R w = m13 * R(nt.l_tul[j] * nt.l_a[j]);
      q.v = q.v + double(w) * double(e.v);
      q.a = q.a + w * e.a;
      q.e = q.e + w * e.e;
      q.t = q.t + w * e.t;
    }
  }

  out.f[0] = rh2.v;
  out.f[1] = re.v;
  out.f[2] = q.v;
  out.J[0][0] = rh2.a; out.J[0][1] = rh2.e; out.J[0][2] = rh2.t * clampT;
  out.J[1][0] = re.a;  out.J[1][1] = re.e;  out.J[1][2] = re.t * clampT;
  out.J[2][0] = q.a;   out.J[2][1] = q.e;   out.J[2][2] = q.t * clampT;
}

// k_H2/k_H3 alone (renormalisation and outputs)
template <class R>
__device__ inline double hm_ratio(const Net& nt, double Tin) {
  using M = Mth<R>;
  const double Tc = Tin < 1.0 ? 1.0 : (Tin > 1.0e8 ? 1.0e8 : Tin);
  TF<R> k2, k3;
  k2k3<R>(Tc, flog(Tc), 1.0 / Tc, k2, k3);
  const R a = R(nt.rm[2]) * k2.v, b = R(nt.rm[3]) * k3.v;
  return b > R(0) ? double(a * M::dv(R(1), b)) : 0.0;
}

// ------------------------------------------------------------------ dust
template <class R>
struct Dust {
  R G, gd, zeta, betad, absir, betair, Sd, Sir, Sg, emis, kir;
};

template <class R>
__device__ inline void kappa(const Net& nt, R T, R& k, R& dk) {
  using M = Mth<R>;
  const R x = T * R(nt.kap_tn);
  const R d = R(1) + x * x;
  const R id = M::dv(R(1), d);
  k = R(nt.kap_max) * x * x * id;
  dk = R(nt.kap_max) * R(2) * x * id * id * R(nt.kap_tn);
}

// Appendix C terms that depend on (T_d, E_IR) alone: grain emission and
// IR absorption with their logarithmic derivatives.  The chemistry solve
// of a subcycle leaves T_d and E_IR as they were, so a subcycle takes
// these once for its timescale and its dust solve.
template <class R>
struct DustRad {
  R betad, absir, betair, emis, kir;
};

template <class R>
__device__ inline void dust_rad(const Net& nt, const Par& pr, double Td_, double Eir_,
                                DustRad<R>& r) {
  using M = Mth<R>;
  const R Td = R(Td_);
  R kd, dkd;
  kappa<R>(nt, Td, kd, dkd);
  r.betad = R(4) * kd + dkd * Td;
  const R ctil = R(pr.c_red * CL);
  if (pr.ir_mode == 1) {
    const R E = R(Eir_);
    const R tir = M::sq(M::sq(R(pr.cr_a) * E));
    R ki, dki;
    kappa<R>(nt, tir, ki, dki);
    r.kir = ki;
    r.absir = ki * ctil * E;
    r.betair = ki + dki * tir * R(0.25);
  } else {
    // FIXED: T_IR = T_CMB, constants of the call
    r.kir = R(pr.kir_fix);
    r.absir = R(pr.absir_fix);
    r.betair = R(pr.betair_fix);
  }
  const R td2 = Td * Td;
  r.emis = kd * R(ARAD * CL) * td2 * td2;
}

// Appendix C sources and coefficients at (T_g, T_d, E_IR), the radiative
// terms of (T_d, E_IR) given
template <class R>
__device__ inline void dust_gas(const Net& nt, double Tg_, double Td_, const CellK& ck,
                                const DustRad<R>& r, Dust<R>& d) {
  using M = Mth<R>;
  const R Tg = R(Tg_), Td = R(Td_);
  const R iTg = M::dv(R(1), Tg);
  d.G = R(nt.pm[13] * RG * ck.n) * M::sq(Tg * R(1.0 / THIGH));
  d.gd = R(1) - R(0.8) * M::ea(-TLOW * frcp(Tg_));
  const R rr = Td * iTg - R(1);
  d.zeta = R(0.5) * d.gd * rr + (d.gd - R(1)) * R(TLOW) * iTg * rr - d.gd;
  d.betad = r.betad;
  d.kir = r.kir;
  d.absir = r.absir;
  d.betair = r.betair;
  d.emis = r.emis;
  const R coup = d.G * d.gd * (Td - Tg);
  d.Sd = d.absir + R(ck.euv) - d.emis - coup;
  d.Sir = R(ck.rho * ck.fd) * (d.emis - d.absir);
  d.Sg = R(ck.fd) * coup;
}

template <class R>
__device__ inline void dust_eval(const Net& nt, const Par& pr, double Tg_, double Td_,
                                 double Eir_, const CellK& ck, Dust<R>& d) {
  DustRad<R> r;
  dust_rad<R>(nt, pr, Td_, Eir_, r);
  dust_gas<R>(nt, Tg_, Td_, ck, r, d);
}

// ------------------------------------------------------------------ LU
// Gaussian elimination with partial pivoting (ties keep the lower row),
// rows exchanged by selects so that everything stays in registers.
__device__ inline void solve3(double a00, double a01, double a02, double a10, double a11,
                              double a12, double a20, double a21, double a22, double b0,
                              double b1, double b2, double& x0, double& x1, double& x2) {
  // pivot column 0
  int p = 0;
  double best = fabs(a00);
  if (fabs(a10) > best) { p = 1; best = fabs(a10); }
  if (fabs(a20) > best) { p = 2; }
  {
    const double r0[4] = {a00, a01, a02, b0};
    const double r1[4] = {a10, a11, a12, b1};
    const double r2[4] = {a20, a21, a22, b2};
    double n0[4], n1[4], n2[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      n0[j] = p == 0 ? r0[j] : (p == 1 ? r1[j] : r2[j]);
      n1[j] = p == 1 ? r0[j] : r1[j];
      n2[j] = p == 2 ? r0[j] : r2[j];
    }
    a00 = n0[0]; a01 = n0[1]; a02 = n0[2]; b0 = n0[3];
    a10 = n1[0]; a11 = n1[1]; a12 = n1[2]; b1 = n1[3];
    a20 = n2[0]; a21 = n2[1]; a22 = n2[2]; b2 = n2[3];
  }
  const double i00 = frcp(a00);
  {
    const double m1 = a10 * i00, m2 = a20 * i00;
    a11 = a11 - m1 * a01; a12 = a12 - m1 * a02; b1 = b1 - m1 * b0;
    a21 = a21 - m2 * a01; a22 = a22 - m2 * a02; b2 = b2 - m2 * b0;
  }
  if (fabs(a21) > fabs(a11)) {
    double t;
    t = a11; a11 = a21; a21 = t;
    t = a12; a12 = a22; a22 = t;
    t = b1; b1 = b2; b2 = t;
  }
  const double i11 = frcp(a11);
  {
    const double m = a21 * i11;
    a22 = a22 - m * a12;
    b2 = b2 - m * b1;
  }
  x2 = b2 * frcp(a22);
  x1 = (b1 - a12 * x2) * i11;
  x0 = (b0 - a01 * x1 - a02 * x2) * i00;
}

__device__ inline void solve2(double a00, double a01, double a10, double a11, double b0, double b1,
                              double& x0, double& x1) {
  if (fabs(a10) > fabs(a00)) {
    double t;
    t = a00; a00 = a10; a10 = t;
    t = a01; a01 = a11; a11 = t;
    t = b0; b0 = b1; b1 = t;
  }
  const double i00 = frcp(a00);
  const double m = a10 * i00;
  a11 = a11 - m * a01;
  b1 = b1 - m * b0;
  x1 = b1 * frcp(a11);
  x0 = (b0 - a01 * x1) * i00;
}

// ------------------------------------------------------------------ lane
struct Lane {
  double y2, ye, E, Td, Eir, rem, Tiso;
  CellK ck;
  int32_t nsub, nit;
  uint32_t fl;
};

constexpr uint32_t F_CAP = 1u, F_TIGHT = 2u, F_NOCONV = 4u, F_INVALID = 8u, F_FLOOR = 16u;

__device__ inline bool finite_bits(double x) {
  const unsigned long long b = __double_as_longlong(x);
  return ((b >> 52) & 0x7ffull) != 0x7ffull;
}

__device__ inline double ntot_rel(const Par& pr, double y2, double ye) {
  return 1.0 - y2 + ye + pr.y_he;
}

// E_th / (k_B n) per unit temperature: n_tot / (gamma - 1)
__device__ inline double cvk(const Par& pr, double y2, double ye) {
  return ntot_rel(pr, y2, ye) * pr.igm1;
}

// Conservation renormalisation (binary64): clamp the unknowns, rebuild
// y_H from H-nuclei conservation, rescale if it went negative, floor E_th.
template <class R>
__device__ inline void renormalise(const Net& nt, const Par& pr, Lane& L, bool iso) {
  if (L.y2 < 0.0) { L.y2 = 0.0; L.fl |= F_FLOOR; }
  if (L.y2 > 0.5) { L.y2 = 0.5; L.fl |= F_FLOOR; }
  if (L.ye < 0.0) { L.ye = 0.0; L.fl |= F_FLOOR; }
  if (L.ye > 1.0) { L.ye = 1.0; L.fl |= F_FLOOR; }
  const double knb = KB * L.ck.n;
  // y_H >= 1 - 2 y_H2 - y_e - 2 r_max y_e: the exact H- ratio is only
  // needed when this bound does not already exclude y_H < 0
  const double yh_lo = 1.0 - 2.0 * L.y2 - L.ye - 2.0 * pr.hm_ratio_max * L.ye;
  if (!(yh_lo >= 0.0)) {
    const double T = iso ? L.Tiso : L.E / (knb * cvk(pr, L.y2, L.ye));
    const double r = hm_ratio<double>(nt, T);
    const double yhm = r * L.ye;
    const double yhp = L.ye + yhm;
    const double yh = 1.0 - 2.0 * L.y2 - yhp - yhm;
    if (yh < 0.0) {
      const double s = 1.0 / (2.0 * L.y2 + yhp + yhm);
      L.y2 = L.y2 * s;
      L.ye = L.ye * s;
      L.fl |= F_FLOOR;
    }
  }
  const double cv = knb * cvk(pr, L.y2, L.ye);
  if (iso) {
    L.E = cv * L.Tiso;
  } else if (L.E < cv * pr.t_cmb) {
    L.E = cv * pr.t_cmb;
    L.fl |= F_FLOOR;
  }
}

// kappa in binary64 for the tight Newton
__device__ inline void kappa_d(const Net& nt, double T, double& k, double& dk) {
  const double x = T * nt.kap_tn;
  const double id = frcp(1.0 + x * x);
  k = nt.kap_max * x * x * id;
  dk = nt.kap_max * 2.0 * x * (id * id) * nt.kap_tn;
}

struct TightC {
  double td0, tg0, e0, h, ggd, dg, P, iqd, absfix, kir, euv, cd;  // iqd = 1 / q_d
};

__device__ inline void tight_phi(const Net& nt, const Par& pr, const TightC& t, double x,
                                 double& phi, double& dphi) {
  const double ac = ARAD * CL;
  const double ctil = pr.c_red * CL;
  double k, dk;
  kappa_d(nt, x, k, dk);
  const double x3 = x * x * x;
  const double emis = k * ac * x3 * x;
  const double demis = ac * x3 * (4.0 * k + dk * x);
  double ab, dab;
  if (pr.ir_mode == 1) {
    const double E = (t.e0 + t.P * emis) * t.iqd;
    ab = t.kir * ctil * E;
    dab = t.kir * ctil * t.P * demis * t.iqd;
  } else {
    ab = t.absfix;
    dab = 0.0;
  }
  phi = t.cd * (x - t.td0) - t.h * (ab + t.euv - emis - t.ggd * t.dg * (x - t.tg0));
  dphi = t.cd - t.h * (dab - demis - t.ggd * t.dg);
}

// Tight gas-dust coupling: backward Euler over h with G, gamma_d and
// kappa(T_IR) frozen; T_g and E_IR are explicit in T_d, leaving one
// increasing convex equation Phi(T_d) = 0.
template <class R>
__device__ inline void dust_tight(const Net& nt, const Par& pr, Lane& L, double h,
                                  const DustRad<double>& rad) {
  const double knb = KB * L.ck.n;
  const double cv = knb * cvk(pr, L.y2, L.ye);
  const double Tg0 = L.E * frcp(cv);
  Dust<double> d;
  dust_gas<double>(nt, Tg0, L.Td, L.ck, rad, d);
  TightC t;
  t.td0 = L.Td;
  t.tg0 = Tg0;
  t.e0 = L.Eir;
  t.h = h;
  t.cd = pr.cd;
  t.euv = L.ck.euv;
  const double alpha = cv * L.ck.irho;
  t.ggd = double(d.G) * double(d.gd);
  const double w = h * L.ck.fd * t.ggd;
  const double iaw = frcp(alpha + w);
  t.dg = alpha * iaw;
  t.P = h * L.ck.rho * L.ck.fd;
  t.kir = double(d.kir);
  t.iqd = frcp(1.0 + t.P * pr.c_red * CL * t.kir);
  t.absfix = double(d.absir);

  double lo = pr.t_cmb, hi, f, fp, x;
  int it = 0;
  bool conv = true;
  tight_phi(nt, pr, t, lo, f, fp);
  if (f >= 0.0) {
    x = lo;
    L.fl |= F_FLOOR;
  } else {
    hi = fmax(fmax(t.td0, t.tg0), lo);
    tight_phi(nt, pr, t, hi, f, fp);
    for (int guard = 0; f <= 0.0 && guard < 200; ++guard) {
      lo = hi;
      hi = hi * 2.0;
      tight_phi(nt, pr, t, hi, f, fp);
    }
    x = t.td0;
    if (!(x > lo && x <= hi)) x = hi;
    conv = false;
    for (it = 1; it <= pr.newton_max; ++it) {
      tight_phi(nt, pr, t, x, f, fp);
      if (f == 0.0) { conv = true; break; }
      double xn = x - f * frcp(fp);  // Phi' >= C_d > 0
      if (f < 0.0) {
        lo = x;
        if (!(xn < hi)) xn = hi;
      } else {
        hi = x;
        if (!(xn > lo)) xn = 0.5 * (lo + hi);
      }
      const double dx = xn - x;
      x = xn;
      if (fabs(dx) <= pr.newton_rtol * x) {
        tight_phi(nt, pr, t, x, f, fp);
        xn = x - f * frcp(fp);
        if (xn >= lo && xn <= hi) x = xn;
        conv = true;
        break;
      }
    }
    if (it > pr.newton_max) it = pr.newton_max;
  }
  if (!conv) L.fl |= F_NOCONV;
  L.nit += it;
  const double tg = (alpha * t.tg0 + w * x) * iaw;
  if (pr.ir_mode == 1) {
    double k, dk;
    kappa_d(nt, x, k, dk);
    L.Eir = (t.e0 + t.P * k * ARAD * CL * x * x * x * x) * t.iqd;
  }
  L.Td = x;
  L.E = L.E + cv * (tg - Tg0);
}

// One Appendix C linear solve over h, rows and columns scaled.
template <class R>
__device__ inline void dust_linear(const Net& nt, const Par& pr, Lane& L, double h,
                                   const DustRad<double>& rad) {
  const double knb = KB * L.ck.n;
  const double cv = knb * cvk(pr, L.y2, L.ye);
  const double Tg = L.E * frcp(cv);
  Dust<double> d;
  dust_gas<double>(nt, Tg, L.Td, L.ck, rad, d);
  const double ctil = pr.c_red * CL;
  const double ac = ARAD * CL;
  const double G = double(d.G), gd = double(d.gd), zeta = double(d.zeta);
  const double betad = double(d.betad), betair = double(d.betair);
  const double alpha = cv * L.ck.irho;
  const double td3 = L.Td * L.Td * L.Td;
  const double rho = L.ck.rho, fd = L.ck.fd, cd = pr.cd;
  const double A00 = cd + h * G * gd + h * ac * td3 * betad;
  const double A02 = h * G * zeta;
  const double A20 = -(h * fd * G * gd);
  const double A22 = alpha - h * fd * G * zeta;
  const double b0 = h * double(d.Sd);
  const double b2 = h * double(d.Sg);
  const double s0 = cd * L.Td, s2 = alpha * Tg;  // row scales
  if (pr.ir_mode == 1) {
    const double A01 = -(h * ctil * betair);
    const double A10 = -(rho * h * ac * td3 * fd * betad);
    const double A11 = 1.0 + rho * h * ctil * fd * betair;
    const double b1 = h * double(d.Sir);
    const double E = L.Eir;
    double x0, x1, x2;
    const double i0 = frcp(s0), i1 = frcp(E), i2 = frcp(s2);
    solve3(A00 * L.Td * i0, A01 * E * i0, A02 * Tg * i0,
           A10 * L.Td * i1, A11, 0.0,
           A20 * L.Td * i2, 0.0, A22 * Tg * i2,
           b0 * i0, b1 * i1, b2 * i2, x0, x1, x2);
    L.Td = L.Td + x0 * L.Td;
    L.Eir = L.Eir + x1 * E;
    L.E = L.E + cv * (x2 * Tg);
  } else {
    double x0, x1;
    const double i0 = frcp(s0), i2 = frcp(s2);
    solve2(A00 * L.Td * i0, A02 * Tg * i0, A20 * L.Td * i2, A22 * Tg * i2, b0 * i0, b2 * i2,
           x0, x1);
    L.Td = L.Td + x0 * L.Td;
    L.E = L.E + cv * (x1 * Tg);
  }
}

__device__ inline void dust_floors(const Par& pr, Lane& L) {
  if (L.Td < pr.t_cmb) { L.Td = pr.t_cmb; L.fl |= F_FLOOR; }
  const double cv = KB * L.ck.n * cvk(pr, L.y2, L.ye);
  if (L.E < cv * pr.t_cmb) { L.E = cv * pr.t_cmb; L.fl |= F_FLOOR; }
  if (pr.ir_mode == 1) {
    const double emin = pr.eir_min;
    if (L.Eir < emin) { L.Eir = emin; L.fl |= F_FLOOR; }
  }
}

// One subcycle; returns true when the cell has covered its interval.
template <class R, bool kS>
__device__ bool subcycle(const Net& nt, const Par& pr, Lane& L) {
  const bool iso = pr.thermal_mode == 1;
  const bool dust_on = (pr.dust_mode == 0) && !iso;
  const double knb = KB * L.ck.n;
  const double ntr = ntot_rel(pr, L.y2, L.ye);
  const double Ek = L.E * L.ck.ikn;             // E_th / (k_B n) [K]
  const double intr = frcp(ntr);
  const double T = iso ? L.Tiso : Ek * pr.gm1 * intr;

  Chem<R> ch;
  assemble<R, kS>(nt, pr, L.y2, L.ye, L.Td, T, L.ck, ch);
  const double f0 = double(ch.f[0]), f1 = double(ch.f[1]), fq = double(ch.f[2]);

  double nu_dust = 0.0, qgg = 0.0;
  DustRad<double> rad;
  if (dust_on) {
    dust_rad<double>(nt, pr, L.Td, L.Eir, rad);
    Dust<double> d;
    dust_gas<double>(nt, T, L.Td, L.ck, rad, d);
    // gas-grain exchange rho S_g / (k_B n) [K/s]
    qgg = double(d.Sg) * L.ck.rho_kn;
    const double alpha = knb * (ntr * pr.igm1) * L.ck.irho;
    // Near radiative equilibrium S_d and S_IR are differences of terms far
    // larger than themselves, known to a few ulps each: a net source within
    // kSrcNoise of its gross terms is rounding noise and sets no timescale
    // (|S| minus that level, floored at 0)
    const double absir = fabs(double(d.absir)), emis = fabs(double(d.emis));
    const double sd_noise =
        kSrcNoise * (absir + fabs(L.ck.euv) + emis + fabs(double(d.G) * double(d.gd) * (L.Td - T)));
    nu_dust = fmax(fabs(double(d.Sd)) - sd_noise, 0.0) * frcp(pr.cd * L.Td);
    nu_dust = fmax(nu_dust, fabs(double(d.Sg)) * frcp(alpha * T));
    if (pr.ir_mode == 1) {
      const double sir_noise = kSrcNoise * (L.ck.rho * L.ck.fd) * (emis + absir);
      nu_dust = fmax(nu_dust, fmax(fabs(double(d.Sir)) - sir_noise, 0.0) * frcp(L.Eir));
    }
  }
  const bool tight = dust_on && (L.rem * nu_dust * pr.inv_f_chem >= double(pr.n_cyc));
  if (tight) L.fl |= F_TIGHT;

  const double iEk = frcp(Ek);
  double nu = fmax(fabs(f0) * frcp(fmax(L.y2, pr.y_abs)), fabs(f1) * frcp(fmax(L.ye, pr.y_abs)));
  if (!iso) nu = fmax(nu, fabs(fq + qgg) * iEk);
  if (!tight) nu = fmax(nu, nu_dust);

  double h;
  bool last = false;
  // below 1e-300 the step is far beyond any interval: take the rest
  h = nu > 1e-300 ? pr.f_chem * frcp(nu) : L.rem;
  if (h >= L.rem) {
    h = L.rem;
    last = true;
  } else if (L.nsub >= pr.n_sub_max / 2) {
    const double hcap = L.rem / double(pr.n_sub_max - L.nsub);
    if (h < hcap) {
      h = hcap;
      L.fl |= F_CAP;
      if (h >= L.rem) { h = L.rem; last = true; }
    }
  }

  // chemistry + energy: (I - h J) du = h f, u = (y_H2, y_e, E/E_ref)
  {
    const double Tn = T * intr;
    const double dTy2 = iso ? 0.0 : Tn;
    const double dTye = iso ? 0.0 : -Tn;
    const double dTu = iso ? 0.0 : T;
    double J00 = double(ch.J[0][0]) + double(ch.J[0][2]) * dTy2;
    double J01 = double(ch.J[0][1]) + double(ch.J[0][2]) * dTye;
    double J02 = double(ch.J[0][2]) * dTu;
    double J10 = double(ch.J[1][0]) + double(ch.J[1][2]) * dTy2;
    double J11 = double(ch.J[1][1]) + double(ch.J[1][2]) * dTye;
    double J12 = double(ch.J[1][2]) * dTu;
    double J20 = 0.0, J21 = 0.0, J22 = 0.0, g2 = 0.0;
    if (!iso) {
      g2 = fq * iEk;
      J20 = (double(ch.J[2][0]) + double(ch.J[2][2]) * dTy2) * iEk;
      J21 = (double(ch.J[2][1]) + double(ch.J[2][2]) * dTye) * iEk;
      J22 = double(ch.J[2][2]) * dTu * iEk;
    }
    double x0, x1, x2;
    solve3(1.0 - h * J00, -(h * J01), -(h * J02), -(h * J10), 1.0 - h * J11, -(h * J12),
           -(h * J20), -(h * J21), 1.0 - h * J22, h * f0, h * f1, h * g2, x0, x1, x2);
    const double Eref = L.E;
    L.y2 = L.y2 + x0;
    L.ye = L.ye + x1;
    if (!iso) L.E = L.E + x2 * Eref;
  }
  renormalise<R>(nt, pr, L, iso);

  if (dust_on) {
    if (!tight) dust_linear<R>(nt, pr, L, h, rad);
    else dust_tight<R>(nt, pr, L, h, rad);
    dust_floors(pr, L);
  }
  L.nsub += 1;
  if (!last) L.rem = L.rem - h;
  return last;
}

// ------------------------------------------------------------------ NR
// Fully implicit Newton-Raphson comparator (Sec. 2, the iterative scheme
// the LI method replaces; binary64 only).  Backward Euler over a substep
// dts for (y_H2, y_e, T_g, T_d, E_IR), solved as three nested groups: the
// outer Newton iteration on T_g (derivative of the energy residual by a
// central difference, step 1e-4 T_g), and at each trial T_g the dust/IR
// group and then the chemistry group.  Tolerance 1e-5 relative, relaxed to
// 1e-3 after half of the 20 allowed outer iterations; every loop gives up
// after 20 iterations, and a failed substep is halved (Eq. substep_NRchem).
// Energies are carried per k_B n_H [K], as in the LI kernel.
struct NRState {
  double y2, ye, T, Td, Eir;
};

// group (ii): (T_d, E_IR) at fixed T_g
__device__ inline bool nr_dust(const Net& nt, const Par& pr, const CellK& ck, double Td0,
                               double Eir0, double dts, double T, double tol, double& Td,
                               double& Eir, int32_t& its) {
  const double ctil = pr.c_red * CL;
  const double ac = ARAD * CL;
  for (int it = 1; it <= 20; ++it) {
    ++its;
    Dust<double> d;
    dust_eval<double>(nt, pr, T, Td, Eir, ck, d);
    const double td3 = Td * Td * Td;
    const double F1 = pr.cd * (Td - Td0) - dts * d.Sd;
    const double J11 = pr.cd + dts * (ac * td3 * d.betad + d.G * d.gd);
    double dTd, dE = 0.0;
    if (pr.ir_mode == 1) {
      const double F2 = Eir - Eir0 - dts * d.Sir;
      const double J12 = -(dts * ctil * d.betair);
      const double J21 = -(dts * ck.rho * ck.fd * ac * td3 * d.betad);
      const double J22 = 1.0 + dts * ck.rho * ck.fd * ctil * d.betair;
      const double det = J11 * J22 - J12 * J21;
      dTd = -(F1 * J22 - J12 * F2) / det;
      dE = -(J11 * F2 - J21 * F1) / det;
    } else {
      dTd = -F1 / J11;
    }
    double Tn = Td + dTd;
    bool ok = fabs(dTd) <= tol * fabs(Tn);
    if (Tn < 0.5 * Td) { Tn = 0.5 * Td; ok = false; }
    if (Tn > 2.0 * Td) { Tn = 2.0 * Td; ok = false; }
    double En = Eir;
    if (pr.ir_mode == 1) {
      En = Eir + dE;
      ok = ok && fabs(dE) <= tol * fabs(En);
      if (En < 0.5 * Eir) { En = 0.5 * Eir; ok = false; }
      if (En > 2.0 * Eir) { En = 2.0 * Eir; ok = false; }
    }
    Td = Tn;
    Eir = En;
    if (ok) return true;
  }
  return false;
}

// group (iii): (y_H2, y_e) at fixed T_g, T_d; steps that would leave the
// bounds are damped towards them
template <bool kS>
__device__ inline bool nr_chem(const Net& nt, const Par& pr, const CellK& ck, double y20,
                               double ye0, double dts, double T, double Td, double tol,
                               double& y2, double& ye, int32_t& its) {
  for (int it = 1; it <= 20; ++it) {
    ++its;
    Chem<double> ch;
    assemble<double, kS>(nt, pr, y2, ye, Td, T, ck, ch);
    const double F1 = y2 - y20 - dts * ch.f[0];
    const double F2 = ye - ye0 - dts * ch.f[1];
    const double J11 = 1.0 - dts * ch.J[0][0], J12 = -(dts * ch.J[0][1]);
    const double J21 = -(dts * ch.J[1][0]), J22 = 1.0 - dts * ch.J[1][1];
    const double det = J11 * J22 - J12 * J21;
    const double d1 = -(F1 * J22 - J12 * F2) / det;
    const double d2 = -(J11 * F2 - J21 * F1) / det;
    double n1 = y2 + d1, n2 = ye + d2;
    bool ok = fabs(d1) <= tol * fmax(fabs(n1), pr.y_abs) &&
              fabs(d2) <= tol * fmax(fabs(n2), pr.y_abs);
    if (n1 < 0.0) { n1 = 0.1 * y2; ok = false; }
    if (n1 > 0.5) { n1 = 0.5 * (y2 + 0.5); ok = false; }
    if (n2 < 0.0) { n2 = 0.1 * ye; ok = false; }
    if (n2 > 1.0) { n2 = 0.5 * (ye + 1.0); ok = false; }
    y2 = n1;
    ye = n2;
    if (ok) return true;
  }
  return false;
}

// inner groups at trial T; G = residual of the gas energy equation / (k_B n).
// Kept out of line: the four inlined copies of this solve (at T - dl, T,
// T + dl and the accepted T) compiled at -O3 into code whose iteration
// counts and, for a few cells, results depended on which other cells shared
// the wavefront (a single cell per wavefront matched the CPU reference);
// called, compiled at -O1, or without the stand-in branches of the source
// assembly, the same source matches the reference cell for cell.
template <bool kS>
__device__ __attribute__((noinline)) bool nr_inner(const Net& nt, const Par& pr, const CellK& ck, const Lane& s0,
                                double dts, double T, double tol, bool dust_on, NRState& g,
                                double& G, int32_t& its) {
  if (dust_on && !nr_dust(nt, pr, ck, s0.Td, s0.Eir, dts, T, tol, g.Td, g.Eir, its)) return false;
  if (!nr_chem<kS>(nt, pr, ck, s0.y2, s0.ye, dts, T, g.Td, tol, g.y2, g.ye, its)) return false;
  Chem<double> ch;
  assemble<double, kS>(nt, pr, g.y2, g.ye, g.Td, T, ck, ch);
  const double knb = KB * ck.n;
  double gas_grain = 0.0;
  if (dust_on) {
    Dust<double> d;
    dust_eval<double>(nt, pr, T, g.Td, g.Eir, ck, d);
    gas_grain = d.Sg * (ck.rho / knb);
  }
  G = cvk(pr, g.y2, g.ye) * T - s0.E / knb - dts * (ch.f[2] + gas_grain);
  return true;
}

// One backward-Euler substep of length dts from L; on success L holds the
// new state.  Outer iterations are counted in L.nit, inner ones in its.
template <bool kS>
__device__ bool nr_substep_iter(const Net& nt, const Par& pr, Lane& L, double dts,
                                int32_t& its) {
  const bool iso = pr.thermal_mode == 1;
  const bool dust_on = (pr.dust_mode == 0) && !iso;
  const double knb = KB * L.ck.n;
  const Lane s0 = L;
  NRState g{L.y2, L.ye, iso ? L.Tiso : L.E / (knb * cvk(pr, L.y2, L.ye)), L.Td, L.Eir};
  if (iso) {
    double Gv;
    if (!nr_inner<kS>(nt, pr, L.ck, s0, dts, L.Tiso, 1e-5, dust_on, g, Gv, its)) return false;
    L.y2 = g.y2;
    L.ye = g.ye;
    L.Td = g.Td;
    L.Eir = g.Eir;
    L.E = knb * cvk(pr, L.y2, L.ye) * L.Tiso;
    L.nit += 1;
    return true;
  }
  double tol = 1e-5;
  for (int it = 1; it <= 20; ++it) {
    L.nit += 1;
    if (it > 10) tol = 1e-3;
    const double T = g.T;
    const double dl = 1e-4 * T;
    NRState gm = g, gc = g, gp = g;
    double Gm, Gc, Gp;
    if (!nr_inner<kS>(nt, pr, L.ck, s0, dts, T - dl, tol, dust_on, gm, Gm, its)) return false;
    if (!nr_inner<kS>(nt, pr, L.ck, s0, dts, T, tol, dust_on, gc, Gc, its)) return false;
    if (!nr_inner<kS>(nt, pr, L.ck, s0, dts, T + dl, tol, dust_on, gp, Gp, its)) return false;
    const double dG = (Gp - Gm) / (2.0 * dl);
    double Tn = T - Gc / dG;
    bool limited = false;
    if (!(Tn > 0.5 * T)) { Tn = 0.5 * T; limited = true; }
    if (!(Tn < 2.0 * T)) { Tn = 2.0 * T; limited = true; }
    if (Tn < pr.t_cmb) { Tn = pr.t_cmb; limited = true; }
    const bool ok = !limited && fabs(Tn - T) <= tol * Tn &&
                    fabs(gc.y2 - g.y2) <= tol * fmax(gc.y2, pr.y_abs) &&
                    fabs(gc.ye - g.ye) <= tol * fmax(gc.ye, pr.y_abs) &&
                    fabs(gc.Td - g.Td) <= tol * gc.Td;
    g = gc;
    g.T = Tn;
    if (ok) {
      double Gv;
      if (!nr_inner<kS>(nt, pr, L.ck, s0, dts, Tn, tol, dust_on, g, Gv, its)) return false;
      L.y2 = g.y2;
      L.ye = g.ye;
      L.Td = g.Td;
      L.Eir = g.Eir;
      L.E = knb * cvk(pr, L.y2, L.ye) * Tn;
      return true;
    }
  }
  return false;
}

// One substep; L.nit counts every Newton iteration of it: outer iterations
// and the inner dust/IR and chemistry iterations (so two runs take the same
// iteration path only if every convergence test came out the same).
template <bool kS>
__device__ bool nr_substep(const Net& nt, const Par& pr, Lane& L, double dts) {
  int32_t its = 0;
  const bool ok = nr_substep_iter<kS>(nt, pr, L, dts, its);
  L.nit += its;
  return ok;
}

constexpr uint32_t F_NRFAIL = 32u;

// One substep attempt of the NR driver (Eq. substep_NRchem): the first
// try covers the whole interval; dts = (dt - t_sub) / 2^lev, lev + 1 on
// failure, max(lev - 1, 0) on success.  L.rem holds dt, tsub and lev the
// driver state.  At most n_sub_max attempts (then NRFAIL), so every cell
// ends.  Returns true when the cell is done.
template <bool kS>
__device__ bool nr_attempt(const Net& nt, const Par& pr, Lane& L, double& tsub, int& lev,
                           int& attempts) {
  const double dts = (L.rem - tsub) / ldexp(1.0, lev);
  Lane trial = L;
  const bool ok = nr_substep<kS>(nt, pr, trial, dts);
  L.nit = trial.nit;
  ++attempts;
  if (ok) {
    const int32_t nit = L.nit;
    L = trial;
    L.nit = nit;
    L.nsub += 1;
    if (lev == 0) return true;
    tsub = tsub + dts;
    lev = lev > 0 ? lev - 1 : 0;
  } else {
    ++lev;
    if (lev > 60) { L.fl |= F_NRFAIL; return true; }
  }
  if (attempts >= pr.n_sub_max) { L.fl |= F_NRFAIL; return true; }
  return false;
}

// ------------------------------------------------------------------ I/O
// Per-cell constants of a call, from the inputs only: the same arithmetic
// at the first load and at a resume, so a resumed cell goes on bit for bit.
__device__ inline void cell_consts(const Net& nt, const Par& pr, double nh, double ne, double nf,
                                   double z, CellK& k) {
  k.n = nh;
  k.fd = z;
  k.rho = (1.0 + 4.0 * pr.y_he) * MH * nh;
  const double g0 = nf * nt.inv_g0;
  k.k9 = nt.rm[9] * (nt.c_sigma * ne);
  k.k10 = nt.rm[10] * (nt.k10g * g0);
  k.k11 = nt.rm[11] * nt.zeta;
  k.g4 = nt.pe_mode == 1 ? g0 : nt.pm[3] * nt.pe_k * g0 * z;  // Gamma_4 / (k_B n), or G0
  k.euv = nt.kap_uv_c * (nf * nt.e_fuv + ne * nt.e_euv);
  const double knb = KB * nh;
  k.ikn = frcp(knb);
  k.irho = frcp(k.rho);
  k.rho_kn = k.rho / knb;
}

// Two-phase dispatch: write a running cell's state back in place (its
// y_H2, y_e, E_th, T_d [, E_IR] slots) and the rest of the lane into slot p.
__device__ inline void suspend_cell(const Par& pr, const Cells& c, const Suspended& s, int64_t i,
                                    unsigned long long p, const Lane& L) {
  c.y_h2[i] = L.y2;
  c.y_e[i] = L.ye;
  c.eint[i] = L.E;
  c.tdust[i] = L.Td;
  if (pr.ir_mode == 1) c.eir[i] = L.Eir;
  s.cell[p] = int32_t(i);
  s.rem[p] = L.rem;
  s.tiso[p] = L.Tiso;
  s.nsub[p] = L.nsub;
  s.nit[p] = L.nit;
  s.fl[p] = L.fl;
}

// ... and take it up again: no validation and no renormalisation, the lane
// is restored exactly as it was suspended.
__device__ inline int64_t resume_cell(const Net& nt, const Par& pr, const Cells& c,
                                      const Suspended& s, int32_t p, Lane& L) {
  const int64_t i = s.cell[p];
  L.y2 = c.y_h2[i];
  L.ye = c.y_e[i];
  L.E = c.eint[i];
  L.Td = c.tdust[i];
  L.Eir = pr.ir_mode == 1 ? c.eir[i] : pr.eir_min;
  cell_consts(nt, pr, c.nh[i], c.n_euv[i], c.n_fuv[i], c.zmet ? c.zmet[i] : pr.z_default, L.ck);
  L.rem = s.rem[p];
  L.Tiso = s.tiso[p];
  L.nsub = s.nsub[p];
  L.nit = s.nit[p];
  L.fl = s.fl[p];
  return i;
}

// Load a cell; returns false (and writes the invalid marker) on bad input.
template <class R>
__device__ bool load_cell(const Net& nt, const Par& pr, const Cells& c, int64_t i, double dt,
                          Lane& L) {
  const double nh = c.nh[i], ne = c.n_euv[i], nf = c.n_fuv[i];
  const double z = c.zmet ? c.zmet[i] : pr.z_default;
  L.y2 = c.y_h2[i];
  L.ye = c.y_e[i];
  L.E = c.eint[i];
  L.Td = c.tdust[i];
  L.Eir = pr.ir_mode == 1 ? c.eir[i] : pr.eir_min;
  bool ok = finite_bits(nh) && nh > 0.0 && finite_bits(ne) && ne >= 0.0 && finite_bits(nf) &&
            nf >= 0.0 && finite_bits(z) && z >= 0.0 && finite_bits(L.y2) && L.y2 >= 0.0 &&
            finite_bits(L.ye) && L.ye >= 0.0 && finite_bits(L.E) && L.E > 0.0 &&
            finite_bits(L.Td) && L.Td > 0.0;
  if (pr.ir_mode == 1) ok = ok && finite_bits(L.Eir) && L.Eir > 0.0;
  if (!ok) {
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    if (c.y_h) c.y_h[i] = nan;
    if (c.y_hp) c.y_hp[i] = nan;
    if (c.y_hm) c.y_hm[i] = nan;
    if (c.tgas) c.tgas[i] = nan;
    if (c.nsub) c.nsub[i] = 0;
    if (c.niter) c.niter[i] = 0;
    if (c.flags) c.flags[i] = F_INVALID;
    if (c.n_euv_out) c.n_euv_out[i] = ne;  // an invalid cell absorbs nothing
    if (c.n_fuv_out) c.n_fuv_out[i] = nf;
    return false;
  }
  cell_consts(nt, pr, nh, ne, nf, z, L.ck);
  L.Tiso = L.E / (KB * nh * cvk(pr, L.y2, L.ye));
  L.rem = dt;
  L.nsub = 0;
  L.nit = 0;
  L.fl = 0;
  renormalise<R>(nt, pr, L, pr.thermal_mode == 1);
  return true;
}

template <class R>
__device__ void store_cell(const Net& nt, const Par& pr, const Cells& c, int64_t i,
                           const Lane& L, double dt = 0.0) {
  c.y_h2[i] = L.y2;
  c.y_e[i] = L.ye;
  c.eint[i] = L.E;
  c.tdust[i] = L.Td;
  if (pr.ir_mode == 1) c.eir[i] = L.Eir;
  const bool iso = pr.thermal_mode == 1;
  const double T = iso ? L.Tiso : L.E / (KB * L.ck.n * cvk(pr, L.y2, L.ye));
  const bool absorb = pr.photon_absorb == 1 && (c.n_euv_out || c.n_fuv_out);
  if (c.y_h || c.y_hp || c.y_hm || absorb) {
    const double r = hm_ratio<double>(nt, T);
    const double yhm = r * L.ye;
    const double yhp = L.ye + yhm;
    const double yh = 1.0 - 2.0 * L.y2 - yhp - yhm;
    if (c.y_h) c.y_h[i] = yh;
    if (c.y_hp) c.y_hp[i] = yhp;
    if (c.y_hm) c.y_hm[i] = yhm;
    if (absorb) {
      // photons absorbed over the step by the updated gas (Sec. 2
      // "Radiation components"; stand-in): N exp(-c~ alpha dt) with
      // c alpha_EUV = c sigma n_H y_H + c kappa_UV rho f_d, c alpha_FUV = c kappa_UV rho f_d
      const double ad = nt.kap_uv_c * L.ck.rho * L.ck.fd;
      const double ae = nt.c_sigma * L.ck.n * fmax(yh, 0.0) + ad;
      if (c.n_euv_out) c.n_euv_out[i] = c.n_euv[i] * fexp(-(pr.c_red * ae * dt));
      if (c.n_fuv_out) c.n_fuv_out[i] = c.n_fuv[i] * fexp(-(pr.c_red * ad * dt));
    }
  }
  if (c.tgas) c.tgas[i] = T;
  if (c.nsub) c.nsub[i] = L.nsub;
  if (c.niter) c.niter[i] = L.nit;
  if (c.flags) c.flags[i] = L.fl;
}

__device__ inline unsigned lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi(unsigned(mask >> 32), __builtin_amdgcn_mbcnt_lo(unsigned(mask), 0u));
}

// The network and parameters are re-read from the context's device copy
// (constant address space, scalar loads) at every subcycle.  Holding the
// ~100 uniform binary64 values they feed across the whole cell loop costs
// SGPR spills and VGPR copies; the opaque pointer keeps the loads (and the
// arithmetic on them) inside the loop.
typedef const __attribute__((address_space(4))) Net CNet;
typedef const __attribute__((address_space(4))) Par CPar;
__device__ inline const Net& fresh(const Net* p) {
  CNet* q = (CNet*)p;
  asm volatile("" : "+s"(q));
  return *(const Net*)q;
}
__device__ inline const Par& fresh(const Par* p) {
  CPar* q = (CPar*)p;
  asm volatile("" : "+s"(q));
  return *(const Par*)q;
}

// The kernel's own argument block, re-read (scalar loads) wherever it is
// used inside the cell loop instead of being held in SGPRs across it: the
// ~40 pointers and scalars it holds would otherwise spill to VGPR lanes.
template <class A>
__device__ inline const A& kargs() {
  typedef const __attribute__((address_space(4))) A CA;
  CA* p = (CA*)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *(const A*)p;
}

}  // namespace
}  // namespace sfk
