// sfk.h -- internal interface between the host library (sfchem.cpp) and the
// gfx950 kernels (sfk_li.hip).  Everything here is passed by value as the
// kernel argument block, so wave-uniform constants are read through the
// scalar cache into SGPRs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfk {

// Network constants in the units the kernels use.  Heating and cooling are
// evaluated as Q / (k_B n_H) [K/s], so energy coefficients are pre-divided
// by k_B on the host.
struct Net {
  double rm[12];        // reaction multipliers
  double pm[14];        // thermal process multipliers
  double c_sigma;       // c * sigma_EUV [cm^3/s]
  double k10g;          // k10 per G0 [1/s]
  double inv_g0;        // 1 / (G0 photon density)
  double zeta;          // cosmic-ray rate [1/s]
  double k4_pre, k4_theta;
  double g2k;           // heat per photoionisation / k_B [K]
  double g3k;           // heat per photodissociation / k_B [K]
  double pe_k;          // pe_coef * pe_eps / k_B [K cm^3/s]
  double kap_max, kap_tn;
  double kap_uv_c;      // c * kappa_UV [cm^3/g/s]
  double e_fuv, e_euv;  // photon energies [erg]
  double x_c, x_o, f_oiii;
  double l_tul[5], l_a[5], l_g[5], l_qn[5], l_qe[5];
};

struct Par {
  double f_chem, y_abs, newton_rtol, c_red, t_cmb, y_he, gm1;  // gm1 = gamma - 1
  double cd;             // C_d [erg/g/K]
  double z_default;
  double hm_ratio_max;   // upper bound of y_H-/y_e = k_H2/k_H3 over the rate range
  int32_t n_cyc, n_sub_max, newton_max, ir_mode, thermal_mode, dust_mode;
};

struct Cells {
  int64_t n;
  double *y_h2, *y_e, *eint, *tdust, *eir;
  double *y_h, *y_hp, *y_hm, *tgas;
  const double *nh, *n_euv, *n_fuv, *zmet;
  int32_t *nsub, *niter;
  uint32_t *flags;
};

struct Args {
  Net net;
  Par par;
  Cells c;
  double dt;
  unsigned long long* counter;  // work counter, zero at launch
  int32_t refill_min;           // refill a wave once this many lanes are idle
};

// Served form: one work item = a contiguous range of cells of one slot.
struct Slot {
  Cells c;          // arena-resident state of the request
  double dt;
  int32_t precision;
  int32_t pad;
};
struct ServedArgs {
  Net net;
  Par par;
  const Slot* slots;          // device copy of the slot table
  const int32_t* item_slot;   // work item -> slot index
  const int64_t* item_begin;  // work item -> first cell
  const int32_t* item_count;  // work item -> number of cells
  int64_t n_items;
  unsigned long long* counter;      // work counter (items)
  int32_t* slot_remaining;          // per slot: items left
  int32_t refill_min;
};

// host-callable launchers (defined in sfk_li.hip)
hipError_t launch_step(const Args& a, int precision, int grid, hipStream_t s);
hipError_t launch_reset(unsigned long long* counter, hipStream_t s);
int max_blocks_per_cu(int precision);
hipError_t launch_served(const ServedArgs& a, int precision, int grid, hipStream_t s);

constexpr int kBlock = 256;

}  // namespace sfk
