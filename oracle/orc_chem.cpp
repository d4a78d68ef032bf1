/*
 * orc_chem.cpp -- CPU reference ("oracle") for the per-cell thermochemistry
 * of SFUMATO# (arXiv 2604.21438): the linearized-implicit (LI) update, the
 * Newton-Raphson (NR) fully implicit comparator and an RK4 reference.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code with
 * the HIP implementation.
 *
 * Sources in the paper (section / equation / table labels of the paper):
 *   network            Appendix A, Table "Chemical reactions" (H0..H11)
 *   heating / cooling  Appendix B, Table "Thermal processes" (1..14)
 *   LI system          Sec. 2 "Thermochemical processes", Eqs. eq_chem2,
 *                      eq_chem3, eq_y, eq_deq; only y_H2 and y_e are
 *                      unknowns, y_H and y_H+ follow from conservation.
 *   gas energy         solved together with the chemistry (same section:
 *                      the "thermochemical solver").
 *   dust / IR / gas    Appendix C, Eqs. ap_eq:dust_temp, ap_eq:Eir,
 *                      ap_eq:Tg, the three difference equations and
 *                      alpha_g, beta_d, beta_IR, gamma_d, zeta.
 *   step size          Sec. 2 "Time stepping", Eqs. timescale_of_dust,
 *                      timescale_chemi, timescale_energy, timestep_subcycle,
 *                      N_cyc = 300, f_chem = 0.03.
 *   NR comparator      same section, three iteration groups, tolerance
 *                      1e-5 relaxed to 1e-3 after N_itr,limit/2, N_itr,limit
 *                      = 20, substeps of Eq. substep_NRchem.
 *
 * Readings where the paper is silent, garbled or points to other papers are
 * listed where they are used ("Reading:").
 * Stand-ins for formulas the paper does not print are labelled "STAND-IN".
 *
 * Pins (tests/test_oracle_*.py): rate values printed by the paper (H II
 * equilibrium y_H ~ 2e-5, alpha_B, H2 formation time), closed-form
 * transients and equilibria, conservation to round-off, the Appendix C
 * energy identity, derivative checks against central differences,
 * first-order convergence to RK4, LI/NR agreement at equilibrium.  The
 * tight gas-dust step (dust_tight_step) has its own: first-order
 * convergence to RK4 with every subcycle tight, energy conservation of a
 * single tight step, quick Newton convergence in strongly coupled cells,
 * and radiative equilibrium in the infinite-step limit; a mutation test
 * builds copies of this file with planted mistakes in that step and
 * checks that each one fails at least one of those pins.
 * Parity unpinned: the full-network trajectories with the stand-in physics
 * (nothing outside the oracle fixes them).
 */
#include "orc.h"
#include "orc_real.h"

#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#ifdef ORC_COUNT
thread_local OrcCounts orc_counts;
#endif

namespace {

/* physical constants, cgs */
const double K_B = 1.380649e-16;       /* erg/K                     */
const double M_H = 1.67262192e-24;     /* g, mass of the H nucleus  */
const double EV = 1.602176634e-12;     /* erg                       */
const double C_LIGHT = 2.99792458e10;  /* cm/s                      */
const double A_RAD = 7.5657e-15;       /* erg cm^-3 K^-4            */
const double G_GRAV = 6.6743e-8;       /* cm^3 g^-1 s^-2            */
const double LN10 = 2.302585092994045684;

/* Appendix C constants: R_g, T_high, T_low */
const double R_G = 5.83e-8;
const double T_HIGH = 1000.0;
const double T_LOW = 75.0;

/* range over which the rate fits are evaluated (Reading: T clamped) */
const double T_RATE_MIN = 1.0;
const double T_RATE_MAX = 1.0e8;

/* ------------------------------------------------------------------ */
/* value with partial derivatives w.r.t. (y_H2, y_e, T)                */
struct G3 {
  real v, a, e, t;
};
static inline G3 cst(real v) { return G3{v, 0.0, 0.0, 0.0}; }
static inline G3 tfun(real v, real dvdT) { return G3{v, 0.0, 0.0, dvdT}; }
static inline G3 operator+(G3 x, G3 y) { return G3{x.v + y.v, x.a + y.a, x.e + y.e, x.t + y.t}; }
static inline G3 operator-(G3 x, G3 y) { return G3{x.v - y.v, x.a - y.a, x.e - y.e, x.t - y.t}; }
static inline G3 operator*(G3 x, G3 y) {
  return G3{x.v * y.v, x.a * y.v + x.v * y.a, x.e * y.v + x.v * y.e, x.t * y.v + x.v * y.t};
}
static inline G3 operator*(real s, G3 x) { return G3{s * x.v, s * x.a, s * x.e, s * x.t}; }
static inline G3 operator*(G3 x, real s) { return G3{x.v * s, x.a * s, x.e * s, x.t * s}; }
static inline G3 operator/(G3 x, G3 y) {
  real q = x.v / y.v;
  return G3{q, (x.a - q * y.a) / y.v, (x.e - q * y.e) / y.v, (x.t - q * y.t) / y.v};
}

/* per-cell quantities that stay fixed during one call */
struct Cell {
  real n, fd, rho;
  real n_euv, n_fuv;
  real k9, k10, k11;   /* photo / CR rates [1/s]                     */
  real g0;             /* FUV field in Habing units                  */
  real e_uv;           /* dust UV absorption [erg/g/s], per gram gas */
};

struct Rates {
  real k[ORC_NREAC];
  real dk[ORC_NREAC];
  real lnT;
};

/* k_H2 (H + e -> H- + photon) and k_H3 (H- + H -> H2 + e) with d/dT */
static void k2k3(real T, real lnT, real& k2, real& dk2, real& k3, real& dk3) {
  (void)lnT;
  k2 = 1.4e-18 * rpow(T, 0.928) * rexp(-T / 16200.0);
  dk2 = k2 * (0.928 / T - 1.0 / 16200.0);
  real p1 = rpow(T, 0.098493), p2 = rpow(T, 0.5561), p3 = rpow(T, 2.1826);
  real q1 = rpow(T, 1.0461), q2 = rpow(T, 3.0424), q3 = rpow(T, 3.7741);
  real N = p1 + 0.32852 * p2 + 2.771e-7 * p3;
  real D = 1.0 + 6.191e-3 * q1 + 8.9712e-11 * q2 + 3.2576e-14 * q3;
  real dN = (0.098493 * p1 + 0.32852 * 0.5561 * p2 + 2.771e-7 * 2.1826 * p3) / T;
  real dD = (6.191e-3 * 1.0461 * q1 + 8.9712e-11 * 3.0424 * q2 + 3.2576e-14 * 3.7741 * q3) / T;
  k3 = 1.35e-9 * N / D;
  dk3 = k3 * (dN / N - dD / D);
}

/* ------------------------------------------------------------------ */
/* Rate coefficients, Table "Chemical reactions".  T in K.             */
static void rates(const orc_network& net, real T, real Td, const Cell& c, Rates& r) {
  const real lnT = rlog(T);
  r.lnT = lnT;

  /* H0: collisional ionisation, fit in ln(T / eV) */
  {
    const double cf[9] = {-32.71396786, 13.536556, -5.73932875, 1.563154998, -0.2877056,
                          3.48255977e-2, -2.63197617e-3, 1.11954395e-4, -2.03914985e-6};
    real x = lnT + std::log(K_B / EV);
    real P = cf[8], dP = 8.0 * cf[8];
    for (int i = 7; i >= 0; --i) P = P * x + cf[i];
    for (int i = 7; i >= 1; --i) dP = dP * x + real(i) * cf[i];
    r.k[0] = rexp(P);
    r.dk[0] = r.k[0] * dP / T;
  }
  /* H1: radiative recombination */
  {
    real w = rpow(115188.0 / T, 0.407);
    r.k[1] = 2.753e-14 * rpow(315614.0 / T, 1.5) * rpow(1.0 + w, -2.242);
    r.dk[1] = r.k[1] / T * (-1.5 + 2.242 * 0.407 * w / (1.0 + w));
  }
  /* H2: H + e -> H- + photon;  H3: H- + H -> H2 + e */
  k2k3(T, lnT, r.k[2], r.dk[2], r.k[3], r.dk[3]);
  /* H4: H2 + H -> 3H.  STAND-IN (the paper defers to its reference):
   * Arrhenius form with the H2 binding energy as threshold. */
  {
    r.k[4] = net.k4_pre * rexp(-net.k4_theta / T);
    r.dk[4] = r.k[4] * net.k4_theta / (T * T);
  }
  /* H5: 3H -> H2 + H (Reading: the garbled reactant list is 3H) */
  real k5 = 6.0e-32 * rpow(T, -0.25) + 2.0e-31 * rpow(T, -0.5);
  real dk5 = (-0.25 * 6.0e-32 * rpow(T, -0.25) - 0.5 * 2.0e-31 * rpow(T, -0.5)) / T;
  r.k[5] = k5;
  r.dk[5] = dk5;
  /* H6: 2H + H2 -> 2H2, k_H6 = k_H5 / 8 */
  r.k[6] = k5 / 8.0;
  r.dk[6] = dk5 / 8.0;
  /* H7: 2H2 -> 2H + H2, k = k_high^(1-a) k_low^a, evaluated in ln space.
   * Reading: the density in a is n_H. */
  {
    real lnkl = std::log(1.18e-10) - 6.95e4 / T;
    real dlnkl = 6.95e4 / (T * T);
    real eb = rexp(-6000.0 / T);
    real lnkh = std::log(8.125e-8) - 0.5 * lnT - 5.2e4 / T + rlog1p(-eb);
    real dlnkh = -0.5 / T + 5.2e4 / (T * T) - eb * (6000.0 / (T * T)) / (1.0 - eb);
    real t = lnT / LN10 - 4.0; /* log10(T / 1e4) */
    real lg = 4.845 - 1.3 * t + 1.62 * t * t;
    real ncr = rexp(LN10 * lg);
    real dncr = ncr * (-1.3 + 3.24 * t) / T;
    real a = ncr / (ncr + c.n);
    real da = c.n * dncr / ((ncr + c.n) * (ncr + c.n));
    real lnk = (1.0 - a) * lnkh + a * lnkl;
    real dlnk = (1.0 - a) * dlnkh + a * dlnkl + (lnkl - lnkh) * da;
    r.k[7] = rexp(lnk);
    r.dk[7] = r.k[7] * dlnk;
  }
  /* H8: 2H + grain -> H2, T_d frozen, scaled by Z / Z_sun */
  {
    real fa = 1.0 / (1.0 + rexp(7.5e2 * (1.0 / 75.0 - 1.0 / Td)));
    real s = rsqrt(T + Td);
    real D = 1.0 + 4.0e-2 * s + 2.0e-3 * T + 8.0e-6 * T * T;
    r.k[8] = 6.0e-17 * rsqrt(T / 300.0) * fa * c.fd / D;
    r.dk[8] = r.k[8] * (0.5 / T - (2.0e-2 / s + 2.0e-3 + 1.6e-5 * T) / D);
  }
  /* H9, H10, H11: photoionisation, photodissociation, cosmic rays */
  r.k[9] = c.k9;
  r.dk[9] = 0.0;
  r.k[10] = c.k10;
  r.dk[10] = 0.0;
  r.k[11] = c.k11;
  r.dk[11] = 0.0;

  for (int i = 0; i < ORC_NREAC; ++i) {
    if (i >= 9) break; /* photo/CR multipliers are already in the cell rates */
    r.k[i] = net.reac_mult[i] * r.k[i];
    r.dk[i] = net.reac_mult[i] * r.dk[i];
  }
}

/* ------------------------------------------------------------------ */
/* H2 self-shielding factor f_sh as a function of (y_H2, T).  STAND-IN for
 * the prescription the paper takes from its reference (text after Table
 * "Thermal processes"): the self-shielding fit of Draine & Bertoldi (1996),
 *   f_sh = 0.965 / (1 + x / b5)^2 + 0.035 / sqrt(1 + x) exp(-8.5e-4 sqrt(1 + x)),
 * x = N_H2 / 5e14 cm^-2, b5 the Doppler parameter in km/s, with the local
 * column N_H2 = y_H2 n_H L, L = shield_len times the Jeans length
 * sqrt(pi k_B T / (G m_H rho)) of the cell (so L grows as sqrt(T)).
 * Returns f_sh as a G3 with its y_H2 and T partials. */
static G3 h2_shield(const orc_network& net, real y2, real T, const Cell& c) {
  const real L = net.shield_len * rsqrt(3.14159265358979323846 * K_B * T / (G_GRAV * M_H * c.rho));
  const real dxdy = c.n * L / 5.0e14;
  const real x = y2 * dxdy;
  const real dxdT = x / (2.0 * T);
  const real b5 = net.shield_b5;
  const real u = 1.0 + x / b5;
  const real sq = rsqrt(1.0 + x);
  const real ex = rexp(-8.5e-4 * sq);
  const real f = 0.965 / (u * u) + 0.035 / sq * ex;
  /* d/dx: -2 0.965 / (b5 u^3) + 0.035 ex (-1/sq^2 - 8.5e-4 / sq) / (2 sq) */
  const real dfdx = -2.0 * 0.965 / (b5 * u * u * u) +
                    0.035 * ex * (-1.0 / (sq * sq) - 8.5e-4 / sq) / (2.0 * sq);
  return G3{f, dfdx * dxdy, 0.0, dfdx * dxdT};
}

/* Photoelectric heating with grain charging and the cooling by electron
 * recombination on grains, as functions of (y_e, T).  STAND-IN for the
 * rates the paper takes from its reference (Table "Thermal processes",
 * process 4, and the text after it): the efficiency of Bakes & Tielens
 * (1994) in the form of Wolfire et al. (2003) with charging parameter
 * psi = G0 sqrt(T) / n_e,
 *   eps = 0.0487 / (1 + 4e-3 psi^0.73) + 0.0365 (T / 1e4)^0.7 / (1 + 2e-4 psi),
 *   Gamma_pe = 1.3e-24 eps G0 n_H f_d,
 *   Lambda_rec = 4.65e-30 T^0.94 psi^beta n_e n_H f_d,  beta = 0.735 T^-0.068.
 * Reading: n_e is floored at y_abs n_H inside psi (psi stays finite in
 * neutral gas; the floor is the abundance floor of the timescales). */
static void photoelectric(const orc_params& p, real ye, real T, const Cell& c, G3& heat,
                          G3& rec) {
  if (!(c.g0 > real(0.0))) { /* no FUV field: no photoelectrons, neutral grains */
    heat = cst(0.0);
    rec = cst(0.0);
    return;
  }
  const bool floored = ye < real(p.y_abs);
  const real yef = floored ? real(p.y_abs) : ye;
  const real ne = yef * c.n;
  const real psi = c.g0 * rsqrt(T) / ne;
  const real dpsi_dye = floored ? real(0.0) : -psi / ye;
  const real dpsi_dT = psi / (2.0 * T);
  const real p73 = rpow(psi, 0.73);
  const real a1 = 1.0 + 4.0e-3 * p73;
  const real tt = rpow(T / 1.0e4, 0.7);
  const real b1 = 1.0 + 2.0e-4 * psi;
  const real eps = 0.0487 / a1 + 0.0365 * tt / b1;
  /* d eps / d psi and the explicit T dependence through (T/1e4)^0.7 */
  const real deps_dpsi = -0.0487 * (4.0e-3 * 0.73 * p73 / psi) / (a1 * a1) -
                         0.0365 * tt * 2.0e-4 / (b1 * b1);
  const real deps_dT = 0.0365 * (0.7 * tt / T) / b1;
  const real ch = 1.3e-24 * c.g0 * c.n * c.fd;
  heat = G3{ch * eps, 0.0, ch * deps_dpsi * dpsi_dye,
            ch * (deps_dpsi * dpsi_dT + deps_dT)};
  /* Lambda_rec = 4.65e-30 n_H^2 f_d y_e T^0.94 psi^beta */
  const real beta = 0.735 * rpow(T, -0.068);
  const real dbeta_dT = -0.068 * beta / T;
  const real lpsi = rlog(psi);
  const real pb = rexp(beta * lpsi);
  const real t94 = rpow(T, 0.94);
  const real cr = 4.65e-30 * c.n * c.n * c.fd;
  const real v = cr * ye * t94 * pb;
  /* d/dy_e: ye psi^beta with psi ~ 1/y_e (unfloored): (1 - beta) psi^beta */
  const real dv_dye = cr * t94 * pb * (1.0 + ye * beta * dpsi_dye / psi);
  const real dv_dT = v * (0.94 / T + dbeta_dT * lpsi + beta * dpsi_dT / psi);
  rec = G3{v, 0.0, dv_dye, dv_dT};
}

/* ------------------------------------------------------------------ */
/* Chemistry and gas heating/cooling, Tables "Chemical reactions" and  */
/* "Thermal processes".  Returns R_H2, R_e [1/s] and Q = Gamma - Lambda */
/* [erg cm^-3 s^-1] with partials w.r.t. (y_H2, y_e, T); T_d frozen.   */
struct ChemOut {
  G3 rh2, re, q;
  real terms[ORC_NPROC];
  real yhm, dyhm_dye, dyhm_dT; /* steady-state H- */
};

static void chem(const orc_network& net, const orc_params& p, real y2, real ye, real Tin,
                 real Td, const Cell& c, ChemOut& o) {
  /* Reading: the fits are evaluated at T clamped to [1, 1e8] K */
  real T = Tin;
  real dTr = 1.0;
  if (T < real(T_RATE_MIN)) { T = T_RATE_MIN; dTr = 0.0; }
  if (T > real(T_RATE_MAX)) { T = T_RATE_MAX; dTr = 0.0; }

  Rates r;
  rates(net, T, Td, c, r);
  const real lnT = r.lnT;
  const real n = c.n;
  const double* pm = net.proc_mult;

  /* H- in steady state between formation (H2) and destruction (H3):
   * y_H- = (k_H2 / k_H3) y_e (Appendix A, H- as an intermediate). */
  real ratio = 0.0, dratio = 0.0;
  if (r.k[3] > real(0.0)) {
    ratio = r.k[2] / r.k[3];
    dratio = (r.dk[2] * r.k[3] - r.k[2] * r.dk[3]) / (r.k[3] * r.k[3]);
  }
  const G3 yH2{y2, 1.0, 0.0, 0.0};
  const G3 yE{ye, 0.0, 1.0, 0.0};
  const G3 yHm{ratio * ye, 0.0, ratio, dratio * ye};
  const G3 yHp = yE + yHm;                              /* charge neutrality    */
  const G3 yH = cst(1.0) - 2.0 * yH2 - yHp - yHm;      /* H-nuclei conservation */

  G3 k[ORC_NREAC];
  for (int i = 0; i < ORC_NREAC; ++i) k[i] = tfun(r.k[i], r.dk[i]);

  /* reaction rates per H nucleus [1/s] */
  G3 r0 = n * (k[0] * yH * yE);            /* H + e -> H+ + 2e           */
  G3 r1 = n * (k[1] * yHp * yE);           /* H+ + e -> H                */
  G3 r23 = n * (k[2] * yH * yE);           /* H- channel: net H2 formation */
  G3 r4 = n * (k[4] * yH2 * yH);           /* H2 + H -> 3H               */
  G3 r5 = (n * n) * (k[5] * yH * yH * yH); /* 3H -> H2 + H               */
  G3 r6 = (n * n) * (k[6] * yH * yH * yH2);/* 2H + H2 -> 2H2             */
  G3 r7 = n * (k[7] * yH2 * yH2);          /* 2H2 -> 2H + H2             */
  G3 r8 = n * (k[8] * yH);                 /* grains: dy_H2/dt = k n y_H */
  G3 r9 = k[9] * yH;                       /* photoionisation            */
  /* photodissociation, with H2 self-shielding in shield_mode 1 */
  const G3 shield = net.shield_mode == 1 ? h2_shield(net, y2, T, c) : cst(1.0);
  G3 r10 = k[10] * (shield * yH2);
  G3 r11 = k[11] * yH;                     /* cosmic rays                */

  o.rh2 = r23 + r5 + r6 + r8 - r4 - r7 - r10;
  o.re = r0 - r1 + r9 + r11;

  /* ---- heating ---- */
  /* Gamma_1, H2 formation heating; f = (1 + n_cr/n_H)^-1 written as
   * n D / (n D + 1e6 T^-1/2) so that it never divides by zero.
   * Reading: the third term is grain formation k_H8 n n(H) (the printed
   * k_H7 n^2(H2) is collisional dissociation, a cooling channel). */
  G3 gam1;
  {
    real e1 = rexp(-(400.0 / T) * (400.0 / T));
    real de1 = e1 * 2.0 * 400.0 * 400.0 / (T * T * T);
    real e2 = rexp(-12000.0 / (T + 1200.0));
    real de2 = e2 * 12000.0 / ((T + 1200.0) * (T + 1200.0));
    G3 D = 1.6 * (yH * tfun(e1, de1)) + 1.4 * (yH2 * tfun(e2, de2));
    real g = 1.0e6 / rsqrt(T);
    G3 nD = n * D;
    G3 f = nD / (nD + tfun(g, -0.5 * g / T));
    G3 a = 3.73 * (f * (k[3] * yH * yHm)) * (n * n);
    G3 b = 4.48 * (f * (k[5] * yH * yH * yH)) * (n * n * n);
    G3 cc = (cst(0.2) + 4.2 * f) * (k[8] * yH) * (n * n);
    gam1 = (pm[0] * EV) * (a + b + cc);
  }
  /* Gamma_2, Gamma_3, Gamma_4: STAND-INS (the paper defers to its
   * references): fixed heat per photoionisation and photodissociation,
   * photoelectric heating with constant efficiency. */
  G3 gam2 = (pm[1] * net.heat_euv_ev * EV * n) * (k[9] * yH);
  G3 gam3 = (pm[2] * net.heat_h2diss_ev * EV * n) * (k[10] * (shield * yH2));
  /* Gamma_4: constant efficiency (pe_mode 0), or grain-charge efficiency
   * with the cooling by electron recombination on the charged grains
   * (pe_mode 1; both scaled by the multiplier of process 4) */
  G3 gam4 = cst(pm[3] * net.pe_coef * net.pe_eps * c.g0 * n * c.fd);
  G3 lamrec = cst(0.0);
  if (net.pe_mode == 1) {
    G3 pe_heat, pe_rec;
    photoelectric(p, ye, T, c, pe_heat, pe_rec);
    gam4 = pm[3] * pe_heat;
    lamrec = pm[3] * pe_rec;
  }

  /* ---- cooling ---- */
  const real n2 = n * n;
  G3 lam5 = (pm[4] * 13.6 * EV * n2) * (k[0] * yH * yE);
  G3 lam6 = (pm[5] * 4.48 * EV * n2) * (k[4] * yH2 * yH + k[7] * yH2 * yH2);
  G3 c7;
  {
    real l = lnT / LN10;
    const double cf[6] = {-25.87, 0.4958, -0.1052, 0.04264, -9.165e-3, 5.491e-4};
    real P = cf[5], dP = 5.0 * cf[5];
    for (int i = 4; i >= 0; --i) P = P * l + cf[i];
    for (int i = 4; i >= 1; --i) dP = dP * l + real(i) * cf[i];
    real v = rexp(LN10 * P);
    c7 = tfun(v, v * dP / T);
  }
  G3 lam7 = (pm[6] * n2) * (c7 * yHp * yE);
  G3 lam8 = (pm[7] * K_B * n2) * (tfun(T, 1.0) * k[2] * yH * yE);
  real sq5 = rsqrt(T / 1.0e5);
  real dsq5 = 0.5 * sq5 / T;
  G3 c9, c10;
  {
    real ex = rexp(-118348.0 / T);
    real v = 7.5e-19 * ex / (1.0 + sq5);
    c9 = tfun(v, v * (118348.0 / (T * T) - dsq5 / (1.0 + sq5)));
  }
  /* Reading: collisional excitation of neutral H, so the partner is n(H)
   * (the table prints n(H+)). */
  G3 lam9 = (pm[8] * n2) * (c9 * yE * yH);
  {
    real ex = rexp(-473638.0 / T);
    real v = 5.54e-17 * rpow(T, -0.397) * ex / (1.0 + sq5);
    c10 = tfun(v, v * (-0.397 / T + 473638.0 / (T * T) - dsq5 / (1.0 + sq5)));
  }
  /* He+ abundance: all helium taken as ionised (table note). */
  G3 lam10 = (pm[9] * n2 * p.y_he) * (c10 * yE);
  G3 c11;
  {
    real l = lnT / LN10;
    real sT = rsqrt(T);
    real gff, dgff;
    if (T < real(3.2e5)) {
      gff = 0.79464 + 0.1243 * l;
      dgff = 0.1243 / (T * LN10);
    } else {
      gff = 2.13164 - 0.1240 * l;
      dgff = -0.1240 / (T * LN10);
    }
    real v = 1.426e-27 * sT * gff;
    c11 = tfun(v, 1.426e-27 * (0.5 * gff / sT + sT * dgff));
  }
  G3 lam11 = (pm[10] * n2) * (c11 * yHp * yE);
  real tc4 = p.t_cmb * p.t_cmb * p.t_cmb * p.t_cmb;
  G3 lam12 = (pm[11] * 1.017e-37 * tc4 * n) * (tfun(T - p.t_cmb, 1.0) * yE);

  /* Lambda_13, line cooling.  STAND-IN (the paper defers to its reference):
   * each coolant is a two-level system in statistical equilibrium,
   *   n_u / n_X = C_lu / (C_lu + C_ul + A),  C_lu = g C_ul exp(-T_ul/T),
   * cooling = n_X n_u/n_X A k_B T_ul.  Emitters: H2 (J = 2 -> 0), all C as
   * C II, O neutral in proportion to 1 - y_H+, O II / O III sharing the
   * ionised part with the fixed fraction f_oiii. */
  G3 lam13 = cst(0.0);
  {
    real s100 = rsqrt(100.0 / T);
    G3 esc = tfun(s100, -0.5 * s100 / T);
    G3 ncolln = n * (yH + yH2);
    G3 emit[ORC_NLINE];
    emit[0] = n * yH2;
    emit[1] = cst(net.x_c * c.fd * n);
    emit[2] = (net.x_o * c.fd * n) * (cst(1.0) - yHp);
    emit[3] = (net.x_o * c.fd * n * (1.0 - net.f_oiii)) * yHp;
    emit[4] = (net.x_o * c.fd * n * net.f_oiii) * yHp;
    for (int j = 0; j < ORC_NLINE; ++j) {
      real b = rexp(-net.line_tul[j] / T);
      G3 bf = tfun(b, b * net.line_tul[j] / (T * T));
      G3 cul = net.line_qn[j] * ncolln + (net.line_qe100[j] * n) * (esc * yE);
      G3 clu = net.line_g[j] * (bf * cul);
      G3 frac = clu / (clu + cul + cst(net.line_a[j]));
      lam13 = lam13 + (K_B * net.line_tul[j] * net.line_a[j]) * (emit[j] * frac);
    }
    lam13 = pm[12] * lam13;
  }

  o.q = gam1 + gam2 + gam3 + gam4 -
        (lam5 + lam6 + lam7 + lam8 + lam9 + lam10 + lam11 + lam12 + lam13 + lamrec);
  G3 all[14] = {gam1, gam2, gam3, gam4, lam5, lam6, lam7, lam8, lam9, lam10, lam11, lam12, lam13,
                lamrec};
  for (int i = 0; i < 14; ++i) o.terms[i] = all[i].v;

  /* temperature clamp: no dependence outside the fitted range */
  o.rh2.t = o.rh2.t * dTr;
  o.re.t = o.re.t * dTr;
  o.q.t = o.q.t * dTr;
  o.yhm = ratio * ye;
  o.dyhm_dye = ratio;
  o.dyhm_dT = dratio * ye * dTr;
}

/* steady-state H- ratio k_H2/k_H3 at temperature T (for renormalisation) */
static real hminus_ratio(const orc_network& net, real T) {
  if (T < real(T_RATE_MIN)) T = T_RATE_MIN;
  if (T > real(T_RATE_MAX)) T = T_RATE_MAX;
  real k2, dk2, k3, dk3;
  k2k3(T, 0.0, k2, dk2, k3, dk3);
  k2 = net.reac_mult[2] * k2;
  k3 = net.reac_mult[3] * k3;
  return k3 > real(0.0) ? k2 / k3 : real(0.0);
}

/* ------------------------------------------------------------------ */
/* Dust opacity per gram of gas at Z_sun.  STAND-IN for the tabulated  */
/* opacity the paper uses: kappa_max x^2/(1+x^2), x = T/T_norm.         */
static inline void kappa(const orc_network& net, real T, real& k, real& dk) {
  real x = T / net.kappa_tnorm;
  real d = 1.0 + x * x;
  k = net.kappa_max * x * x / d;
  dk = net.kappa_max * 2.0 * x / (d * d) / net.kappa_tnorm;
}

/* Appendix C sources and linear-system coefficients */
struct Dust {
  real G, gd, zeta;       /* R_g n sqrt(T_g/T_high), gamma_d, zeta      */
  real kd, betad;         /* kappa(T_d), beta_d                          */
  real absir, betair;     /* kappa(T_IR) c~ E_IR, beta_IR                */
  real Sd, Sir, Sg, alpha;/* sources; alpha_g = c_v / rho                */
  real sd_noise, sir_noise; /* rounding level of S_d and S_IR (dust_rate) */
};

/* Reading (the dust timescale at radiative equilibrium): near equilibrium
 * the net sources S_d and S_IR are differences of terms many orders of
 * magnitude larger than themselves, each known to a few units in the last
 * place, so their computed values are rounding noise; Eq.
 * timescale_of_dust would then take its step limit from that noise.  A net
 * source within SRC_NOISE of the sum of its gross terms (64 ulps) sets no
 * timescale: the rate entering Eq. timescale_of_dust is |S| minus that
 * level, floored at zero (continuous in S). */
const double SRC_NOISE = 64.0 * 2.220446049250313e-16;

static void dust_eval(const orc_network& net, const orc_params& p, real Tg, real Td, real Eir,
                      real cv, const Cell& c, Dust& d) {
  const real ctil = p.c_red * C_LIGHT;
  d.G = net.proc_mult[13] * R_G * c.n * rsqrt(Tg / T_HIGH);
  real el = rexp(-T_LOW / Tg);
  d.gd = 1.0 - 0.8 * el;
  real ratio = Td / Tg - 1.0;
  d.zeta = 0.5 * d.gd * ratio + (d.gd - 1.0) * (T_LOW / Tg) * ratio - d.gd;
  real kd, dkd;
  kappa(net, Td, kd, dkd);
  d.kd = kd;
  d.betad = 4.0 * kd + dkd * Td;
  if (p.ir_mode == ORC_IR_EVOLVE) {
    real tir = rsqrt(rsqrt(p.c_red * Eir / A_RAD));
    real ki, dki;
    kappa(net, tir, ki, dki);
    d.absir = ki * ctil * Eir;
    d.betair = ki + dki * tir / 4.0;
  } else {
    /* FIXED: E_IR = (c/c~) a T_CMB^4, i.e. T_IR = T_CMB */
    real ki, dki;
    kappa(net, p.t_cmb, ki, dki);
    real tc4 = p.t_cmb * p.t_cmb * p.t_cmb * p.t_cmb;
    d.absir = ki * C_LIGHT * A_RAD * tc4;
    d.betair = ki + dki * p.t_cmb / 4.0;
  }
  real td4 = Td * Td * Td * Td;
  real emis = kd * A_RAD * C_LIGHT * td4;
  real coup = d.G * d.gd * (Td - Tg);
  d.Sd = d.absir + c.e_uv - emis - coup;
  d.Sir = c.rho * c.fd * (emis - d.absir);
  d.Sg = d.G * c.fd * d.gd * (Td - Tg);
  d.alpha = cv / c.rho;
  d.sd_noise = SRC_NOISE * (rabs(d.absir) + rabs(real(c.e_uv)) + rabs(emis) + rabs(coup));
  d.sir_noise = SRC_NOISE * (c.rho * c.fd) * (rabs(emis) + rabs(d.absir));
}

/* Gaussian elimination with partial pivoting (ties: lowest row). */
static int lu_solve(int n, real A[3][3], real b[3], real x[3]) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    real best = rabs(A[k][k]);
    for (int i = k + 1; i < n; ++i) {
      if (rabs(A[i][k]) > best) {
        best = rabs(A[i][k]);
        piv = i;
      }
    }
    if (piv != k) {
      for (int j = 0; j < n; ++j) {
        real t = A[k][j];
        A[k][j] = A[piv][j];
        A[piv][j] = t;
      }
      real t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
    if (A[k][k] == real(0.0)) return -1;
    for (int i = k + 1; i < n; ++i) {
      real m = A[i][k] / A[k][k];
      for (int j = k + 1; j < n; ++j) A[i][j] = A[i][j] - m * A[k][j];
      b[i] = b[i] - m * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    real s = b[i];
    for (int j = i + 1; j < n; ++j) s = s - A[i][j] * x[j];
    x[i] = s / A[i][i];
  }
  return 0;
}

/* ------------------------------------------------------------------ */
struct State {
  real y2, ye, E, Td, Eir;
};

static inline real ntot_rel(const orc_params& p, real y2, real ye) {
  /* particles per H nucleus: H + H2 + H+ + H- + e + He = 1 - y_H2 + y_e + y_He */
  return 1.0 - y2 + ye + p.y_he;
}
static inline real cv_of(const orc_params& p, const Cell& c, real y2, real ye) {
  return K_B * c.n * ntot_rel(p, y2, ye) / (p.gamma_ad - 1.0);
}

/* Renormalisation after a chemistry update (Reading: clamp the two
 * unknowns, rebuild y_H-, y_H+, y_H from conservation; if y_H < 0 rescale
 * the molecular/ionic set so that H nuclei are conserved; floor E_th at
 * T_g = T_CMB).  Returns the flags raised. */
static uint32_t renormalise(const orc_network& net, const orc_params& p, const Cell& c, State& s,
                            bool isothermal, real Tiso) {
  uint32_t fl = 0;
  if (s.y2 < real(0.0)) { s.y2 = 0.0; fl |= ORC_F_FLOOR; }
  if (s.y2 > real(0.5)) { s.y2 = 0.5; fl |= ORC_F_FLOOR; }
  if (s.ye < real(0.0)) { s.ye = 0.0; fl |= ORC_F_FLOOR; }
  if (s.ye > real(1.0)) { s.ye = 1.0; fl |= ORC_F_FLOOR; }
  real T = isothermal ? Tiso : s.E / cv_of(p, c, s.y2, s.ye);
  real ratio = hminus_ratio(net, T);
  real yhm = ratio * s.ye;
  real yhp = s.ye + yhm;
  real yh = 1.0 - 2.0 * s.y2 - yhp - yhm;
  if (yh < real(0.0)) {
    real sc = 1.0 / (2.0 * s.y2 + yhp + yhm);
    s.y2 = s.y2 * sc;
    s.ye = s.ye * sc;
    fl |= ORC_F_FLOOR;
  }
  real cv = cv_of(p, c, s.y2, s.ye);
  if (isothermal) {
    s.E = cv * Tiso;
  } else if (s.E < cv * p.t_cmb) {
    s.E = cv * p.t_cmb;
    fl |= ORC_F_FLOOR;
  }
  return fl;
}

static void make_cell(const orc_network& net, const orc_params& p, double nh, double neuv,
                      double nfuv, double z, Cell& c) {
  c.n = nh;
  c.fd = z;
  c.rho = (1.0 + 4.0 * p.y_he) * M_H * c.n;
  c.n_euv = neuv;
  c.n_fuv = nfuv;
  c.g0 = c.n_fuv / net.g0_photon_density;
  /* STAND-INS (photo rates; the paper derives them from the EUV/FUV
   * energy densities in its reference): k_H9 = c sigma N_EUV,
   * k_H10 = k10_per_g0 G0, k_H11 = zeta_CR. */
  c.k9 = net.reac_mult[9] * (C_LIGHT * net.sigma_euv * c.n_euv);
  c.k10 = net.reac_mult[10] * (net.k10_per_g0 * c.g0);
  c.k11 = net.reac_mult[11] * net.zeta_cr;
  /* STAND-IN: dust UV absorption c kappa_UV (N_FUV e_FUV + N_EUV e_EUV) */
  c.e_uv = C_LIGHT * net.kappa_uv * (c.n_fuv * net.e_fuv_ev + c.n_euv * net.e_euv_ev) * EV;
}

/* Appendix C: one linearised solve of the dust / IR / gas-grain system.
 * Unknowns (dT_d, dE_IR, dT_g); FIXED IR mode drops dE_IR. */
static void dust_matrix(const orc_params& p, const Dust& d, const Cell& c, real Td, real Tg, real h,
                        real A[3][3], real rhs[3]) {
  const real ctil = p.c_red * C_LIGHT;
  const real ac = A_RAD * C_LIGHT;
  const real td3 = Td * Td * Td;
  A[0][0] = p.dust_cap + h * d.G * d.gd + h * ac * td3 * d.betad;
  A[0][1] = -(h * ctil * d.betair);
  A[0][2] = h * d.G * d.zeta;
  A[1][0] = -(c.rho * h * ac * td3 * c.fd * d.betad);
  A[1][1] = 1.0 + c.rho * h * ctil * c.fd * d.betair;
  A[1][2] = 0.0;
  A[2][0] = -(h * c.fd * d.G * d.gd);
  A[2][1] = 0.0;
  A[2][2] = d.alpha - h * c.fd * d.G * d.zeta;
  rhs[0] = h * d.Sd;
  rhs[1] = h * d.Sir;
  rhs[2] = h * c.fd * d.G * d.gd * (Td - Tg);
}

static void dust_linear_step(const orc_network& net, const orc_params& p, const Cell& c, State& s,
                             real h) {
  (void)net;
  real cv = cv_of(p, c, s.y2, s.ye);
  real Tg = s.E / cv;
  Dust d;
  dust_eval(net, p, Tg, s.Td, s.Eir, cv, c, d);
  real A[3][3], rhs[3];
  dust_matrix(p, d, c, s.Td, Tg, h, A, rhs);
  /* column scaling by (T_d, E_IR, T_g), row scaling by the capacities */
  real x[3] = {0.0, 0.0, 0.0};
  if (p.ir_mode == ORC_IR_EVOLVE) {
    real cs[3] = {s.Td, s.Eir, Tg};
    real rs[3] = {p.dust_cap * s.Td, s.Eir, d.alpha * Tg};
    real M[3][3], b[3];
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) M[i][j] = A[i][j] * cs[j] / rs[i];
      b[i] = rhs[i] / rs[i];
    }
    lu_solve(3, M, b, x);
    s.Td = s.Td + x[0] * s.Td;
    s.Eir = s.Eir + x[1] * s.Eir;
    s.E = s.E + cv * (x[2] * Tg);
  } else {
    real cs[2] = {s.Td, Tg};
    real rs[2] = {p.dust_cap * s.Td, d.alpha * Tg};
    const int id[2] = {0, 2};
    real M[3][3], b[3];
    for (int i = 0; i < 2; ++i) {
      for (int j = 0; j < 2; ++j) M[i][j] = A[id[i]][id[j]] * cs[j] / rs[i];
      b[i] = rhs[id[i]] / rs[i];
    }
    lu_solve(2, M, b, x);
    s.Td = s.Td + x[0] * s.Td;
    s.E = s.E + cv * (x[1] * Tg);
  }
}

/* Tight gas-dust coupling (Reading of "iterative calculations are required
 * only when gas and dust grains are tightly coupled"): backward Euler of
 * the Appendix C system over h with G, gamma_d and kappa(T_IR) frozen at
 * the substep start.  T_g and E_IR are then explicit functions of T_d and
 * the system reduces to one strictly increasing scalar equation Phi(T_d)=0,
 * solved by bracketed (safeguarded) Newton.  Returns iterations; sets
 * *conv = false if newton_max is reached, *floored if the root is below the
 * floor. */
struct Tight {
  const orc_network* net;
  const orc_params* p;
  const Cell* c;
  real td0, tg0, e0, h, alpha, ggd, w, dg, P, qd, absfix, kir;
};

static void tight_phi(const Tight& t, real x, real& phi, real& dphi) {
  const orc_params& p = *t.p;
  const real ac = A_RAD * C_LIGHT;
  const real ctil = p.c_red * C_LIGHT;
  real k, dk;
  kappa(*t.net, x, k, dk);
  real x3 = x * x * x;
  real emis = k * ac * x3 * x;
  real demis = ac * x3 * (4.0 * k + dk * x);
  real ab, dab;
  if (p.ir_mode == ORC_IR_EVOLVE) {
    real E = (t.e0 + t.P * emis) / t.qd;
    ab = t.kir * ctil * E;
    dab = t.kir * ctil * t.P * demis / t.qd;
  } else {
    ab = t.absfix;
    dab = 0.0;
  }
  real coup = t.ggd * t.dg * (x - t.tg0);
  phi = t.p->dust_cap * (x - t.td0) - t.h * (ab + t.c->e_uv - emis - coup);
  dphi = t.p->dust_cap - t.h * (dab - demis - t.ggd * t.dg);
}

static int dust_tight_step(const orc_network& net, const orc_params& p, const Cell& c, State& s,
                           real h, bool& conv, bool& floored) {
  const real ac = A_RAD * C_LIGHT;
  const real ctil = p.c_red * C_LIGHT;
  real cv = cv_of(p, c, s.y2, s.ye);
  real Tg0 = s.E / cv;
  Tight t;
  t.net = &net;
  t.p = &p;
  t.c = &c;
  t.td0 = s.Td;
  t.tg0 = Tg0;
  t.e0 = s.Eir;
  t.h = h;
  t.alpha = cv / c.rho;
  real G = net.proc_mult[13] * R_G * c.n * rsqrt(Tg0 / T_HIGH);
  real gd = 1.0 - 0.8 * rexp(-T_LOW / Tg0);
  t.ggd = G * gd;
  t.w = h * c.fd * t.ggd;
  t.dg = t.alpha / (t.alpha + t.w); /* T_d - T_g(T_d) = dg (T_d - T_g0) */
  t.P = h * c.rho * c.fd;
  t.kir = 0.0;
  t.qd = 1.0;
  t.absfix = 0.0;
  if (p.ir_mode == ORC_IR_EVOLVE) {
    real tir = rsqrt(rsqrt(p.c_red * s.Eir / A_RAD));
    real dk;
    kappa(net, tir, t.kir, dk);
    t.qd = 1.0 + t.P * ctil * t.kir;
  } else {
    real ki, dk;
    kappa(net, p.t_cmb, ki, dk);
    real tc4 = p.t_cmb * p.t_cmb * p.t_cmb * p.t_cmb;
    t.absfix = ki * ac * tc4;
  }
  conv = true;
  floored = false;
  int it = 0;
  real lo = p.t_cmb, hi;
  real f, fp;
  tight_phi(t, lo, f, fp);
  real x;
  if (f >= real(0.0)) {
    x = lo;
    floored = true;
  } else {
    hi = rmax(rmax(t.td0, t.tg0), lo);
    tight_phi(t, hi, f, fp);
    int guard = 0;
    while (f <= real(0.0) && guard < 200) {
      lo = hi;
      hi = hi * 2.0;
      tight_phi(t, hi, f, fp);
      ++guard;
    }
    /* Phi is increasing and convex (the T^4 emission term dominates and the
     * IR back-coupling only scales it by a factor below one), so Newton
     * started where Phi >= 0 decreases monotonically to the root; a step
     * taken from the left lands right of the root, or at hi. */
    x = t.td0;
    if (!(x > lo && x <= hi)) x = hi;
    conv = false;
    for (it = 1; it <= p.newton_max; ++it) {
      tight_phi(t, x, f, fp);
      if (f == real(0.0)) { conv = true; break; }
      real xn = x - f / fp;
      if (f < real(0.0)) {
        lo = x;
        if (!(xn < hi)) xn = hi;
      } else {
        hi = x;
        if (!(xn > lo)) xn = 0.5 * (lo + hi);
      }
      real dx = xn - x;
      x = xn;
      if (rabs(dx) <= p.newton_rtol * x) {
        /* one polishing Newton step */
        tight_phi(t, x, f, fp);
        xn = x - f / fp;
        if (xn >= lo && xn <= hi) x = xn;
        conv = true;
        break;
      }
    }
    if (it > p.newton_max) it = p.newton_max;
  }
  /* back-substitute T_g and E_IR */
  real tg = (t.alpha * t.tg0 + t.w * x) / (t.alpha + t.w);
  if (p.ir_mode == ORC_IR_EVOLVE) {
    real k, dk;
    kappa(net, x, k, dk);
    s.Eir = (t.e0 + t.P * k * ac * x * x * x * x) / t.qd;
  }
  s.Td = x;
  s.E = s.E + cv * (tg - Tg0);
  return it;
}

/* floors after the dust update (Reading: T_g, T_d >= T_CMB, T_IR >= T_CMB) */
static uint32_t dust_floors(const orc_params& p, const Cell& c, State& s) {
  uint32_t fl = 0;
  if (s.Td < real(p.t_cmb)) { s.Td = p.t_cmb; fl |= ORC_F_FLOOR; }
  real cv = cv_of(p, c, s.y2, s.ye);
  if (s.E < cv * p.t_cmb) { s.E = cv * p.t_cmb; fl |= ORC_F_FLOOR; }
  if (p.ir_mode == ORC_IR_EVOLVE) {
    real tc4 = p.t_cmb * p.t_cmb * p.t_cmb * p.t_cmb;
    real emin = A_RAD * tc4 / p.c_red;
    if (s.Eir < emin) { s.Eir = emin; fl |= ORC_F_FLOOR; }
  }
  return fl;
}

/* inverse dust timescale, Eq. timescale_of_dust (gas side: gas-grain only) */
static real dust_rate(const orc_params& p, const Dust& d, real Td, real Tg, real Eir) {
  real nu = rmax(rabs(d.Sd) - d.sd_noise, real(0.0)) / (p.dust_cap * Td);
  nu = rmax(nu, rabs(d.Sg) / (d.alpha * Tg));
  if (p.ir_mode == ORC_IR_EVOLVE) nu = rmax(nu, rmax(rabs(d.Sir) - d.sir_noise, real(0.0)) / Eir);
  return nu;
}

static bool input_ok(const orc_params& p, double nh, double neuv, double nfuv, double z, double y2,
                     double ye, double E, double Td, double Eir) {
  auto fin = [](double v) { return std::isfinite(v); };
  if (!(fin(nh) && nh > 0.0)) return false;
  if (!(fin(neuv) && neuv >= 0.0)) return false;
  if (!(fin(nfuv) && nfuv >= 0.0)) return false;
  if (!(fin(z) && z >= 0.0)) return false;
  if (!(fin(y2) && y2 >= 0.0)) return false;
  if (!(fin(ye) && ye >= 0.0)) return false;
  if (!(fin(E) && E > 0.0)) return false;
  if (!(fin(Td) && Td > 0.0)) return false;
  if (p.ir_mode == ORC_IR_EVOLVE && !(fin(Eir) && Eir > 0.0)) return false;
  return true;
}

struct CellIn {
  double nh, neuv, nfuv, z;
};

static void load(const orc_params& p, const orc_cells& cs, int64_t i, CellIn& ci, State& s) {
  ci.nh = cs.nh[i];
  ci.neuv = cs.n_euv[i];
  ci.nfuv = cs.n_fuv[i];
  ci.z = cs.zmet ? cs.zmet[i] : p.z_default;
  s.y2 = cs.y_h2[i];
  s.ye = cs.y_e[i];
  s.E = cs.eint[i];
  s.Td = cs.tdust[i];
  real tc4 = p.t_cmb * p.t_cmb * p.t_cmb * p.t_cmb;
  s.Eir = (p.ir_mode == ORC_IR_EVOLVE) ? real(cs.eir[i]) : real(A_RAD * tc4 / p.c_red);
}

/* EUV and FUV photons absorbed over the hydro step after the update (Sec. 2
 * "Radiation components": absorptions are accounted for after the
 * abundances and temperatures are updated).  The absorption term of the
 * reduced-speed-of-light transport, dN/dt = -c~ alpha N, integrated
 * exactly over dt with the absorbers of the updated state: alpha_EUV =
 * sigma_EUV n_H y_H + kappa_UV rho f_d (photoionisation and dust),
 * alpha_FUV = kappa_UV rho f_d (dust).  STAND-IN for the scheme of the
 * paper's reference (its Appendix C is not reproduced in the paper). */
static void absorb_photons(const orc_network& net, const orc_params& p, const Cell& c, real yh,
                           double dt, real& neuv, real& nfuv) {
  const real ctil = p.c_red * C_LIGHT;
  const real a_dust = net.kappa_uv * c.rho * c.fd;
  const real a_euv = net.sigma_euv * c.n * rmax(yh, real(0.0)) + a_dust;
  neuv = c.n_euv * rexp(-ctil * a_euv * dt);
  nfuv = c.n_fuv * rexp(-ctil * a_dust * dt);
}

static void store(const orc_network& net, const orc_params& p, const orc_cells& cs, int64_t i,
                  const Cell& c, const State& s, bool isothermal, real Tiso, int nsub, int nit,
                  uint32_t fl, double dt) {
  cs.y_h2[i] = rval(s.y2);
  cs.y_e[i] = rval(s.ye);
  cs.eint[i] = rval(s.E);
  cs.tdust[i] = rval(s.Td);
  if (p.ir_mode == ORC_IR_EVOLVE) cs.eir[i] = rval(s.Eir);
  real T = isothermal ? Tiso : s.E / cv_of(p, c, s.y2, s.ye);
  real ratio = hminus_ratio(net, T);
  real yhm = ratio * s.ye;
  real yhp = s.ye + yhm;
  real yh = 1.0 - 2.0 * s.y2 - yhp - yhm;
  if (cs.y_h) cs.y_h[i] = rval(yh);
  if (cs.y_hp) cs.y_hp[i] = rval(yhp);
  if (cs.y_hm) cs.y_hm[i] = rval(yhm);
  if (cs.tgas) cs.tgas[i] = rval(T);
  if (cs.nsub) cs.nsub[i] = nsub;
  if (cs.niter) cs.niter[i] = nit;
  if (cs.flags) cs.flags[i] = fl;
  if (p.photon_absorb == 1 && (cs.n_euv_out || cs.n_fuv_out)) {
    real neuv, nfuv;
    absorb_photons(net, p, c, yh, dt, neuv, nfuv);
    if (cs.n_euv_out) cs.n_euv_out[i] = rval(neuv);
    if (cs.n_fuv_out) cs.n_fuv_out[i] = rval(nfuv);
  }
}

static void store_invalid(const orc_cells& cs, int64_t i) {
  const double nan = std::nan("");
  if (cs.y_h) cs.y_h[i] = nan;
  if (cs.y_hp) cs.y_hp[i] = nan;
  if (cs.y_hm) cs.y_hm[i] = nan;
  if (cs.tgas) cs.tgas[i] = nan;
  if (cs.nsub) cs.nsub[i] = 0;
  if (cs.niter) cs.niter[i] = 0;
  if (cs.flags) cs.flags[i] = ORC_F_INVALID;
  /* an invalid cell absorbs nothing */
  if (cs.n_euv_out) cs.n_euv_out[i] = cs.n_euv[i];
  if (cs.n_fuv_out) cs.n_fuv_out[i] = cs.n_fuv[i];
}

/* ------------------------------------------------------------------ */
/* LI update of one cell over dt.                                     */
static void li_cell(const orc_network& net, const orc_params& p, const orc_cells& cs, int64_t i,
                    double dt) {
  CellIn ci;
  State s;
  load(p, cs, i, ci, s);
  if (!input_ok(p, ci.nh, ci.neuv, ci.nfuv, ci.z, rval(s.y2), rval(s.ye), rval(s.E), rval(s.Td),
                rval(s.Eir))) {
    store_invalid(cs, i);
    return;
  }
  Cell c;
  make_cell(net, p, ci.nh, ci.neuv, ci.nfuv, ci.z, c);
  const bool iso = (p.thermal_mode == ORC_THERMAL_ISOTHERMAL);
  const bool dust_on = (p.dust_mode == ORC_DUST_EVOLVE) && !iso;
  const real Tiso = s.E / cv_of(p, c, s.y2, s.ye);

  uint32_t fl = renormalise(net, p, c, s, iso, Tiso);
  real rem = dt;
  int nsub = 0, nit = 0;
  bool tight = false;

  for (;;) {
    /* derived quantities at the substep start */
    real nt = ntot_rel(p, s.y2, s.ye);
    real cv = cv_of(p, c, s.y2, s.ye);
    real T = iso ? Tiso : s.E / cv;
    ChemOut co;
    chem(net, p, s.y2, s.ye, T, s.Td, c, co);

    /* timescales (written as inverse timescales, zero rate -> no limit) */
    real nu_dust = 0.0, qgg = 0.0;
    if (dust_on) {
      Dust d;
      dust_eval(net, p, T, s.Td, s.Eir, cv, c, d);
      qgg = c.rho * d.Sg; /* gas-grain exchange = -Lambda_14 [erg cm^-3 s^-1] */
      nu_dust = dust_rate(p, d, s.Td, T, s.Eir);
    }
    /* Reading: the number of subcycles the dust would need to cover the
     * rest of the interval, N_req = rem / (f_chem dt_dust), is re-estimated
     * at every subcycle; the dust is "tightly coupled" (implicit solve,
     * dust timescale dropped from the step size) while N_req >= N_cyc. */
    {
      real nreq = rem * nu_dust / p.f_chem;
      tight = dust_on && (nreq >= real(double(p.n_cyc)));
      if (tight) fl |= ORC_F_TIGHT;
    }
    real nu_chem = rmax(rabs(co.rh2.v) / rmax(s.y2, p.y_abs), rabs(co.re.v) / rmax(s.ye, p.y_abs));
    real nu = nu_chem;
    /* Eq. timescale_energy: |Gamma - Lambda| over all heating and cooling
     * processes, gas-grain exchange (Lambda_14) included */
    if (!iso) nu = rmax(nu, rabs(co.q.v + qgg) / s.E);
    if (!tight) nu = rmax(nu, nu_dust);

    real h;
    bool last = false;
    if (nu > real(0.0)) h = p.f_chem / nu; else h = rem;
    if (h >= rem) {
      h = rem;
      last = true;
    } else if (nsub >= p.n_sub_max / 2) {
      /* Reading (no bound in the paper): once half of the allowed n_sub_max
       * subcycles are used, the remaining ones share the rest of dt evenly
       * at least, so that every call ends within n_sub_max subcycles. */
      real hcap = rem / real(double(p.n_sub_max - nsub));
      if (h < hcap) {
        h = hcap;
        fl |= ORC_F_CAP;
        if (h >= rem) { h = rem; last = true; }
      }
    }

#ifdef ORC_DUST_FIRST
    /* measurement build (split-order study): the same Lie split in the
     * other order, the Appendix C step over h first, then the chemistry +
     * energy step with its coefficients taken again at the updated state */
    if (dust_on) {
      if (!tight) {
        dust_linear_step(net, p, c, s, h);
      } else {
        bool conv, floored;
        nit += dust_tight_step(net, p, c, s, h, conv, floored);
        if (!conv) fl |= ORC_F_NOCONV;
        if (floored) fl |= ORC_F_FLOOR;
      }
      fl |= dust_floors(p, c, s);
      nt = ntot_rel(p, s.y2, s.ye);
      cv = cv_of(p, c, s.y2, s.ye);
      T = iso ? Tiso : s.E / cv;
      chem(net, p, s.y2, s.ye, T, s.Td, c, co);
    }
#endif
    /* chemistry + energy: (I - h J) du = h f, u = (y_H2, y_e, E/E_ref) */
    {
      real Eref = s.E;
      real J[3][3], f[3];
      /* T = (gamma-1) E / (k_B n ntot): dT/dy_H2 = T/ntot, dT/dy_e = -T/ntot,
       * dT/dE = T/E */
      real dTdy2 = iso ? real(0.0) : T / nt;
      real dTdye = iso ? real(0.0) : -(T / nt);
      real dTdu3 = iso ? real(0.0) : T; /* (T/E) * E_ref with E = E_ref */
      const G3* rows[2] = {&co.rh2, &co.re};
      for (int r = 0; r < 2; ++r) {
        const G3& g = *rows[r];
        f[r] = g.v;
        J[r][0] = g.a + g.t * dTdy2;
        J[r][1] = g.e + g.t * dTdye;
        J[r][2] = g.t * dTdu3;
      }
      if (iso) {
        f[2] = 0.0;
        J[2][0] = 0.0;
        J[2][1] = 0.0;
        J[2][2] = 0.0;
      } else {
        f[2] = co.q.v / Eref;
        J[2][0] = (co.q.a + co.q.t * dTdy2) / Eref;
        J[2][1] = (co.q.e + co.q.t * dTdye) / Eref;
        J[2][2] = co.q.t * dTdu3 / Eref;
      }
#ifdef ORC_JAC32
      /* measurement build: partials of binary32 accuracy (mixed bar) */
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) J[r][k] = real(double(float(rval(J[r][k]))));
#endif
      real A[3][3], b[3], x[3] = {0.0, 0.0, 0.0};
      for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) A[r][k] = (r == k ? real(1.0) : real(0.0)) - h * J[r][k];
        b[r] = h * f[r];
      }
      lu_solve(3, A, b, x);
      s.y2 = s.y2 + x[0];
      s.ye = s.ye + x[1];
      if (!iso) s.E = s.E + x[2] * Eref;
    }
    fl |= renormalise(net, p, c, s, iso, Tiso);

#ifndef ORC_DUST_FIRST
    /* dust, IR and gas-grain exchange (Appendix C) */
    if (dust_on) {
      if (!tight) {
        dust_linear_step(net, p, c, s, h);
      } else {
        bool conv, floored;
        nit += dust_tight_step(net, p, c, s, h, conv, floored);
        if (!conv) fl |= ORC_F_NOCONV;
        if (floored) fl |= ORC_F_FLOOR;
      }
      fl |= dust_floors(p, c, s);
    }
#endif

    ++nsub;
    if (last) break;
    rem = rem - h;
  }
  store(net, p, cs, i, c, s, iso, Tiso, nsub, nit, fl, dt);
}

/* ------------------------------------------------------------------ */
/* Newton-Raphson fully implicit comparator.                          */
struct NRState {
  real y2, ye, T, Td, Eir;
};

/* group (ii): (T_d, E_IR) at fixed T_g */
static bool nr_dust(const orc_network& net, const orc_params& p, const Cell& c, const State& s0,
                    real dts, real T, real cv, real tol, real& Td, real& Eir, int& its) {
  const real ctil = p.c_red * C_LIGHT;
  const real ac = A_RAD * C_LIGHT;
  for (int it = 1; it <= 20; ++it) {
    ++its;
    Dust d;
    dust_eval(net, p, T, Td, Eir, cv, c, d);
    real td3 = Td * Td * Td;
    real F1 = p.dust_cap * (Td - s0.Td) - dts * d.Sd;
    real J11 = p.dust_cap + dts * (ac * td3 * d.betad + d.G * d.gd);
    real dTd, dE = 0.0;
    if (p.ir_mode == ORC_IR_EVOLVE) {
      real F2 = Eir - s0.Eir - dts * d.Sir;
      real J12 = -(dts * ctil * d.betair);
      real J21 = -(dts * c.rho * c.fd * ac * td3 * d.betad);
      real J22 = 1.0 + dts * c.rho * c.fd * ctil * d.betair;
      real det = J11 * J22 - J12 * J21;
      dTd = -(F1 * J22 - J12 * F2) / det;
      dE = -(J11 * F2 - J21 * F1) / det;
    } else {
      dTd = -F1 / J11;
    }
    real Tn = Td + dTd;
    bool ok = rabs(dTd) <= tol * rabs(Tn);
    if (Tn < real(0.5) * Td) { Tn = 0.5 * Td; ok = false; }
    if (Tn > real(2.0) * Td) { Tn = 2.0 * Td; ok = false; }
    real En = Eir;
    if (p.ir_mode == ORC_IR_EVOLVE) {
      En = Eir + dE;
      ok = ok && rabs(dE) <= tol * rabs(En);
      if (En < real(0.5) * Eir) { En = 0.5 * Eir; ok = false; }
      if (En > real(2.0) * Eir) { En = 2.0 * Eir; ok = false; }
    }
    Td = Tn;
    Eir = En;
    if (ok) return true;
  }
  return false;
}

/* group (iii): chemistry (y_H2, y_e) at fixed T_g, T_d */
static bool nr_chem(const orc_network& net, const orc_params& p, const Cell& c, const State& s0,
                    real dts, real T, real Td, real tol, real& y2, real& ye, int& its) {
  for (int it = 1; it <= 20; ++it) {
    ++its;
    ChemOut co;
    chem(net, p, y2, ye, T, Td, c, co);
    real F1 = y2 - s0.y2 - dts * co.rh2.v;
    real F2 = ye - s0.ye - dts * co.re.v;
    real J11 = 1.0 - dts * co.rh2.a, J12 = -(dts * co.rh2.e);
    real J21 = -(dts * co.re.a), J22 = 1.0 - dts * co.re.e;
    real det = J11 * J22 - J12 * J21;
    real d1 = -(F1 * J22 - J12 * F2) / det;
    real d2 = -(J11 * F2 - J21 * F1) / det;
    /* damped towards the bounds instead of clamped onto them, so that an
     * iterate never sits on a bound with a non-zero residual */
    real n1 = y2 + d1, n2 = ye + d2;
    /* converged when the (undamped) Newton correction is small */
    bool ok = rabs(d1) <= tol * rmax(rabs(n1), p.y_abs) && rabs(d2) <= tol * rmax(rabs(n2), p.y_abs);
    if (n1 < real(0.0)) { n1 = 0.1 * y2; ok = false; }
    if (n1 > real(0.5)) { n1 = 0.5 * (y2 + 0.5); ok = false; }
    if (n2 < real(0.0)) { n2 = 0.1 * ye; ok = false; }
    if (n2 > real(1.0)) { n2 = 0.5 * (ye + 1.0); ok = false; }
    y2 = n1;
    ye = n2;
    if (ok) return true;
  }
  return false;
}

/* inner solves at trial T; returns G(T) of the gas-energy equation */
static bool nr_inner(const orc_network& net, const orc_params& p, const Cell& c, const State& s0,
                     real dts, real T, real tol, bool dust_on, NRState& g, real& Gval, int& idust,
                     int& ichem) {
  real cv0 = cv_of(p, c, g.y2, g.ye);
  if (dust_on) {
    if (!nr_dust(net, p, c, s0, dts, T, cv0, tol, g.Td, g.Eir, idust)) return false;
  }
  if (!nr_chem(net, p, c, s0, dts, T, g.Td, tol, g.y2, g.ye, ichem)) return false;
  ChemOut co;
  chem(net, p, g.y2, g.ye, T, g.Td, c, co);
  real cv = cv_of(p, c, g.y2, g.ye);
  real gas_grain = 0.0;
  if (dust_on) {
    Dust d;
    dust_eval(net, p, T, g.Td, g.Eir, cv, c, d);
    gas_grain = c.rho * d.Sg;
  }
  Gval = cv * T - s0.E - dts * (co.q.v + gas_grain);
  return true;
}

static bool nr_substep_iter(const orc_network& net, const orc_params& p, const Cell& c,
                            State& s, real dts, bool iso, real Tiso, bool dust_on, int& outer,
                            int& idust, int& ichem) {
  State s0 = s;
  NRState g{s.y2, s.ye, iso ? Tiso : s.E / cv_of(p, c, s.y2, s.ye), s.Td, s.Eir};
  if (iso) {
    real Gv;
    if (!nr_inner(net, p, c, s0, dts, Tiso, 1e-5, dust_on, g, Gv, idust, ichem)) return false;
    s.y2 = g.y2;
    s.ye = g.ye;
    s.Td = g.Td;
    s.Eir = g.Eir;
    s.E = cv_of(p, c, s.y2, s.ye) * Tiso;
    outer += 1;
    return true;
  }
  real tol = 1e-5;
  for (int it = 1; it <= 20; ++it) {
    ++outer;
    if (it > 10) tol = 1e-3; /* relaxed after N_itr,limit / 2 */
    real T = g.T;
    real dl = 1e-4 * T;
    NRState gm = g, gc = g, gp = g;
    real Gm, Gc, Gp;
    if (!nr_inner(net, p, c, s0, dts, T - dl, tol, dust_on, gm, Gm, idust, ichem)) return false;
    if (!nr_inner(net, p, c, s0, dts, T, tol, dust_on, gc, Gc, idust, ichem)) return false;
    if (!nr_inner(net, p, c, s0, dts, T + dl, tol, dust_on, gp, Gp, idust, ichem)) return false;
    real dG = (Gp - Gm) / (2.0 * dl);
    real Tn = T - Gc / dG;
    bool limited = false;
    if (!(Tn > real(0.5) * T)) { Tn = 0.5 * T; limited = true; }
    if (!(Tn < real(2.0) * T)) { Tn = 2.0 * T; limited = true; }
    if (Tn < real(p.t_cmb)) { Tn = p.t_cmb; limited = true; }
    bool ok = !limited && rabs(Tn - T) <= tol * Tn && rabs(gc.y2 - g.y2) <= tol * rmax(gc.y2, p.y_abs) &&
              rabs(gc.ye - g.ye) <= tol * rmax(gc.ye, p.y_abs) &&
              rabs(gc.Td - g.Td) <= tol * gc.Td;
    g = gc;
    g.T = Tn;
    if (ok) {
      /* accept: inner solve at the converged T */
      real Gv;
      if (!nr_inner(net, p, c, s0, dts, Tn, tol, dust_on, g, Gv, idust, ichem)) return false;
      s.y2 = g.y2;
      s.ye = g.ye;
      s.Td = g.Td;
      s.Eir = g.Eir;
      s.E = cv_of(p, c, s.y2, s.ye) * Tn;
      return true;
    }
  }
  return false;
}

/* One substep; `iters` counts every Newton iteration: the outer ones and
 * the inner dust/IR and chemistry iterations (the count reported per cell,
 * so that equal counts mean the same convergence decisions). */
static bool nr_substep(const orc_network& net, const orc_params& p, const Cell& c, State& s,
                       real dts, bool iso, real Tiso, bool dust_on, int& iters) {
  int outer = 0, idust = 0, ichem = 0;
  const bool ok = nr_substep_iter(net, p, c, s, dts, iso, Tiso, dust_on, outer, idust, ichem);
  iters += outer + idust + ichem;
  return ok;
}

static void nr_cell(const orc_network& net, const orc_params& p, const orc_cells& cs, int64_t i,
                    double dt) {
  CellIn ci;
  State s;
  load(p, cs, i, ci, s);
  if (!input_ok(p, ci.nh, ci.neuv, ci.nfuv, ci.z, rval(s.y2), rval(s.ye), rval(s.E), rval(s.Td),
                rval(s.Eir))) {
    store_invalid(cs, i);
    return;
  }
  Cell c;
  make_cell(net, p, ci.nh, ci.neuv, ci.nfuv, ci.z, c);
  const bool iso = (p.thermal_mode == ORC_THERMAL_ISOTHERMAL);
  const bool dust_on = (p.dust_mode == ORC_DUST_EVOLVE) && !iso;
  const real Tiso = s.E / cv_of(p, c, s.y2, s.ye);
  uint32_t fl = renormalise(net, p, c, s, iso, Tiso);
  /* substeps, Eq. substep_NRchem: first try the whole interval; on failure
   * i <- i+1, on success i <- max(i-1, 0); dt_sub = (dt - t_sub)/2^i. */
  real tsub = 0.0;
  int lev = 0, nsub = 0, outer = 0, attempts = 0;
  for (;;) {
    real dts = (dt - tsub) / std::ldexp(1.0, lev);
    State trial = s;
    if (nr_substep(net, p, c, trial, dts, iso, Tiso, dust_on, outer)) {
      s = trial;
      ++nsub;
      if (lev == 0) break;
      tsub = tsub + dts;
      lev = lev > 0 ? lev - 1 : 0;
    } else {
      ++lev;
      if (lev > 60) {
        fl |= ORC_F_NRFAIL;
        break;
      }
    }
    /* Reading (no bound in the paper): at most n_sub_max substep attempts */
    if (++attempts >= p.n_sub_max) {
      fl |= ORC_F_NRFAIL;
      break;
    }
  }
  store(net, p, cs, i, c, s, iso, Tiso, nsub, outer, fl, dt);
}

/* ------------------------------------------------------------------ */
/* RK4 reference on the ODE dy_H2/dt = R_H2, dy_e/dt = R_e,            */
/* dE/dt = Q + rho S_g, dT_d/dt = S_d / C_d, dE_IR/dt = S_IR.           */
static void rk_rhs(const orc_network& net, const orc_params& p, const Cell& c, const State& s,
                   bool iso, real Tiso, bool dust_on, real out[5]) {
  real cv = cv_of(p, c, s.y2, s.ye);
  real T = iso ? Tiso : s.E / cv;
  ChemOut co;
  chem(net, p, s.y2, s.ye, T, s.Td, c, co);
  out[0] = co.rh2.v;
  out[1] = co.re.v;
  out[2] = iso ? real(0.0) : co.q.v;
  out[3] = 0.0;
  out[4] = 0.0;
  if (dust_on) {
    Dust d;
    dust_eval(net, p, T, s.Td, s.Eir, cv, c, d);
    out[2] = out[2] + c.rho * d.Sg;
    out[3] = d.Sd / p.dust_cap;
    if (p.ir_mode == ORC_IR_EVOLVE) out[4] = d.Sir;
  }
}

static void rk_cell(const orc_network& net, const orc_params& p, const orc_cells& cs, int64_t i,
                    double dt, double frac) {
  CellIn ci;
  State s;
  load(p, cs, i, ci, s);
  if (!input_ok(p, ci.nh, ci.neuv, ci.nfuv, ci.z, rval(s.y2), rval(s.ye), rval(s.E), rval(s.Td),
                rval(s.Eir))) {
    store_invalid(cs, i);
    return;
  }
  Cell c;
  make_cell(net, p, ci.nh, ci.neuv, ci.nfuv, ci.z, c);
  const bool iso = (p.thermal_mode == ORC_THERMAL_ISOTHERMAL);
  const bool dust_on = (p.dust_mode == ORC_DUST_EVOLVE) && !iso;
  const real Tiso = s.E / cv_of(p, c, s.y2, s.ye);
  uint32_t fl = renormalise(net, p, c, s, iso, Tiso);
  real t = 0.0;
  int nsub = 0;
  auto add = [](const State& a, const real* k, real w) {
    State r = a;
    r.y2 = a.y2 + w * k[0];
    r.ye = a.ye + w * k[1];
    r.E = a.E + w * k[2];
    r.Td = a.Td + w * k[3];
    r.Eir = a.Eir + w * k[4];
    return r;
  };
  while (t < real(dt)) {
    real k1[5], k2[5], k3[5], k4[5];
    rk_rhs(net, p, c, s, iso, Tiso, dust_on, k1);
    real nu = rmax(rabs(k1[0]) / rmax(s.y2, p.y_abs), rabs(k1[1]) / rmax(s.ye, p.y_abs));
    nu = rmax(nu, rabs(k1[2]) / s.E);
    nu = rmax(nu, rabs(k1[3]) / s.Td);
    nu = rmax(nu, rabs(k1[4]) / s.Eir);
    real h = nu > real(0.0) ? frac / nu : real(dt) - t;
    if (h > real(dt) - t) h = real(dt) - t;
    rk_rhs(net, p, c, add(s, k1, 0.5 * h), iso, Tiso, dust_on, k2);
    rk_rhs(net, p, c, add(s, k2, 0.5 * h), iso, Tiso, dust_on, k3);
    rk_rhs(net, p, c, add(s, k3, h), iso, Tiso, dust_on, k4);
    real kk[5];
    for (int j = 0; j < 5; ++j) kk[j] = (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]) / 6.0;
    s = add(s, kk, h);
    if (iso) s.E = cv_of(p, c, s.y2, s.ye) * Tiso;
    t = t + h;
    ++nsub;
  }
  store(net, p, cs, i, c, s, iso, Tiso, nsub, 0, fl, dt);
}

template <class F>
static void run_threads(int64_t n, int nthreads, F fn) {
  if (nthreads <= 1 || n < 2) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
    if (b >= e) break;
    th.emplace_back([=]() {
      for (int64_t i = b; i < e; ++i) fn(i);
    });
  }
  for (auto& x : th) x.join();
}

static bool cells_ok(const orc_params* p, const orc_cells* cs) {
  if (!cs || cs->n < 0) return false;
  if (cs->n == 0) return true;
  if (!cs->y_h2 || !cs->y_e || !cs->eint || !cs->tdust || !cs->nh || !cs->n_euv || !cs->n_fuv)
    return false;
  if (p->ir_mode == ORC_IR_EVOLVE && !cs->eir) return false;
  return true;
}

} /* namespace */

/* ------------------------------------------------------------------ */
extern "C" {

void orc_network_default(orc_network* net) {
  std::memset(net, 0, sizeof(*net));
  for (int i = 0; i < ORC_NREAC; ++i) net->reac_mult[i] = 1.0;
  for (int i = 0; i < ORC_NPROC; ++i) net->proc_mult[i] = 1.0;
  net->sigma_euv = 3.0e-18;
  net->k10_per_g0 = 5.0e-11;
  net->g0_photon_density = 3.7e-3;
  net->zeta_cr = 1.0e-17;
  net->k4_pre = 1.0e-10;
  net->k4_theta = 52000.0;
  net->heat_euv_ev = 4.4;
  net->heat_h2diss_ev = 0.4;
  net->pe_coef = 1.0e-24;
  net->pe_eps = 0.05;
  net->kappa_max = 20.0;
  net->kappa_tnorm = 200.0;
  net->kappa_uv = 400.0;
  net->e_fuv_ev = 9.0;
  net->e_euv_ev = 18.0;
  net->x_c = 1.4e-4;
  net->x_o = 3.2e-4;
  net->f_oiii = 0.2;
  const double tul[5] = {510.0, 91.2, 227.7, 38600.0, 29000.0};
  const double a[5] = {2.94e-11, 2.29e-6, 8.91e-5, 1.0e-4, 2.0e-2};
  const double g[5] = {5.0, 2.0, 0.6, 2.5, 5.0 / 9.0};
  const double qn[5] = {1.0e-11, 8.0e-10, 1.0e-10, 0.0, 0.0};
  const double qe[5] = {0.0, 2.8e-7, 1.4e-8, 8.629e-8, 1.7258e-7};
  for (int j = 0; j < 5; ++j) {
    net->line_tul[j] = tul[j];
    net->line_a[j] = a[j];
    net->line_g[j] = g[j];
    net->line_qn[j] = qn[j];
    net->line_qe100[j] = qe[j];
  }
  net->shield_len = 0.5;
  net->shield_b5 = 2.0;
  net->pe_mode = 0;
  net->shield_mode = 0;
}

void orc_params_default(orc_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->f_chem = 0.03;
  p->y_abs = 1e-10;
  p->newton_rtol = 1e-12;
  p->c_red = 1e-4;
  p->t_cmb = 2.73;
  p->y_he = 0.1;
  p->gamma_ad = 5.0 / 3.0;
  p->dust_cap = 1.0e4;
  p->z_default = 1.0;
  p->n_cyc = 300;
  p->n_sub_max = 100000;
  p->newton_max = 60;
  p->ir_mode = ORC_IR_EVOLVE;
  p->thermal_mode = ORC_THERMAL_EVOLVE;
  p->dust_mode = ORC_DUST_EVOLVE;
}

int orc_li_step(const orc_network* net, const orc_params* p, const orc_cells* cs, double dt,
                int nthreads) {
  if (!net || !p || !cells_ok(p, cs) || !(dt > 0.0) || !std::isfinite(dt)) return -1;
  run_threads(cs->n, nthreads, [&](int64_t i) { li_cell(*net, *p, *cs, i, dt); });
  return 0;
}

int orc_nr_step(const orc_network* net, const orc_params* p, const orc_cells* cs, double dt,
                int nthreads) {
  if (!net || !p || !cells_ok(p, cs) || !(dt > 0.0) || !std::isfinite(dt)) return -1;
  run_threads(cs->n, nthreads, [&](int64_t i) { nr_cell(*net, *p, *cs, i, dt); });
  return 0;
}

int orc_rk_reference(const orc_network* net, const orc_params* p, const orc_cells* cs, double dt,
                     double step_frac) {
  if (!net || !p || !cells_ok(p, cs) || !(dt > 0.0) || !(step_frac > 0.0)) return -1;
  for (int64_t i = 0; i < cs->n; ++i) rk_cell(*net, *p, *cs, i, dt, step_frac);
  return 0;
}

void orc_rate_coeffs(const orc_network* net, const orc_params* p, double T, double tdust,
                     double nh, double fd, double n_euv, double n_fuv, double* k, double* dk) {
  Cell c;
  make_cell(*net, *p, nh, n_euv, n_fuv, fd, c);
  Rates r;
  rates(*net, T, tdust, c, r);
  for (int i = 0; i < ORC_NREAC; ++i) {
    k[i] = rval(r.k[i]);
    dk[i] = rval(r.dk[i]);
  }
}

void orc_chem_sources(const orc_network* net, const orc_params* p, double y_h2, double y_e,
                      double T, double tdust, double nh, double fd, double n_euv, double n_fuv,
                      double* out, double* jac, double* terms) {
  Cell c;
  make_cell(*net, *p, nh, n_euv, n_fuv, fd, c);
  ChemOut co;
  chem(*net, *p, y_h2, y_e, T, tdust, c, co);
  const G3* g[3] = {&co.rh2, &co.re, &co.q};
  for (int i = 0; i < 3; ++i) {
    out[i] = rval(g[i]->v);
    jac[3 * i + 0] = rval(g[i]->a);
    jac[3 * i + 1] = rval(g[i]->e);
    jac[3 * i + 2] = rval(g[i]->t);
  }
  if (terms)
    for (int i = 0; i < ORC_NPROC; ++i) terms[i] = rval(co.terms[i]);
}

void orc_dust_system(const orc_network* net, const orc_params* p, double tg, double tdust,
                     double eir, double nh, double fd, double ntot, double n_euv, double n_fuv,
                     double h, double* A, double* rhs, double* src) {
  Cell c;
  make_cell(*net, *p, nh, n_euv, n_fuv, fd, c);
  real cv = K_B * c.n * ntot / (p->gamma_ad - 1.0);
  Dust d;
  dust_eval(*net, *p, tg, tdust, eir, cv, c, d);
  real M[3][3], b[3];
  dust_matrix(*p, d, c, tdust, tg, h, M, b);
  if (p->ir_mode != ORC_IR_EVOLVE) {
    M[0][1] = 0.0;
    M[1][0] = 0.0;
    M[1][1] = 1.0;
    M[1][2] = 0.0;
    M[2][1] = 0.0;
    b[1] = 0.0;
  }
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) A[3 * i + j] = rval(M[i][j]);
    rhs[i] = rval(b[i]);
  }
  src[0] = rval(d.Sd);
  src[1] = rval(d.Sir);
  src[2] = rval(d.Sg);
  src[3] = rval(d.alpha);
}

int orc_count_li_cell(const orc_network* net, const orc_params* p, const orc_cells* cs, int64_t i,
                      double dt, double* counts) {
#ifdef ORC_COUNT
  if (!net || !p || !cells_ok(p, cs) || i < 0 || i >= cs->n) return -1;
  orc_counts = OrcCounts{0, 0, 0, 0, 0, 0};
  li_cell(*net, *p, *cs, i, dt);
  counts[0] = orc_counts.add;
  counts[1] = orc_counts.mul;
  counts[2] = orc_counts.div;
  counts[3] = orc_counts.sqrt_;
  counts[4] = orc_counts.transc;
  counts[5] = orc_counts.cmp;
  return 0;
#else
  (void)net; (void)p; (void)cs; (void)i; (void)dt; (void)counts;
  return -1;
#endif
}

} /* extern "C" */
