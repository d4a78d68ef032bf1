// sfk.h -- internal interface between the host library (sfchem.cpp) and the
// gfx950 plain-step kernels (sfk_li.hip, with the per-lane code in
// sfk_lane.h).  Everything here is passed by value as the kernel argument
// block, so wave-uniform constants are read through the scalar cache into
// SGPRs.
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
  double sh_b5;         // Doppler parameter of the H2 self-shielding fit [km/s]
  double pe_ch, pe_cr;  // photoelectric heating and grain recombination prefactors / k_B
  int32_t pe_mode;      // 0 constant photoelectric efficiency, 1 grain charging
  int32_t shield_mode;  // 0 no H2 self-shielding, 1 local H2 column
};

struct Par {
  double f_chem, y_abs, newton_rtol, c_red, t_cmb, y_he, gm1;  // gm1 = gamma - 1
  double igm1;           // 1 / (gamma - 1)
  double cd;             // C_d [erg/g/K]
  double z_default;
  double hm_ratio_max;   // upper bound of y_H-/y_e = k_H2/k_H3 over the rate range
  double sh_k;           // H2 column / 5e14 cm^-2 = y_H2 sh_k sqrt(n_H T) (self-shielding)
  // per-call constants, formed on the host
  double inv_f_chem;     // 1 / f_chem
  double cr_a;           // c~ / a_r: T_IR^4 = cr_a E_IR
  double eir_min;        // a_r T_CMB^4 / c~: E_IR of FIXED IR and its floor
  double compton;        // Lambda_12 / (k_B n_e (T - T_CMB)) [1/s]
  double kir_fix, absir_fix, betair_fix;  // FIXED IR: kappa(T_CMB), kappa c a T_CMB^4, beta_IR
  int32_t n_cyc, n_sub_max, newton_max, ir_mode, thermal_mode, dust_mode;
  int32_t photon_absorb; // 1: attenuated photon densities written after the step
};

struct Cells {
  int64_t n;
  double *y_h2, *y_e, *eint, *tdust, *eir;
  double *y_h, *y_hp, *y_hm, *tgas;
  const double *nh, *n_euv, *n_fuv, *zmet;
  int32_t *nsub, *niter;
  uint32_t *flags;
  double *n_euv_out, *n_fuv_out;  // photon densities after absorption (optional)
};

// Cells suspended by the first pass of two-phase dispatch, one slot each
// (slots handed out in suspension order; capacity = the call's cell count).
struct Suspended {
  unsigned long long* count;  // slots used
  int32_t* cell;              // cell index per slot
  double *rem, *tiso;         // remaining time of the interval, isothermal T
  int32_t *nsub, *nit;        // counters so far
  uint32_t* fl;               // flags so far
  int32_t* bucket;            // estimated-cost bucket per slot, written at suspension
};

struct Args {
  Net net;
  Par par;
  Cells c;
  double dt;
  unsigned long long* counter;  // work counter, zero at launch
  int32_t refill_min;           // refill a wave once this many lanes are idle
  const Net* netc;              // device copies of net and par (read-only)
  const Par* parc;
  const int32_t* order;         // lane work item -> cell (null: identity)
  const uint32_t* dense;        // length of the density-ordered head of order (null: 0)
  // Two-phase dispatch.  budget > 0: a cell not done after `budget`
  // subcycles is suspended (its state written back in place, the rest into
  // sus) and the lane takes another cell.  resume: work items are slots of
  // sus, taken through order, and each continues exactly where it stopped.
  int32_t budget;
  const uint32_t* budget_dev;        // if set, the budget read on the device instead
  int32_t resume;
  int32_t fine;                      // claim per refill only what idle lanes take, everywhere
  const unsigned long long* limit;   // number of work items, on the device (null: c.n)
  Suspended sus;
};

// host-callable launchers (defined in sfk_li.hip)
// True when the network switches on a piece beside the solver (H2
// self-shielding or the grain-charge photoelectric heating).  Those pieces
// are compiled into separate kernel instantiations, so that the default
// kernels carry none of their code and none of their register pressure;
// the launches pick the instantiation from the network.
inline bool stand_ins(const Net& n) { return n.shield_mode == 1 || n.pe_mode == 1; }

hipError_t launch_step(const Args& a, int precision, int grid, hipStream_t s);
hipError_t launch_step_nr(const Args& a, int grid, hipStream_t s);  // binary64 NR comparator
hipError_t launch_reset(unsigned long long* counter, hipStream_t s);
int max_blocks_per_cu(int precision, bool stand_ins);  // 0 LI binary64, 1 LI mixed, 2 NR
// Density dispatch: order[0..n) = the densest quarter of the cells (all of
// them with all_dense) by decreasing half-octave of n_H, then the rest in
// index order (n < 2^31; work holds kOrderWork uint32 counters).
constexpr int kOrderBuckets = 128;
constexpr int kOrderBlocks = 1024;
constexpr int kOrderWork = 2 * kOrderBuckets + 4 + 2 * kOrderBlocks;
constexpr int kOrderDenseWord = 2 * kOrderBuckets + 1;  // plan[1]: length of the dense head
constexpr int kOrderBudgetWord = 2 * kOrderBuckets + 2;  // plan[2]: first-pass budget (progress)
// With all_dense (the first pass of progress dispatch) the plan also
// writes the first pass's suspension budget into work[kOrderBudgetWord]:
// `budget` when at least `lanes` cells have n_H >= 1e6 cm^-3, else 0.
hipError_t launch_order(const double* nh, int64_t n, bool all_dense, int32_t* order,
                        uint32_t* work, hipStream_t s, int64_t lanes = 0, int32_t budget = 0);
// Two-phase dispatch, second phase: order[0..*sus.count) = the suspended
// slots, longest estimated remainder first (cap = slot capacity; each
// slot's cost bucket was written when its cell was suspended).
hipError_t launch_progress_order(const Suspended& sus, int64_t cap, uint32_t* work,
                                 int32_t* order, hipStream_t s);

constexpr int kBlock = 256;

}  // namespace sfk
