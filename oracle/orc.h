/*
 * orc.h -- CPU reference ("oracle") for the linearized-implicit (LI)
 * thermochemistry update of SFUMATO# (arXiv 2604.21438).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this library: only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with
 * the HIP implementation; both are written independently from the paper.
 *
 * Plain serial C++ in double precision, built with -O2 -ffp-contract=off and
 * no fast-math, so that every operation is a correctly rounded IEEE-754
 * binary64 operation in program order.
 *
 * What is computed (paper sections cited in orc_chem.cpp):
 *   orc_li_step      LI subcycled update: chemistry + gas energy as one 3x3
 *                    linearised system (Sec. "Thermochemical processes",
 *                    Eq. eq_deq), dust / IR / gas-grain exchange with the
 *                    pseudo dust heat capacity (Appendix C), subcycle step
 *                    size (Eqs. timescale_of_dust .. timestep_subcycle).
 *   orc_nr_step      Newton-Raphson fully implicit comparator (three nested
 *                    iteration groups, substep halving, Eq. substep_NRchem).
 *   orc_rk_reference Classical RK4 on the same ODE with a tiny step: the
 *                    "fine explicit integration" used for the convergence pin.
 *
 * Parity status per function is listed in the header comment of orc_chem.cpp.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_NREAC = 12, ORC_NPROC = 14, ORC_NLINE = 5 };

/* Reaction network and the labelled stand-ins for the formulas that the
 * paper leaves to its references.  reac_mult[i] scales k_Hi (i = 0..11);
 * proc_mult[p-1] scales thermal process p (1..4 heating Gamma_p, 5..14
 * cooling Lambda_p; 14 is the gas-grain coupling used in the dust system). */
typedef struct {
  double reac_mult[ORC_NREAC];
  double proc_mult[ORC_NPROC];
  double sigma_euv;          /* H photoionisation cross section [cm^2]      */
  double k10_per_g0;         /* H2 photodissociation rate per unit G0 [1/s] */
  double g0_photon_density;  /* FUV photon density of G0 = 1 [cm^-3]        */
  double zeta_cr;            /* cosmic-ray ionisation rate [1/s]            */
  double k4_pre, k4_theta;   /* k_H4 = k4_pre exp(-k4_theta/T)              */
  double heat_euv_ev;        /* heat per photoionisation [eV]               */
  double heat_h2diss_ev;     /* heat per photodissociation [eV]             */
  double pe_coef, pe_eps;    /* photoelectric: pe_coef*pe_eps*G0*n*f_d      */
  double kappa_max, kappa_tnorm; /* kappa(T)=kappa_max x^2/(1+x^2), x=T/tnorm */
  double kappa_uv;           /* UV dust opacity per gram of gas [cm^2/g]    */
  double e_fuv_ev, e_euv_ev; /* mean photon energies [eV]                   */
  double x_c, x_o, f_oiii;   /* C, O abundances at Z_sun; O III share of O+ */
  /* two-level coolants: 0 H2, 1 C II, 2 O I, 3 O II, 4 O III */
  double line_tul[ORC_NLINE];   /* Delta E / k_B [K]                        */
  double line_a[ORC_NLINE];     /* A_ul [1/s]                               */
  double line_g[ORC_NLINE];     /* g_u / g_l                                */
  double line_qn[ORC_NLINE];    /* de-excitation by H + H2 [cm^3/s]         */
  double line_qe100[ORC_NLINE]; /* de-excitation by e at 100 K [cm^3/s], ~T^-1/2 */
  /* The pieces the paper takes from its references beside the solver
   * (H2 self-shielding and photoelectric heating with grain charging, the
   * text after Table "Thermal processes"); STAND-INS, off by default. */
  double shield_len;  /* H2 column length in Jeans lengths (shield_mode 1) */
  double shield_b5;   /* Doppler parameter of the self-shielding fit [km/s] */
  int32_t pe_mode;    /* 0: constant efficiency; 1: grain-charge efficiency
                         and recombination cooling                          */
  int32_t shield_mode;/* 0: no self-shielding; 1: local H2 column          */
} orc_network;

enum { ORC_IR_FIXED = 0, ORC_IR_EVOLVE = 1 };
enum { ORC_THERMAL_EVOLVE = 0, ORC_THERMAL_ISOTHERMAL = 1 };
enum { ORC_DUST_EVOLVE = 0, ORC_DUST_FROZEN = 1 };

typedef struct {
  double f_chem;       /* subcycle fraction                      [0.03]  */
  double y_abs;        /* abundance floor in Delta t_chem        [1e-10] */
  double newton_rtol;  /* tight-case dust Newton tolerance       [1e-12] */
  double c_red;        /* reduced speed of light c~/c            [1e-4]  */
  double t_cmb;        /* CMB temperature = temperature floor    [2.73]  */
  double y_he;         /* helium abundance by number             [0.1]   */
  double gamma_ad;     /* adiabatic index                        [5/3]   */
  double dust_cap;     /* pseudo dust heat capacity C_d [erg/g/K][1e4]   */
  double z_default;    /* metallicity used when zmet == NULL     [1]     */
  int32_t n_cyc;       /* subcycle limit deciding "tight"        [300]   */
  int32_t n_sub_max;   /* hard cap on subcycles per call         [100000]*/
  int32_t newton_max;  /* tight-case Newton iteration cap        [60]    */
  int32_t ir_mode;     /* ORC_IR_FIXED / ORC_IR_EVOLVE          [EVOLVE] */
  int32_t thermal_mode;/* ORC_THERMAL_*                          [EVOLVE]*/
  int32_t dust_mode;   /* ORC_DUST_*                             [EVOLVE]*/
  int32_t photon_absorb; /* 1: attenuate N_EUV, N_FUV over dt after the
                            update (Sec. 2 "Radiation components")   [0]  */
  int32_t reserved;
} orc_params;

/* Host structure-of-arrays cell buffers, all of length n.  In/out arrays
 * are overwritten; optional arrays may be NULL. */
typedef struct {
  int64_t n;
  double *y_h2, *y_e, *eint, *tdust, *eir;  /* in/out (eir: EVOLVE only)   */
  double *y_h, *y_hp, *y_hm, *tgas;         /* out, optional               */
  const double *nh, *n_euv, *n_fuv, *zmet;  /* in; zmet optional           */
  int32_t *nsub, *niter;                    /* out, optional               */
  uint32_t *flags;                          /* out, optional               */
  double *n_euv_out, *n_fuv_out;            /* out, optional (photon_absorb) */
} orc_cells;

/* per-cell flag bits */
enum {
  ORC_F_CAP = 1u << 0,      /* step raised by the n_sub_max cap           */
  ORC_F_TIGHT = 1u << 1,    /* dust handled by the implicit scalar solve  */
  ORC_F_NOCONV = 1u << 2,   /* tight Newton hit newton_max                */
  ORC_F_INVALID = 1u << 3,  /* non-finite / non-positive input: unchanged */
  ORC_F_FLOOR = 1u << 4,    /* a floor, clamp or rescale was applied      */
  ORC_F_NRFAIL = 1u << 5    /* NR comparator: substep limit reached       */
};

void orc_network_default(orc_network* net);
void orc_params_default(orc_params* p);

/* LI update of every cell over dt seconds; nthreads >= 1 splits the cells
 * statically over host threads.  Returns 0, or -1 on bad arguments. */
int orc_li_step(const orc_network* net, const orc_params* p,
                const orc_cells* cells, double dt, int nthreads);

/* Newton-Raphson fully implicit comparator over dt. */
int orc_nr_step(const orc_network* net, const orc_params* p,
                const orc_cells* cells, double dt, int nthreads);

/* RK4 reference: step = step_frac / (fastest inverse timescale). */
int orc_rk_reference(const orc_network* net, const orc_params* p,
                     const orc_cells* cells, double dt, double step_frac);

/* ---- pieces exposed for the pins in tests/ ---- */

/* k[i] = k_Hi(T, T_d) and dk[i] = d k_Hi / d T (at fixed T_d) for
 * i = 0..8; k[9..11] are the photo / CR rates of the cell (dk = 0). */
void orc_rate_coeffs(const orc_network* net, const orc_params* p, double T,
                     double tdust, double nh, double fd, double n_euv,
                     double n_fuv, double* k, double* dk);

/* Chemistry + heating/cooling sources at (y_H2, y_e, T) with T_d frozen:
 * out[0..2] = (R_H2, R_e, Q);  jac[3*i + j] = d out[i] / d (y_H2, y_e, T)[j].
 * terms[0..12] = Gamma_1..Gamma_4, Lambda_5..Lambda_13 (erg cm^-3 s^-1);
 * terms[13] = cooling by electron recombination on grains (pe_mode 1, else
 * 0; the gas-grain exchange Lambda_14 lives in the dust system). */
void orc_chem_sources(const orc_network* net, const orc_params* p,
                      double y_h2, double y_e, double T, double tdust,
                      double nh, double fd, double n_euv, double n_fuv,
                      double* out, double* jac, double* terms);

/* Appendix-C dust / IR / gas-grain linear system for one subcycle h:
 * A (row-major, 3x3 over (dT_d, dE_IR, dT_g); in FIXED IR mode the E_IR
 * row/column is the identity and rhs 0) and rhs; src = (S_d, S_IR, S_g,
 * alpha_g). */
void orc_dust_system(const orc_network* net, const orc_params* p, double tg,
                     double tdust, double eir, double nh, double fd,
                     double ntot_rel, double n_euv, double n_fuv, double h,
                     double* A, double* rhs, double* src);

/* Operation counts of orc_li_step for one cell: filled only by the counting
 * build (liborc_count.so); counts[0..5] = add/sub, mul, div, sqrt,
 * transcendental (exp/log/log1p), comparisons. Returns 0 in the counting
 * build, -1 in the plain build. */
int orc_count_li_cell(const orc_network* net, const orc_params* p,
                      const orc_cells* cells, int64_t i, double dt,
                      double* counts);

#ifdef __cplusplus
}
#endif
#endif
