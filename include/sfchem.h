/*
 * sfchem.h -- C ABI of the MI355X (gfx950) thermochemistry library.
 *
 * The library advances, cell by cell, the non-equilibrium hydrogen chemistry
 * (H, H2, H+, H-, e-), the gas internal energy and the dust temperature of
 * SFUMATO# (arXiv 2604.21438) over a hydrodynamic time step, with the
 * paper's linearized-implicit (LI) method:
 *   - chemistry and gas energy as one linearised implicit system
 *     (I - h J) du = h f, u = (y_H2, y_e, E_th)  (Sec. "Thermochemical
 *     processes", Eq. eq_deq; only y_H2 and y_e are unknowns, y_H and y_H+
 *     follow from H-nuclei and charge conservation);
 *   - dust temperature carried by a pseudo heat capacity C_d together with
 *     the IR energy density and the gas-grain exchange (Appendix C);
 *   - adaptive subcycles h = f_chem * min(dt_dust, dt_chem, dt_energy)
 *     (Eqs. timescale_of_dust .. timestep_subcycle, N_cyc = 300).
 * The rate coefficients are those of Table "Chemical reactions", the
 * heating and cooling those of Table "Thermal processes"; formulas the
 * paper leaves to its references are replaced by labelled stand-ins whose
 * constants are fields of sfc_network.
 *
 * Conventions.  Every entry point returns an int status (SFC_OK == 0, or a
 * negative SFC_E_* code); nothing throws or aborts across the ABI.  Cell
 * buffers are structure-of-arrays of length n, contiguous, in DEVICE memory
 * of the context's device, owned by the caller.  Units are cgs: densities
 * cm^-3, energies erg cm^-3, temperatures K, times s.
 */
#ifndef SFCHEM_H
#define SFCHEM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Version of sfc_network and sfc_params (both checked through
 * sfc_network.abi_version). */
#define SFC_ABI_VERSION 4u

enum {
  SFC_OK = 0,
  SFC_E_INVAL = -1,   /* bad argument (NULL, size, range, mode)           */
  SFC_E_NOMEM = -2,   /* host or device allocation failed                  */
  SFC_E_BUDGET = -3,  /* request larger than the whole served HBM budget   */
  SFC_E_DEVICE = -4,  /* HIP runtime error (message in sfc_last_error)     */
  SFC_E_PENDING = -5, /* sfc_chem_poll: request not finished yet           */
  SFC_E_VERSION = -6, /* sfc_network.abi_version / size mismatch           */
  SFC_E_STATE = -7    /* call not valid in the context's current state     */
};

typedef enum { SFC_FP64 = 0, SFC_MIXED = 1 } sfc_precision;
typedef enum { SFC_IR_FIXED = 0, SFC_IR_EVOLVE = 1 } sfc_ir_mode;
typedef enum { SFC_THERMAL_EVOLVE = 0, SFC_THERMAL_ISOTHERMAL = 1 } sfc_thermal_mode;
typedef enum { SFC_DUST_EVOLVE = 0, SFC_DUST_FROZEN = 1 } sfc_dust_mode;
/* Order in which the plain step hands cells to GPU lanes (scheduling only;
 * every cell's result is bitwise the same in all three).
 *   INDEX     cells in index order.
 *   DENSITY   the densest cells first: their stiffer chemistry and
 *             gas-grain coupling need the most subcycles, and starting them
 *             early keeps them off the end of the call.
 *   PROGRESS  two passes.  The first runs every cell (densest first) for
 *             at most sfc_params.phase_nsub subcycles; a cell still running
 *             then is suspended (its state written back in place, the rest
 *             of it kept by the context).  The second resumes the suspended
 *             cells, longest estimated remainder first, the estimate being
 *             the subcycles still needed at the larger of the cell's average
 *             pace so far and the pace of its last subcycle.  Cells that
 *             cost ~1e5 subcycles then start first instead of wherever
 *             density puts them.  On calls of more than two cells per GPU
 *             lane the first pass suspends only when the cells with n_H >=
 *             1e6 cm^-3 (the long ones) outnumber the lanes; with fewer it
 *             runs every cell to its end, as density order does.  Uses 36 B of context-owned device memory
 *             per cell (allocated at the first call that needs more).
 *   NR comparator calls (sfc_chem_step_nr) use DENSITY under PROGRESS. */
typedef enum {
  SFC_DISPATCH_INDEX = 0,
  SFC_DISPATCH_DENSITY = 1,
  SFC_DISPATCH_PROGRESS = 2
} sfc_dispatch;

enum { SFC_NREAC = 12, SFC_NPROC = 14, SFC_NLINE = 5 };

/* Reaction network and stand-in constants (copied at sfc_chem_init).
 * reac_mult[i] scales k_Hi, i = 0..11 (Table "Chemical reactions");
 * proc_mult[p-1] scales thermal process p = 1..14 (Table "Thermal
 * processes"; 14 is the gas-grain exchange of Appendix C).  Fill with
 * sfc_network_default() and edit. */
typedef struct {
  uint32_t abi_version;          /* = SFC_ABI_VERSION                       */
  uint32_t size;                 /* = sizeof(sfc_network)                   */
  double reac_mult[SFC_NREAC];
  double proc_mult[SFC_NPROC];
  double sigma_euv;              /* photoionisation cross section [cm^2]    */
  double k10_per_g0;             /* H2 photodissociation per G0 [1/s]       */
  double g0_photon_density;      /* FUV photons of G0 = 1 [cm^-3]           */
  double zeta_cr;                /* cosmic-ray ionisation [1/s]             */
  double k4_pre, k4_theta;       /* k_H4 = k4_pre exp(-k4_theta / T)        */
  double heat_euv_ev;            /* heat per photoionisation [eV]           */
  double heat_h2diss_ev;         /* heat per photodissociation [eV]         */
  double pe_coef, pe_eps;        /* photoelectric heating pe_coef*pe_eps*G0*n*Z */
  double kappa_max, kappa_tnorm; /* dust opacity kappa_max x^2/(1+x^2), x = T/tnorm */
  double kappa_uv;               /* dust UV opacity per gram of gas [cm^2/g] */
  double e_fuv_ev, e_euv_ev;     /* mean FUV / EUV photon energies [eV]     */
  double x_c, x_o, f_oiii;       /* C, O abundances at Z_sun; O III share of ionised O */
  double line_tul[SFC_NLINE];    /* two-level coolants H2, C II, O I, O II, O III: */
  double line_a[SFC_NLINE];      /*   Delta E/k_B [K], A_ul [1/s], g_u/g_l, */
  double line_g[SFC_NLINE];      /*   de-excitation by H+H2 [cm^3/s] and by */
  double line_qn[SFC_NLINE];     /*   electrons at 100 K [cm^3/s] (~T^-1/2) */
  double line_qe100[SFC_NLINE];
  /* Beside the solver (the paper takes these from its references; text
   * after Table "Thermal processes"), labelled stand-ins, off by default:
   * pe_mode 1: photoelectric efficiency with grain charging, psi =
   *   G0 sqrt(T) / n_e, eps = 0.0487 / (1 + 4e-3 psi^0.73) + 0.0365
   *   (T/1e4)^0.7 / (1 + 2e-4 psi), Gamma_pe = 1.3e-24 eps G0 n_H Z, and
   *   the cooling by electron recombination on grains 4.65e-30 T^0.94
   *   psi^beta n_e n_H Z, beta = 0.735 T^-0.068 (n_e floored at y_abs n_H
   *   inside psi; both scaled by proc_mult[3]);
   * shield_mode 1: H2 photodissociation times the self-shielding factor
   *   0.965 / (1 + x/b5)^2 + 0.035 / sqrt(1 + x) exp(-8.5e-4 sqrt(1 + x)),
   *   x = N_H2 / 5e14 cm^-2 with N_H2 = y_H2 n_H L, L = shield_len Jeans
   *   lengths sqrt(pi k_B T / (G m_H rho)). */
  double shield_len;             /* column length in Jeans lengths [0.5]   */
  double shield_b5;              /* Doppler parameter [km/s] [2]           */
  int32_t pe_mode;               /* [0]                                    */
  int32_t shield_mode;           /* [0]                                    */
} sfc_network;

/* Numerical and physical parameters; defaults in brackets. */
typedef struct {
  double f_chem;       /* subcycle fraction [0.03]                        */
  double y_abs;        /* abundance floor of dt_chem [1e-10]              */
  double newton_rtol;  /* tight dust solve tolerance [1e-12]              */
  double c_red;        /* reduced speed of light c~/c [1e-4]              */
  double t_cmb;        /* CMB temperature, also the temperature floor [2.73] */
  double y_he;         /* helium abundance by number [0.1]                */
  double gamma_ad;     /* adiabatic index [5/3]                           */
  int32_t n_cyc;       /* subcycle limit deciding tight coupling [300]    */
  int32_t n_sub_max;   /* hard cap on subcycles per call [100000]         */
  int32_t newton_max;  /* tight dust Newton iteration cap [60]            */
  int32_t ir_mode;     /* sfc_ir_mode [SFC_IR_EVOLVE]                     */
  int32_t thermal_mode;/* sfc_thermal_mode [SFC_THERMAL_EVOLVE]           */
  int32_t dust_mode;   /* sfc_dust_mode [SFC_DUST_EVOLVE]                 */
  int32_t dispatch;    /* sfc_dispatch [SFC_DISPATCH_PROGRESS]            */
  int32_t phase_nsub;  /* PROGRESS: subcycles of the first pass, >= 1 [4096] */
  int32_t photon_absorb; /* 1: after the update, the EUV and FUV photon
                          densities absorbed over dt are written to
                          sfc_cells.n_euv_out / n_fuv_out (plain path and
                          served form; the served arena then holds two more
                          float64 arrays, 16 B per cell):
                          N exp(-c~ alpha dt), alpha_EUV = sigma_EUV n_H y_H
                          + kappa_UV rho Z, alpha_FUV = kappa_UV rho Z, with
                          the updated y_H (Sec. 2 "Radiation components")
                          [0] */
  int32_t reserved;    /* must be 0 */
} sfc_params;

void sfc_network_default(sfc_network* net);
void sfc_params_default(sfc_params* p);

typedef struct sfc_ctx sfc_ctx; /* opaque, owned by the library */

/* Create a context on HIP device `hip_device`.
 *   net              reaction network (copied); NULL -> defaults.
 *   z_default        metallicity [Z_sun] used where sfc_cells.zmet is NULL.
 *   dust_cap_factor  pseudo dust heat capacity C_d = factor * 1e4 erg/g/K
 *                    (1 = the realistic value at Z_sun; the paper
 *                    recommends 1000), must be > 0.
 *   p                parameters (copied); NULL -> defaults.
 *   served_budget_bytes  device memory the served form may hold for
 *                    request state (0 -> served form disabled).
 * Errors: SFC_E_INVAL, SFC_E_VERSION, SFC_E_DEVICE, SFC_E_NOMEM. */
int sfc_chem_init(const sfc_network* net, double z_default, double dust_cap_factor,
                  const sfc_params* p, int hip_device, uint64_t served_budget_bytes,
                  sfc_ctx** out);

/* Device SoA cell buffers, length n, float64 unless noted.
 *   in/out: y_h2, y_e (abundances per H nucleus), eint (gas internal energy
 *           density), tdust, eir (IR energy density; required only in
 *           SFC_IR_EVOLVE mode, else may be NULL).
 *   out (optional, NULL to skip): y_h, y_hp, y_hm (derived abundances),
 *           tgas (gas temperature), nsub (int32 subcycles), niter (int32
 *           tight-dust Newton iterations), flags (uint32, SFC_F_* bits).
 *   in: nh (H nuclei density), n_euv, n_fuv (photon number densities),
 *       zmet (metallicity; NULL -> z_default).
 * A cell whose inputs are non-finite or non-positive (n_euv, n_fuv, zmet,
 * y_h2, y_e may be zero) is left unchanged, its derived outputs are NaN and
 * SFC_F_INVALID is set. */
typedef struct {
  int64_t n;
  double *y_h2, *y_e, *eint, *tdust, *eir;
  double *y_h, *y_hp, *y_hm, *tgas;
  const double *nh, *n_euv, *n_fuv, *zmet;
  int32_t *nsub, *niter;
  uint32_t *flags;
  double *n_euv_out, *n_fuv_out; /* out (optional; sfc_params.photon_absorb,
                                    plain path only; an invalid cell copies
                                    its inputs) */
} sfc_cells;

enum {
  SFC_F_CAP = 1u << 0,     /* a step was raised by the n_sub_max cap     */
  SFC_F_TIGHT = 1u << 1,   /* some subcycle used the implicit dust solve */
  SFC_F_NOCONV = 1u << 2,  /* that solve reached newton_max              */
  SFC_F_INVALID = 1u << 3, /* invalid input, cell unchanged              */
  SFC_F_FLOOR = 1u << 4,   /* a floor, clamp or rescale was applied      */
  SFC_F_NRFAIL = 1u << 5   /* NR comparator: a substep could not be made
                              to converge (after 60 halvings or n_sub_max
                              attempts); the cell keeps its last state    */
};

/* Advance every cell by dt_seconds (> 0, finite) on `hip_stream` (a
 * hipStream_t; NULL = default stream).  Asynchronous: returns after the
 * launches are queued; buffers must stay valid until the stream reaches the
 * end of the call.  n == 0 is a no-op.  precision: SFC_FP64 (everything in
 * binary64) or SFC_MIXED (rates, heating/cooling and Jacobian assembly in
 * binary32; LU solves, state update and renormalisation in binary64).
 * Calls on one context must not overlap (the context owns one work
 * counter); use one context per concurrent stream.
 * The call launches kernels only (no memset, no host synchronisation) and
 * can be captured into a HIP graph, with one condition: the first call of
 * a context with more cells than any before allocates the dispatch buffers
 * (hipMalloc, about 40 B per cell), so make one uncaptured call of at
 * least the captured size first.
 * Errors: SFC_E_INVAL, SFC_E_NOMEM, SFC_E_DEVICE. */
int sfc_chem_step(sfc_ctx* ctx, const sfc_cells* cells, double dt_seconds, int precision,
                  void* hip_stream);

/* Fully implicit Newton-Raphson comparator (the paper's Sec. 2 scheme that
 * the LI update replaces; validation and timing only): every cell is
 * advanced over dt_seconds by backward-Euler substeps of (y_H2, y_e, T_g,
 * T_d, E_IR), each solved by an outer Newton iteration on T_g (central
 * difference, step 1e-4 T_g) around the dust/IR and chemistry groups,
 * tolerance 1e-5 relaxed to 1e-3 after 10 outer iterations, 20 iterations
 * per loop; a substep that fails is halved (Eq. substep_NRchem).  Binary64.
 * Same buffers, ownership and asynchrony as sfc_chem_step; nsub receives
 * the accepted substeps, niter every Newton iteration (outer, dust/IR and
 * chemistry, failed substeps included), flags SFC_F_NRFAIL
 * for a cell that could not finish.  C_d is the context's (the paper runs
 * NR with the realistic value).
 * Errors: SFC_E_INVAL, SFC_E_NOMEM, SFC_E_DEVICE. */
int sfc_chem_step_nr(sfc_ctx* ctx, const sfc_cells* cells, double dt_seconds, void* hip_stream);

/* sfc_chem_step for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results (bitwise), asynchrony and errors as
 * sfc_chem_step, but the call allocates nothing: the dispatch buffers of
 * the call (work counter, cell order, suspended-cell slots; ~40 B per cell)
 * live in a file-scope device array of the library, one per GPU (80 MiB,
 * held until the process ends), so n is limited to SFC_NOALLOC_MAX_CELLS;
 * larger n returns SFC_E_INVAL.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other contexts,
 * other threads) race and must not be issued; calls in stream order are
 * fine.  The array needs no clearing between calls (the call's kernels
 * reset what they count with).  SFC_E_DEVICE if the array's device address
 * could not be taken when the context was created. */
#define SFC_NOALLOC_MAX_CELLS 2097152
int sfc_chem_step_noalloc(sfc_ctx* ctx, const sfc_cells* cells, double dt_seconds,
                          int precision, void* hip_stream);

/* ---- served form: continuous batching of AMR blocks ---- */

/* One request: a set of cells (typically whole 8^3 blocks) with its own dt
 * (the AMR substep of its level, Eqs. timestep and timestep2 of the paper).
 *
 * Without a block key (block_key == 0) the request's cells are copied from
 * the caller's buffers into the library's arena when it is admitted, and
 * its results are copied back into the same buffers when it completes; the
 * buffers must stay valid until sfc_chem_poll returns SFC_OK.
 *
 * With a block key the block's state stays resident in the arena between
 * requests, as AMR substeps of one block follow each other:
 *   - a request without SFC_REQ_RESUME uploads `cells` into the key's range
 *     (the first substep, or a restart); the key keeps its cell count;
 *   - a request with SFC_REQ_RESUME continues from the state the key's
 *     previous request left (and its inputs n_H, photon densities, Z): no
 *     copy-in, `cells` is not read (cells.n may be 0 or the key's count);
 *   - results stay in the arena: sfc_chem_fetch copies them out, and
 *     SFC_REQ_WRITEBACK also copies them into `cells` at completion;
 *   - the key's requests run one after the other in submission order; a
 *     request may be submitted before its predecessor is done;
 *   - the key holds its arena range until sfc_chem_release.
 * hip_stream, if not NULL, is the stream that produced the input buffers:
 * the library's copy-in waits for the work queued on it before the submit
 * call (otherwise the caller must have completed that work first). */
enum {
  SFC_REQ_RESUME = 1u << 0,    /* continue from the block key's resident state */
  SFC_REQ_WRITEBACK = 1u << 1  /* keyed request: also copy results into cells */
};

typedef struct {
  sfc_cells cells;
  double dt_seconds;
  int32_t level;       /* AMR level: claim priority (see submit)  */
  int32_t precision;   /* SFC_FP64 or SFC_MIXED                   */
  uint64_t tag;        /* caller's tag, returned in sfc_result    */
  uint64_t block_key;  /* resident block (0: none)                */
  uint32_t flags;      /* SFC_REQ_* bits                          */
  uint32_t reserved;   /* must be 0                               */
  void* hip_stream;    /* producer stream of the inputs, or NULL  */
} sfc_request;

typedef struct {
  int32_t status;      /* SFC_OK when done                        */
  int32_t level;
  uint64_t tag;
  int64_t cells;
  double t_submit, t_admit, t_done; /* seconds on the library's steady clock */
} sfc_result;

/* Queue a request (non-blocking; the descriptor is copied).  The library's
 * scheduler thread admits requests in arrival order while their state fits
 * the HBM budget (a keyed request whose block already holds its range needs
 * no room and is not held back by others waiting for room), stages them
 * into its arena and drains all admitted work with a persistent kernel
 * replayed as a HIP graph.  Idle lanes take the cells of the oldest
 * admitted request with cells left.  The waves holding cells of a finer
 * AMR level issue first on their SIMD (level >= 5, 4, 3 above the rest): a
 * level-L block is advanced 2^L times per coarse step, so the finest
 * level's substeps form the longest chain of dependent requests, each as
 * long as its slowest cell.  Results do not depend on either order.
 * Environment variables read when the context is created:
 * SFC_SERVE_LEVEL_CLAIMS=1 hands out the cells of the highest level first
 * (levels above 7 count as 7, negative ones as 0; a steady stream of fine
 * requests then delays coarse ones without bound), SFC_SERVE_LEVEL_PRIO=0
 * turns the issue priority off, SFC_SERVE_RING (a power of two, 2..16384,
 * default 16384) sets how many requests per level class and precision may
 * be in flight; admission waits beyond that.
 * Errors: SFC_E_INVAL (bad buffers, dt, precision or flags; 2^31 cells or
 * more; a block key resubmitted with another cell count; SFC_REQ_RESUME
 * without a key), SFC_E_STATE (served form disabled; SFC_REQ_RESUME on a key
 * with no resident state, or on a key being released), SFC_E_BUDGET (larger
 * than the whole budget). */
int sfc_chem_submit(sfc_ctx* ctx, const sfc_request* req, uint64_t* ticket);

/* Copy the results of a completed keyed request (ticket) from the arena
 * into dst (device buffers of the key's cell count; any array may be NULL
 * and is then skipped: y_h2, y_e, eint, tdust, eir, y_h, y_hp, y_hm, tgas,
 * nsub, niter, flags) on hip_stream (NULL = default stream).  Asynchronous:
 * the copy is queued on that stream, and the key's next request does not
 * start before it has run.  Valid while the ticket is its key's latest
 * request and the key is not released (also after sfc_chem_poll).
 * Errors: SFC_E_PENDING (not done yet), SFC_E_STATE (a later request of the
 * key was submitted, the key was released, the request failed, or the
 * ticket has no block key), SFC_E_INVAL (bad arguments or cell count),
 * SFC_E_DEVICE. */
int sfc_chem_fetch(sfc_ctx* ctx, uint64_t ticket, const sfc_cells* dst, void* hip_stream);

/* Give a block key's arena range back, once the key's requests are done
 * (immediately if none is in flight).  Its results can no longer be
 * fetched.  Errors: SFC_E_INVAL (unknown key), SFC_E_STATE (served form
 * disabled). */
int sfc_chem_release(sfc_ctx* ctx, uint64_t block_key);

/* Non-blocking completion check: SFC_OK and *out filled when done (the
 * ticket is then released), SFC_E_PENDING otherwise, SFC_E_INVAL for an
 * unknown ticket. */
int sfc_chem_poll(sfc_ctx* ctx, uint64_t ticket, sfc_result* out);

/* Block until every submitted request is done. */
int sfc_chem_drain(sfc_ctx* ctx);

/* Release the context (waits for outstanding served work).  NULL is a no-op. */
int sfc_chem_destroy(sfc_ctx* ctx);

/* Static text for a status code. */
const char* sfc_strerror(int status);
/* Last error message recorded on the context (thread-local per context). */
const char* sfc_last_error(const sfc_ctx* ctx);
/* Library clock (seconds) used for sfc_result times. */
double sfc_now(void);

#ifdef __cplusplus
}
#endif
#endif
