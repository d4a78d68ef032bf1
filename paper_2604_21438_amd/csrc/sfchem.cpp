// sfchem.cpp -- host side of the C ABI declared in include/sfchem.h:
// contexts, argument checks, kernel launches and the served scheduler.
#include "sfchem.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "sfk.h"
#include "sfserve.h"

namespace {

constexpr double KB = 1.380649e-16;
constexpr double EV = 1.602176634e-12;
constexpr double CL = 2.99792458e10;
constexpr double ARAD = 7.5657e-15;

// k_H2 / k_H3 at temperature T (host, binary64): used only to bound the
// steady-state H- ratio over the temperature range of the rate fits.
double host_hm_ratio(double T) {
  const double k2 = 1.4e-18 * std::pow(T, 0.928) * std::exp(-T / 16200.0);
  const double N = std::pow(T, 0.098493) + 0.32852 * std::pow(T, 0.5561) +
                   2.771e-7 * std::pow(T, 2.1826);
  const double D = 1.0 + 6.191e-3 * std::pow(T, 1.0461) + 8.9712e-11 * std::pow(T, 3.0424) +
                   3.2576e-14 * std::pow(T, 3.7741);
  const double k3 = 1.35e-9 * N / D;
  return k2 / k3;
}

bool fill_net(const sfc_network& in, sfk::Net& o) {
  for (int i = 0; i < 12; ++i) o.rm[i] = in.reac_mult[i];
  for (int i = 0; i < 14; ++i) o.pm[i] = in.proc_mult[i];
  if (!(in.g0_photon_density > 0.0) || !(in.kappa_tnorm > 0.0)) return false;
  o.c_sigma = CL * in.sigma_euv;
  o.k10g = in.k10_per_g0;
  o.inv_g0 = 1.0 / in.g0_photon_density;
  o.zeta = in.zeta_cr;
  o.k4_pre = in.k4_pre;
  o.k4_theta = in.k4_theta;
  o.g2k = in.heat_euv_ev * EV / KB;
  o.g3k = in.heat_h2diss_ev * EV / KB;
  o.pe_k = in.pe_coef * in.pe_eps / KB;
  o.kap_max = in.kappa_max;
  o.kap_tn = 1.0 / in.kappa_tnorm;
  o.kap_uv_c = CL * in.kappa_uv;
  o.e_fuv = in.e_fuv_ev * EV;
  o.e_euv = in.e_euv_ev * EV;
  o.x_c = in.x_c;
  o.x_o = in.x_o;
  o.f_oiii = in.f_oiii;
  for (int j = 0; j < 5; ++j) {
    o.l_tul[j] = in.line_tul[j];
    o.l_a[j] = in.line_a[j];
    o.l_g[j] = in.line_g[j];
    o.l_qn[j] = in.line_qn[j];
    o.l_qe[j] = in.line_qe100[j];
    if (!(in.line_a[j] > 0.0)) return false;
  }
  if ((in.pe_mode != 0 && in.pe_mode != 1) || (in.shield_mode != 0 && in.shield_mode != 1))
    return false;
  if (in.shield_mode == 1 && (!(in.shield_len > 0.0) || !(in.shield_b5 > 0.0))) return false;
  o.sh_b5 = in.shield_b5;
  o.pe_ch = o.pm[3] * 1.3e-24 / KB;
  o.pe_cr = o.pm[3] * 4.65e-30 / KB;
  o.pe_mode = in.pe_mode;
  o.shield_mode = in.shield_mode;
  return true;
}

bool fill_par(const sfc_params& p, double z_default, double cd, const sfk::Net& net,
              double shield_len, sfk::Par& o) {
  if (!(p.f_chem > 0.0) || !(p.y_abs > 0.0) || !(p.newton_rtol > 0.0) || !(p.c_red > 0.0) ||
      !(p.t_cmb > 0.0) || !(p.y_he >= 0.0) || !(p.gamma_ad > 1.0) || p.n_cyc < 0 ||
      p.n_sub_max < 2 || p.newton_max < 1 || (p.ir_mode != 0 && p.ir_mode != 1) ||
      (p.thermal_mode != 0 && p.thermal_mode != 1) || (p.dust_mode != 0 && p.dust_mode != 1) ||
      !(z_default >= 0.0) || !(cd > 0.0) || (p.photon_absorb != 0 && p.photon_absorb != 1) ||
      p.reserved != 0)
    return false;
  o.f_chem = p.f_chem;
  o.y_abs = p.y_abs;
  o.newton_rtol = p.newton_rtol;
  o.c_red = p.c_red;
  o.t_cmb = p.t_cmb;
  o.y_he = p.y_he;
  o.gm1 = p.gamma_ad - 1.0;
  o.igm1 = 1.0 / o.gm1;
  o.cd = cd;
  o.z_default = z_default;
  o.n_cyc = p.n_cyc;
  o.n_sub_max = p.n_sub_max;
  o.newton_max = p.newton_max;
  o.ir_mode = p.ir_mode;
  o.thermal_mode = p.thermal_mode;
  o.dust_mode = p.dust_mode;
  o.photon_absorb = p.photon_absorb;
  // x = N_H2 / 5e14 = y_H2 n_H shield_len sqrt(pi k_B T / (G m_H rho)) / 5e14
  //   = y_H2 sh_k sqrt(n_H T), rho = (1 + 4 y_He) m_H n_H
  constexpr double kGrav = 6.6743e-8, kMH = 1.67262192e-24, kPi = 3.14159265358979323846;
  o.sh_k = shield_len * std::sqrt(kPi * KB / (kGrav * kMH * kMH * (1.0 + 4.0 * p.y_he))) / 5.0e14;
  // per-call constants of the kernels, formed once here
  const double tc = p.t_cmb, tc2 = tc * tc, tc4 = tc * tc * tc * tc;
  o.inv_f_chem = 1.0 / p.f_chem;
  o.cr_a = p.c_red / ARAD;
  o.eir_min = ARAD * tc2 * tc2 / p.c_red;
  o.compton = net.pm[11] * 1.017e-37 * tc4 / KB;
  {
    // kappa(T) = kappa_max x^2 / (1 + x^2), x = T / T_norm, at T_CMB
    const double x = tc * net.kap_tn, d = 1.0 + x * x;
    const double k = net.kap_max * x * x / d;
    const double dk = net.kap_max * 2.0 * x / (d * d) * net.kap_tn;
    o.kir_fix = k;
    o.absir_fix = k * (CL * ARAD) * (tc * tc) * (tc * tc);
    o.betair_fix = k + dk * tc * 0.25;
  }
  // bound of k_H2/k_H3 over [1, 1e8] K (fine log grid, 5 % margin)
  double mx = 0.0;
  for (int i = 0; i <= 8000; ++i) {
    const double T = std::pow(10.0, 8.0 * i / 8000.0);
    const double r = host_hm_ratio(T);
    if (r > mx) mx = r;
  }
  const double scale = net.rm[3] > 0.0 ? net.rm[2] / net.rm[3] : 0.0;
  o.hm_ratio_max = net.rm[3] > 0.0 ? 1.05 * mx * scale : 0.0;
  return true;
}

// Dispatch buffers of the entry point that allocates nothing
// (sfc_chem_step_noalloc): a file-scope device array, one per GPU, holding
// for a call of n <= kNoAllocMaxCells cells the work counter, the order
// buckets, the cell order and the suspended-cell slots (layout_scratch).
constexpr int64_t kNoAllocMaxCells = int64_t(1) << 21;

constexpr size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// bytes of the dispatch buffers of an n-cell call, carved in this order:
// work counter | order buckets | cell order | slot counter | rem | tiso |
// cell | nsub | nit | fl | bucket
constexpr size_t dispatch_bytes(int64_t n) {
  return 256 + al256(size_t(sfk::kOrderWork) * 4) + al256(size_t(n) * 4) + 256 +
         2 * al256(size_t(n) * 8) + 5 * al256(size_t(n) * 4);
}
constexpr size_t kScratchBytes = dispatch_bytes(kNoAllocMaxCells);  // 80.01 MiB

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per HIP device, taken once at the first
// context created on that device (its host-side name is not an address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

}  // namespace

struct sfc_ctx {
  int device = 0;
  sfk::Net net{};
  sfk::Par par{};
  unsigned long long* d_counter = nullptr;
  sfk::Net* d_net = nullptr;  // device copies read by the kernels
  sfk::Par* d_par = nullptr;
  int dispatch = SFC_DISPATCH_PROGRESS;
  int32_t phase_nsub = 4096;
  int32_t* d_order = nullptr;  // density dispatch: cell order and bucket counters
  int64_t order_cap = 0;
  uint32_t* d_buckets = nullptr;
  void* d_sus = nullptr;  // progress dispatch: suspended-cell slots (one block)
  int64_t sus_cap = 0;
  int cus = 0;
  int bpc[3] = {1, 1, 1};  // blocks per CU: LI binary64, LI mixed, NR
  int refill_min = 1;
  std::string last_error;
  sfserve::Server* server = nullptr;
  void* scratch = nullptr;  // this device's copy of `scratch` (null if unavailable)
  std::string scratch_error;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Frees a context's device buffers and the context itself.
void release(sfc_ctx* ctx) {
  if (ctx->d_sus) (void)hipFree(ctx->d_sus);
  if (ctx->d_order) (void)hipFree(ctx->d_order);
  if (ctx->d_buckets) (void)hipFree(ctx->d_buckets);
  if (ctx->d_counter) (void)hipFree(ctx->d_counter);
  if (ctx->d_net) (void)hipFree(ctx->d_net);
  if (ctx->d_par) (void)hipFree(ctx->d_par);
  delete ctx;
}

int fail(sfc_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

int hip_fail(sfc_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, SFC_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool cells_ok(const sfk::Par& par, const sfc_cells* c) {
  if (!c || c->n < 0) return false;
  if (c->n == 0) return true;
  if (!c->y_h2 || !c->y_e || !c->eint || !c->tdust || !c->nh || !c->n_euv || !c->n_fuv)
    return false;
  if (par.ir_mode == 1 && !c->eir) return false;
  return true;
}

sfk::Cells to_kcells(const sfc_cells* c) {
  sfk::Cells k;
  k.n = c->n;
  k.y_h2 = c->y_h2; k.y_e = c->y_e; k.eint = c->eint; k.tdust = c->tdust; k.eir = c->eir;
  k.y_h = c->y_h; k.y_hp = c->y_hp; k.y_hm = c->y_hm; k.tgas = c->tgas;
  k.nh = c->nh; k.n_euv = c->n_euv; k.n_fuv = c->n_fuv; k.zmet = c->zmet;
  k.nsub = c->nsub; k.niter = c->niter; k.flags = c->flags;
  k.n_euv_out = c->n_euv_out; k.n_fuv_out = c->n_fuv_out;
  return k;
}

}  // namespace

extern "C" {

void sfc_network_default(sfc_network* net) {
  if (!net) return;
  std::memset(net, 0, sizeof(*net));
  net->abi_version = SFC_ABI_VERSION;
  net->size = sizeof(sfc_network);
  for (int i = 0; i < SFC_NREAC; ++i) net->reac_mult[i] = 1.0;
  for (int i = 0; i < SFC_NPROC; ++i) net->proc_mult[i] = 1.0;
  net->sigma_euv = 3.0e-18;
  net->k10_per_g0 = 5.0e-11;
  net->g0_photon_density = 3.7e-3;
  net->zeta_cr = 1.0e-17;
  net->k4_pre = 1.0e-10;
  net->k4_theta = 5.2e4;
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
  // H2 (J=2-0), C II 158um, O I 63um, O II 3727A, O III 5007A
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

void sfc_params_default(sfc_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->f_chem = 0.03;
  p->y_abs = 1e-10;
  p->newton_rtol = 1e-12;
  p->c_red = 1e-4;
  p->t_cmb = 2.73;
  p->y_he = 0.1;
  p->gamma_ad = 5.0 / 3.0;
  p->n_cyc = 300;
  p->n_sub_max = 100000;
  p->newton_max = 60;
  p->ir_mode = SFC_IR_EVOLVE;
  p->thermal_mode = SFC_THERMAL_EVOLVE;
  p->dust_mode = SFC_DUST_EVOLVE;
  p->dispatch = SFC_DISPATCH_PROGRESS;
  p->phase_nsub = 4096;
}

int sfc_chem_init(const sfc_network* net_in, double z_default, double dust_cap_factor,
                  const sfc_params* p_in, int hip_device, uint64_t served_budget_bytes,
                  sfc_ctx** out) {
  if (!out) return SFC_E_INVAL;
  *out = nullptr;
  sfc_network net;
  if (net_in) {
    if (net_in->abi_version != SFC_ABI_VERSION || net_in->size != sizeof(sfc_network))
      return SFC_E_VERSION;
    net = *net_in;
  } else {
    sfc_network_default(&net);
  }
  sfc_params p;
  if (p_in) p = *p_in; else sfc_params_default(&p);
  if (!(dust_cap_factor > 0.0) || !std::isfinite(dust_cap_factor)) return SFC_E_INVAL;
  sfk::Net knet;
  sfk::Par kpar;
  if (!fill_net(net, knet) ||
      !fill_par(p, z_default, dust_cap_factor * 1.0e4, knet, net.shield_len, kpar))
    return SFC_E_INVAL;
  if (p.dispatch != SFC_DISPATCH_INDEX && p.dispatch != SFC_DISPATCH_DENSITY &&
      p.dispatch != SFC_DISPATCH_PROGRESS)
    return SFC_E_INVAL;
  if (p.dispatch == SFC_DISPATCH_PROGRESS && p.phase_nsub < 1) return SFC_E_INVAL;
  if (hip_device < 0) return SFC_E_INVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device >= ndev) return SFC_E_DEVICE;
  sfc_ctx* ctx = new (std::nothrow) sfc_ctx();
  if (!ctx) return SFC_E_NOMEM;
  ctx->device = hip_device;
  ctx->net = knet;
  ctx->par = kpar;
  ctx->dispatch = p.dispatch;
  ctx->phase_nsub = p.phase_nsub;
  DeviceGuard g(hip_device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
    delete ctx;
    return SFC_E_DEVICE;
  }
  ctx->cus = prop.multiProcessorCount;
  ctx->bpc[0] = sfk::max_blocks_per_cu(0, sfk::stand_ins(knet));
  ctx->bpc[1] = sfk::max_blocks_per_cu(1, sfk::stand_ins(knet));
  ctx->bpc[2] = sfk::max_blocks_per_cu(2, sfk::stand_ins(knet));
  if (hipMalloc(&ctx->d_counter, sizeof(unsigned long long)) != hipSuccess) {
    delete ctx;
    return SFC_E_NOMEM;
  }
  if (hipMalloc(&ctx->d_net, sizeof(sfk::Net)) != hipSuccess ||
      hipMalloc(&ctx->d_par, sizeof(sfk::Par)) != hipSuccess) {
    release(ctx);
    return SFC_E_NOMEM;
  }
  if (hipMemset(ctx->d_counter, 0, sizeof(unsigned long long)) != hipSuccess ||
      hipMemcpy(ctx->d_net, &ctx->net, sizeof(sfk::Net), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ctx->d_par, &ctx->par, sizeof(sfk::Par), hipMemcpyHostToDevice) != hipSuccess) {
    release(ctx);
    return SFC_E_DEVICE;
  }
  if (hip_device < kMaxDevices) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[hip_device] && g_scratch_err[hip_device] == hipSuccess) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e == hipSuccess && ptr) g_scratch_ptr[hip_device] = ptr;
      else g_scratch_err[hip_device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    ctx->scratch = g_scratch_ptr[hip_device];
    if (!ctx->scratch)
      ctx->scratch_error = std::string("hipGetSymbolAddress: ") +
                           hipGetErrorString(g_scratch_err[hip_device]);
  } else {
    ctx->scratch_error = "device index beyond the scratch table";
  }
  if (const char* e = std::getenv("SFC_REFILL_MIN")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= 64) ctx->refill_min = v;
  }
  if (served_budget_bytes > 0) {
    sfserve::Config sc;
    sc.device = hip_device;
    sc.budget_bytes = served_budget_bytes;
    sc.net = ctx->net;
    sc.par = ctx->par;
    sc.cus = ctx->cus;
    sc.refill_min = ctx->refill_min;
    sc.netc = ctx->d_net;
    sc.parc = ctx->d_par;
    std::string err;
    int code = SFC_E_NOMEM;
    ctx->server = sfserve::create(sc, &err, &code);
    if (!ctx->server) {
      release(ctx);
      return code;
    }
  }
  *out = ctx;
  return SFC_OK;
}

}  // extern "C"

namespace {

// Dispatch buffers of one plain-path call: work counter, density / progress
// order with its bucket counters, and the suspended-cell slots.
struct StepBuffers {
  unsigned long long* counter = nullptr;
  int32_t* order = nullptr;
  uint32_t* buckets = nullptr;
  sfk::Suspended sus{};
  int64_t sus_cap = 0;
};

// Slot arrays of progress dispatch carved from one block of n slots: the
// slot counter, then rem, tiso (binary64), cell, nsub, nit, flags, bucket
// (32-bit), each array 256-byte aligned.
sfk::Suspended carve_suspended(void* base, int64_t n) {
  sfk::Suspended sus;
  char* b = static_cast<char*>(base);
  const size_t cap = size_t(n);
  sus.count = reinterpret_cast<unsigned long long*>(b);
  b += 256;
  sus.rem = reinterpret_cast<double*>(b);
  b += al256(cap * 8);
  sus.tiso = reinterpret_cast<double*>(b);
  b += al256(cap * 8);
  sus.cell = reinterpret_cast<int32_t*>(b);
  b += al256(cap * 4);
  sus.nsub = reinterpret_cast<int32_t*>(b);
  b += al256(cap * 4);
  sus.nit = reinterpret_cast<int32_t*>(b);
  b += al256(cap * 4);
  sus.fl = reinterpret_cast<uint32_t*>(b);
  b += al256(cap * 4);
  sus.bucket = reinterpret_cast<int32_t*>(b);
  return sus;
}

// The context's own buffers, grown (hipMalloc) to n cells.
bool context_buffers(sfc_ctx* ctx, int64_t n, bool order, bool suspended, StepBuffers& b) {
  b.counter = ctx->d_counter;
  if (order) {
    if (n > ctx->order_cap) {
      if (ctx->d_order) (void)hipFree(ctx->d_order);
      ctx->d_order = nullptr;
      ctx->order_cap = 0;
      if (hipMalloc(&ctx->d_order, size_t(n) * sizeof(int32_t)) != hipSuccess) return false;
      ctx->order_cap = n;
    }
    if (!ctx->d_buckets &&
        hipMalloc(&ctx->d_buckets, sfk::kOrderWork * sizeof(uint32_t)) != hipSuccess)
      return false;
    b.order = ctx->d_order;
    b.buckets = ctx->d_buckets;
  }
  if (suspended) {
    if (n > ctx->sus_cap) {
      if (ctx->d_sus) (void)hipFree(ctx->d_sus);
      ctx->d_sus = nullptr;
      ctx->sus_cap = 0;
      const size_t bytes = 256 + 2 * al256(size_t(n) * 8) + 5 * al256(size_t(n) * 4);
      if (hipMalloc(&ctx->d_sus, bytes) != hipSuccess) return false;
      ctx->sus_cap = n;
    }
    b.sus = carve_suspended(ctx->d_sus, ctx->sus_cap);
    b.sus_cap = ctx->sus_cap;
  }
  return true;
}

// The same buffers for an n-cell call carved from this device's scratch
// array (no allocation); the layout of dispatch_bytes.
StepBuffers scratch_buffers(void* scratch_ptr, int64_t n) {
  StepBuffers b;
  char* p = static_cast<char*>(scratch_ptr);
  b.counter = reinterpret_cast<unsigned long long*>(p);
  p += 256;
  b.buckets = reinterpret_cast<uint32_t*>(p);
  p += al256(size_t(sfk::kOrderWork) * 4);
  b.order = reinterpret_cast<int32_t*>(p);
  p += al256(size_t(n) * 4);
  b.sus = carve_suspended(p, n);
  b.sus_cap = n;
  return b;
}

// Plain path launch; method 0 = LI binary64, 1 = LI mixed, 2 = NR binary64.
// fixed: dispatch buffers to use (no allocation), else the context's own.
int step_launch(sfc_ctx* ctx, const sfc_cells* cells, double dt, int method, void* hip_stream,
                const char* who, const StepBuffers* fixed = nullptr) {
  if (!ctx) return SFC_E_INVAL;
  if (!cells_ok(ctx->par, cells))
    return fail(ctx, SFC_E_INVAL, std::string(who) + ": bad cell buffers");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(ctx, SFC_E_INVAL, std::string(who) + ": dt must be positive and finite");
  if (cells->n == 0) return SFC_OK;
  DeviceGuard g(ctx->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  sfk::Args a;
  a.net = ctx->net;
  a.par = ctx->par;
  a.c = to_kcells(cells);
  a.dt = dt;
  a.refill_min = ctx->refill_min;
  a.netc = ctx->d_net;
  a.parc = ctx->d_par;
  const int64_t need = (cells->n + sfk::kBlock - 1) / sfk::kBlock;
  const int64_t cap = int64_t(ctx->cus) * ctx->bpc[method];
  const int grid = int(need < cap ? need : cap);
  a.order = nullptr;
  a.dense = nullptr;
  a.budget = 0;
  a.budget_dev = nullptr;
  a.resume = 0;
  a.fine = 0;
  a.limit = nullptr;
  a.sus = sfk::Suspended{};
  const bool small_ids = cells->n < (int64_t(1) << 31);
  const bool progress = ctx->dispatch == SFC_DISPATCH_PROGRESS && method != 2 && small_ids;
  // density order pays off once lanes take several cells each
  const bool density = ctx->dispatch != SFC_DISPATCH_INDEX && small_ids &&
                       cells->n > 2 * int64_t(grid) * sfk::kBlock;
  StepBuffers buf;
  if (fixed) {
    buf = *fixed;
  } else if (!context_buffers(ctx, cells->n, density || progress, progress, buf)) {
    return fail(ctx, SFC_E_NOMEM, std::string(who) + ": dispatch buffers");
  }
  a.counter = buf.counter;
  if (density) {
    // the first pass of progress dispatch orders every cell by density
    // (cells of one density share a wave and branch alike); plain density
    // dispatch orders the densest quarter and keeps the rest in index order
    const hipError_t oe = sfk::launch_order(cells->nh, cells->n, progress, buf.order,
                                            buf.buckets, s, int64_t(grid) * sfk::kBlock,
                                            ctx->phase_nsub);
    if (oe != hipSuccess) return hip_fail(ctx, oe, "dispatch order launch");
    a.order = buf.order;
    a.dense = buf.buckets + sfk::kOrderDenseWord;
  }
  if (progress) {
    a.sus = buf.sus;
    a.budget = ctx->phase_nsub;
    // with the density order in place the plan decides on the device
    if (density) a.budget_dev = buf.buckets + sfk::kOrderBudgetWord;
    const hipError_t re = sfk::launch_reset(a.sus.count, s);
    if (re != hipSuccess) return hip_fail(ctx, re, "reset launch");
  }
  hipError_t e = sfk::launch_reset(buf.counter, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "reset launch");
  e = method == 2 ? sfk::launch_step_nr(a, grid, s) : sfk::launch_step(a, method, grid, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "step launch");
  if (progress) {
    // second pass: the suspended cells, longest estimated remainder first
    e = sfk::launch_progress_order(a.sus, buf.sus_cap, buf.buckets, buf.order, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "progress order launch");
    sfk::Args b = a;
    b.budget = 0;
    b.budget_dev = nullptr;
    b.resume = 1;
    b.fine = 1;
    b.order = buf.order;
    b.dense = nullptr;
    b.limit = a.sus.count;
    e = sfk::launch_reset(buf.counter, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "reset launch");
    e = sfk::launch_step(b, method, grid, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "step launch");
  }
  return SFC_OK;
}

}  // namespace

extern "C" {

int sfc_chem_step(sfc_ctx* ctx, const sfc_cells* cells, double dt, int precision,
                  void* hip_stream) {
  if (ctx && precision != SFC_FP64 && precision != SFC_MIXED)
    return fail(ctx, SFC_E_INVAL, "sfc_chem_step: unknown precision");
  return step_launch(ctx, cells, dt, precision, hip_stream, "sfc_chem_step");
}

int sfc_chem_step_nr(sfc_ctx* ctx, const sfc_cells* cells, double dt, void* hip_stream) {
  return step_launch(ctx, cells, dt, 2, hip_stream, "sfc_chem_step_nr");
}

int sfc_chem_step_noalloc(sfc_ctx* ctx, const sfc_cells* cells, double dt, int precision,
                          void* hip_stream) {
  if (!ctx) return SFC_E_INVAL;
  if (precision != SFC_FP64 && precision != SFC_MIXED)
    return fail(ctx, SFC_E_INVAL, "sfc_chem_step_noalloc: unknown precision");
  if (!cells || cells->n < 0 || cells->n > kNoAllocMaxCells)
    return fail(ctx, SFC_E_INVAL,
                "sfc_chem_step_noalloc: at most " + std::to_string(kNoAllocMaxCells) +
                    " cells per call (the scratch array's size)");
  if (!ctx->scratch) return fail(ctx, SFC_E_DEVICE, "sfc_chem_step_noalloc: " + ctx->scratch_error);
  const StepBuffers buf = scratch_buffers(ctx->scratch, cells->n);
  return step_launch(ctx, cells, dt, precision, hip_stream, "sfc_chem_step_noalloc", &buf);
}

int sfc_chem_submit(sfc_ctx* ctx, const sfc_request* req, uint64_t* ticket) {
  if (!ctx || !req || !ticket) return SFC_E_INVAL;
  if (!ctx->server) return fail(ctx, SFC_E_STATE, "served form disabled (budget 0)");
  const uint32_t known = SFC_REQ_RESUME | SFC_REQ_WRITEBACK;
  if ((req->flags & ~known) != 0 || req->reserved != 0)
    return fail(ctx, SFC_E_INVAL, "sfc_chem_submit: unknown flags");
  const bool resume = (req->flags & SFC_REQ_RESUME) != 0;
  if (req->cells.n < 0 || (!resume && (!cells_ok(ctx->par, &req->cells) || req->cells.n == 0)))
    return fail(ctx, SFC_E_INVAL, "sfc_chem_submit: bad cell buffers");
  if (!(req->dt_seconds > 0.0) || !std::isfinite(req->dt_seconds))
    return fail(ctx, SFC_E_INVAL, "sfc_chem_submit: dt must be positive and finite");
  if (req->precision != SFC_FP64 && req->precision != SFC_MIXED)
    return fail(ctx, SFC_E_INVAL, "sfc_chem_submit: unknown precision");
  DeviceGuard g(ctx->device);
  std::string err;
  const int rc = sfserve::submit(ctx->server, *req, ticket, &err);
  if (rc != SFC_OK) return fail(ctx, rc, "sfc_chem_submit: " + err);
  return SFC_OK;
}

int sfc_chem_poll(sfc_ctx* ctx, uint64_t ticket, sfc_result* out) {
  if (!ctx || !out) return SFC_E_INVAL;
  if (!ctx->server) return fail(ctx, SFC_E_STATE, "served form disabled (budget 0)");
  return sfserve::poll(ctx->server, ticket, out);
}

int sfc_chem_fetch(sfc_ctx* ctx, uint64_t ticket, const sfc_cells* dst, void* hip_stream) {
  if (!ctx || !dst || dst->n <= 0) return SFC_E_INVAL;
  if (!ctx->server) return fail(ctx, SFC_E_STATE, "served form disabled (budget 0)");
  DeviceGuard g(ctx->device);
  std::string err;
  const int rc = sfserve::fetch(ctx->server, ticket, *dst, hip_stream, &err);
  if (rc != SFC_OK && rc != SFC_E_PENDING) return fail(ctx, rc, "sfc_chem_fetch: " + err);
  return rc;
}

int sfc_chem_release(sfc_ctx* ctx, uint64_t block_key) {
  if (!ctx) return SFC_E_INVAL;
  if (!ctx->server) return fail(ctx, SFC_E_STATE, "served form disabled (budget 0)");
  std::string err;
  const int rc = sfserve::release(ctx->server, block_key, &err);
  if (rc != SFC_OK) return fail(ctx, rc, "sfc_chem_release: " + err);
  return SFC_OK;
}

int sfc_chem_drain(sfc_ctx* ctx) {
  if (!ctx) return SFC_E_INVAL;
  if (!ctx->server) return SFC_OK;
  std::string err;
  const int rc = sfserve::drain(ctx->server, &err);
  if (rc != SFC_OK) return fail(ctx, rc, err);
  return SFC_OK;
}

int sfc_chem_destroy(sfc_ctx* ctx) {
  if (!ctx) return SFC_OK;
  DeviceGuard g(ctx->device);
  if (ctx->server) sfserve::destroy(ctx->server);
  ctx->server = nullptr;
  release(ctx);
  return SFC_OK;
}

const char* sfc_strerror(int status) {
  switch (status) {
    case SFC_OK: return "ok";
    case SFC_E_INVAL: return "invalid argument";
    case SFC_E_NOMEM: return "out of memory";
    case SFC_E_BUDGET: return "request exceeds the served HBM budget";
    case SFC_E_DEVICE: return "HIP device error";
    case SFC_E_PENDING: return "request pending";
    case SFC_E_VERSION: return "network ABI version mismatch";
    case SFC_E_STATE: return "invalid state";
    default: return "unknown status";
  }
}

const char* sfc_last_error(const sfc_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : "";
}

double sfc_now(void) { return sfserve::now(); }

}  // extern "C"
