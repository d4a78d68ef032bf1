// sfserve.cpp -- served form: continuous batching of cell requests (AMR
// blocks of any level, each with its own dt) on one GPU.
//
// Flow of a request (the bookkeeping is sfsched::Core, host-only; this file
// implements its device actions):
//   submit   -> queued (caller thread; descriptor copied; an event recorded
//               on the caller's producer stream if it names one)
//   admit    -> arena range reserved against the HBM budget (a block key
//               keeps its range across its requests), then staged on the
//               copy stream: copy-in from the caller's buffers (not for a
//               request that continues a resident block), and the arm kernel
//               that writes the ring slot's descriptor and claim word
//   publish  -> the published count of the request's claim class is raised
//               (release store to coherent pinned host memory); each
//               precision has one ring per claim class: one class for all
//               requests (admission order, the default) or one per AMR level
//   drain    -> the persistent drain kernel, replayed from a HIP graph on a
//               drain stream whenever it is not running and published work
//               is left, claims cells lane by lane; the lane storing a
//               request's last cell raises that request's done word
//   complete -> results copied back into the caller's buffers (copy stream)
//               for requests without a block key or with write-back; a
//               keyed block's results stay in the arena for sfc_chem_fetch
//               and its next substep.
// One scheduler thread runs every stage after submit.  The drain streams are
// masked to fewer CUs than the device has, so the copy and arm kernels of
// newly admitted and finished requests always find a free CU.
#include "sfserve.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sfsched.h"

namespace sfserve {

namespace {

// What the device layer keeps per request.
struct ReqDev {
  sfc_cells cells{};          // caller buffers (descriptor copy)
  hipEvent_t ev = nullptr;    // stage / copy-out completion
  hipEvent_t in_ev = nullptr; // producer stream of the inputs (may be null)
};

// One set of rings (and drain graphs) per precision; every per-slot array
// is class-major, `ring` slots per class.
struct Queue {
  uint64_t* published = nullptr;       // coherent pinned host memory, kClasses words
  uint64_t* done = nullptr;            // coherent pinned host memory, per slot
  uint64_t* d_published = nullptr;     // device views of the two above
  uint64_t* d_done = nullptr;
  unsigned long long* ctr = nullptr;   // device, 3 x kClasses + 1: head | seen | staged | newest
  unsigned long long* claimed = nullptr;  // device, per slot: tag << 32 | cells handed out
  int32_t* remaining = nullptr;        // device, per slot: cells not yet stored
  sfk::SlotMeta* meta = nullptr;       // device, per slot: descriptor
  hipGraph_t graph[2] = {nullptr, nullptr};     // one per drain slot (its slot is an argument)
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int grid = 0;
};

uint32_t env_ring() {
  const char* v = std::getenv("SFC_SERVE_RING");
  if (!v || !*v) return uint32_t(sfk::kRingMax);
  const long r = std::strtol(v, nullptr, 10);
  if (r < 2 || r > sfk::kRingMax || (r & (r - 1)) != 0) return uint32_t(sfk::kRingMax);
  return uint32_t(r);
}

double env_num(const char* name, double dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  char* end = nullptr;
  const double x = std::strtod(v, &end);
  return (end && *end == 0) ? x : dflt;
}

int64_t cell_bytes(bool evolve, bool absorb) {
  // 12 float64 arrays (one more with E_IR, two more with the absorbed
  // photon densities) and 3 int32 arrays per arena cell
  return 8 * (12 + (evolve ? 1 : 0) + (absorb ? 2 : 0)) + 4 * 3;
}

}  // namespace

struct Server : sfsched::Ops {
  Config cfg;
  sfk::Cells arena{};
  void* arena_mem = nullptr;
  int64_t cap = 0;
  bool evolve = false;
  uint32_t ring = 0;
  Queue q[2];
  hipStream_t copy_stream = nullptr;
  // Two drain slots, each a CU-masked stream (its own hardware queue).  A
  // drain kernel's waves leave once idle, but the kernel lives on while a
  // few of them finish long cells; a second kernel launched meanwhile takes
  // the freed slots, so newly published requests find a full complement of
  // waves instead of the few survivors.  Once the newer kernel's waves
  // start, the older kernel's waves stop claiming and leave as their cells
  // finish, so its slot frees up for the next launch.  The second kernel is
  // launched only once a wave of the live one has exited: while the live
  // kernel holds all its waves they claim the new requests themselves, and
  // a handover then would stop them claiming while the newer kernel's waves
  // wait for room behind their long cells.
  hipStream_t drain_stream[2] = {nullptr, nullptr};
  hipEvent_t drain_ev[2] = {nullptr, nullptr};
  bool drain_live[2] = {false, false};
  int drain_prec[2] = {0, 0};
  uint64_t drain_pub[2] = {0, 0};  // requests of its precision published at its launch
  uint64_t* gen = nullptr;         // coherent pinned host memory, per slot: latest launch generation
  uint64_t* d_gen = nullptr;
  uint64_t* left = nullptr;        // same allocation, per slot: a wave of its latest launch has exited
  uint64_t* d_left = nullptr;
  uint64_t gen_count = 0;
  int last_prec = 1;
  std::vector<hipEvent_t> events;  // pool

  std::mutex mu;                   // guards core and everything the scheduler thread touches
  std::condition_variable cv_work, cv_done;
  sfsched::Core* core = nullptr;
  bool quit = false;
  std::string fatal;
  std::thread th;

  // ---- sfsched::Ops (called with mu held) ----
  sfk::CopyArgs copy_args(const sfsched::Req& r, const sfc_cells& c) const {
    sfk::CopyArgs a{};
    a.user.n = r.n;
    a.user.y_h2 = c.y_h2;
    a.user.y_e = c.y_e;
    a.user.eint = c.eint;
    a.user.tdust = c.tdust;
    a.user.eir = c.eir;
    a.user.y_h = c.y_h;
    a.user.y_hp = c.y_hp;
    a.user.y_hm = c.y_hm;
    a.user.tgas = c.tgas;
    a.user.nh = c.nh;
    a.user.n_euv = c.n_euv;
    a.user.n_fuv = c.n_fuv;
    a.user.zmet = c.zmet;
    a.user.nsub = c.nsub;
    a.user.niter = c.niter;
    a.user.flags = c.flags;
    a.user.n_euv_out = c.n_euv_out;
    a.user.n_fuv_out = c.n_fuv_out;
    a.arena = arena;
    a.off = r.off;
    a.z_default = cfg.par.z_default;
    a.ir_evolve = evolve ? 1 : 0;
    return a;
  }
  hipEvent_t get_event() {
    if (!events.empty()) {
      hipEvent_t e = events.back();
      events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }
  void put_event(hipEvent_t& e) {
    if (e) events.push_back(e);
    e = nullptr;
  }
  int query(hipEvent_t e) {
    const hipError_t x = hipEventQuery(e);
    if (x == hipSuccess) return 1;
    if (x == hipErrorNotReady) return 0;
    return -1;
  }

  int stage(sfsched::Req& r, size_t slot) override {
    ReqDev* d = static_cast<ReqDev*>(r.dev);
    Queue& qq = q[r.prec];
    if (d->in_ev && hipStreamWaitEvent(copy_stream, d->in_ev, 0) != hipSuccess) return -4;
    if (r.copy_in && sfk::launch_copy_in(copy_args(r, d->cells), copy_stream) != hipSuccess)
      return -4;
    sfk::ArmArgs a{};
    a.meta = qq.meta + slot;
    a.claimed = qq.claimed + slot;
    a.remaining = qq.remaining + slot;
    a.staged = qq.ctr + 2 * sfk::kClasses + r.cls;
    a.seq = r.seq;
    a.off = uint64_t(r.off);
    a.n = uint64_t(r.n);
    a.level = uint64_t(r.level < 0 ? 0 : r.level > 255 ? 255 : r.level);
    a.dt = r.dt;
    if (sfk::launch_arm(a, copy_stream) != hipSuccess) return -4;
    d->ev = get_event();
    if (!d->ev || hipEventRecord(d->ev, copy_stream) != hipSuccess) return -4;
    return 0;
  }
  int staged(sfsched::Req& r) override {
    ReqDev* d = static_cast<ReqDev*>(r.dev);
    const int x = query(d->ev);
    if (x == 1) put_event(d->ev);
    return x;
  }
  void publish(int prec, int cls, uint64_t count) override {
    __atomic_store_n(q[prec].published + cls, count, __ATOMIC_RELEASE);
  }
  bool done(const sfsched::Req& r, size_t slot) override {
    return __atomic_load_n(q[r.prec].done + slot, __ATOMIC_ACQUIRE) == r.seq + 1;
  }
  int copy_out(sfsched::Req& r) override {
    ReqDev* d = static_cast<ReqDev*>(r.dev);
    if (sfk::launch_copy_out(copy_args(r, d->cells), copy_stream) != hipSuccess) return -4;
    d->ev = get_event();
    if (!d->ev || hipEventRecord(d->ev, copy_stream) != hipSuccess) return -4;
    return 0;
  }
  int copied_out(sfsched::Req& r) override {
    ReqDev* d = static_cast<ReqDev*>(r.dev);
    const int x = query(d->ev);
    if (x == 1) put_event(d->ev);
    return x;
  }
  void retire(sfsched::Req& r) override {
    ReqDev* d = static_cast<ReqDev*>(r.dev);
    if (d) {
      put_event(d->ev);
      put_event(d->in_ev);
      delete d;
    }
    r.dev = nullptr;
  }
  double now() override { return sfserve::now(); }

  // keep drain kernels running while published work is left: a free slot
  // takes a precision that has published work and no live kernel
  // (alternating when both wait), else a second kernel for a precision
  // whose live kernel was launched before its latest publications
  bool drive_drain() {
    bool moved = false;
    for (int i = 0; i < 2; ++i) {
      if (!drain_live[i]) continue;
      const hipError_t e = hipEventQuery(drain_ev[i]);
      if (e == hipSuccess) drain_live[i] = false;
      else if (e != hipErrorNotReady) return set_fatal(std::string("drain kernel: ") + hipGetErrorString(e)), false;
    }
    for (int i = 0; i < 2; ++i) {
      if (drain_live[i]) continue;
      const int o = 1 - i;
      int pick = -1;
      for (int k = 1; k <= 2 && pick < 0; ++k) {
        const int p = (last_prec + k) % 2;
        const bool covered = drain_live[o] && drain_prec[o] == p;
        if (core->running(p) > 0 && !covered) pick = p;
      }
      if (pick < 0 && drain_live[o]) {
        const int p = drain_prec[o];
        if (core->running(p) > 0 && core->published_total(p) > drain_pub[o] &&
            __atomic_load_n(left + o, __ATOMIC_ACQUIRE) != 0)
          pick = p;
      }
      if (pick < 0) continue;
      // a launch's waves read its generation when they start; older waves of
      // the same precision stop claiming once a newer launch has started.
      // The slot's previous kernel has ended, so nothing writes its left word.
      __atomic_store_n(left + i, uint64_t(0), __ATOMIC_RELEASE);
      __atomic_store_n(gen + i, ++gen_count, __ATOMIC_RELEASE);
      hipError_t e = hipGraphLaunch(q[pick].exec[i], drain_stream[i]);
      if (e == hipSuccess) e = hipEventRecord(drain_ev[i], drain_stream[i]);
      if (e != hipSuccess) return set_fatal(std::string("graph launch: ") + hipGetErrorString(e)), false;
      drain_live[i] = true;
      drain_prec[i] = pick;
      drain_pub[i] = core->published_total(pick);
      last_prec = pick;
      moved = true;
    }
    return moved;
  }
  void set_fatal(const std::string& m) {
    if (fatal.empty()) fatal = m;
  }
};

namespace {

void run(Server* s) {
  (void)hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (!s->fatal.empty()) break;
    std::string f;
    bool moved = s->core->step(*s, &f);
    if (!f.empty()) s->set_fatal(f);
    if (!s->fatal.empty()) break;
    moved = s->drive_drain() || moved;
    if (!s->fatal.empty()) break;
    if (moved) s->cv_done.notify_all();
    const bool idle = s->core->idle();
    const bool live = s->drain_live[0] || s->drain_live[1];
    if (s->quit && idle && !live) break;
    if (!moved) {
      if (idle && !live)
        s->cv_work.wait(lk, [&] { return s->quit || !s->core->idle(); });
      else
        s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }
  // after a device error every request still outstanding fails
  if (!s->fatal.empty()) s->core->fail_all(SFC_E_DEVICE, now());
  s->cv_done.notify_all();
}

void free_all(Server* s) {
  for (auto& q : s->q) {
    for (auto& x : q.exec)
      if (x) (void)hipGraphExecDestroy(x);
    for (auto& g : q.graph)
      if (g) (void)hipGraphDestroy(g);
    if (q.published) (void)hipHostFree(q.published);
    if (q.done) (void)hipHostFree(q.done);
    if (q.ctr) (void)hipFree(q.ctr);
    if (q.claimed) (void)hipFree(q.claimed);
    if (q.remaining) (void)hipFree(q.remaining);
    if (q.meta) (void)hipFree(q.meta);
  }
  if (s->gen) (void)hipHostFree(s->gen);
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  for (auto& e : s->drain_ev)
    if (e) (void)hipEventDestroy(e);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  for (auto& d : s->drain_stream)
    if (d) (void)hipStreamDestroy(d);
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  delete s->core;
  s->core = nullptr;
}

}  // namespace

Server* create(const Config& cfg, std::string* err, int* code) {
  auto fail = [&](Server* s, int c, const std::string& m) -> Server* {
    if (err) *err = m;
    if (code) *code = c;
    if (s) {
      free_all(s);
      delete s;
    }
    return nullptr;
  };
  Server* s = new (std::nothrow) Server();
  if (!s) return fail(nullptr, SFC_E_NOMEM, "server allocation");
  s->cfg = cfg;
  s->evolve = cfg.par.ir_mode == 1;
  const bool absorb = cfg.par.photon_absorb == 1;
  s->ring = env_ring();
  const int64_t cb = cell_bytes(s->evolve, absorb);
  s->cap = int64_t(cfg.budget_bytes / uint64_t(cb));
  s->cap = (s->cap / 64) * 64;
  if (s->cap < 64) return fail(s, SFC_E_INVAL, "served budget below 64 cells");
  // arena: one allocation, each array 256-byte aligned
  const int64_t nd = 12 + (s->evolve ? 1 : 0) + (absorb ? 2 : 0);
  const int64_t dbytes = ((s->cap * 8 + 255) / 256) * 256;
  const int64_t ibytes = ((s->cap * 4 + 255) / 256) * 256;
  if (hipMalloc(&s->arena_mem, size_t(nd * dbytes + 3 * ibytes)) != hipSuccess)
    return fail(s, SFC_E_NOMEM, "arena allocation (budget too large for free device memory)");
  char* p = static_cast<char*>(s->arena_mem);
  auto dnext = [&]() {
    double* r = reinterpret_cast<double*>(p);
    p += dbytes;
    return r;
  };
  auto inext = [&]() {
    int32_t* r = reinterpret_cast<int32_t*>(p);
    p += ibytes;
    return r;
  };
  sfk::Cells& A = s->arena;
  A.n = s->cap;
  A.y_h2 = dnext();
  A.y_e = dnext();
  A.eint = dnext();
  A.tdust = dnext();
  A.eir = s->evolve ? dnext() : nullptr;
  A.y_h = dnext();
  A.y_hp = dnext();
  A.y_hm = dnext();
  A.tgas = dnext();
  A.nh = dnext();
  A.n_euv = dnext();
  A.n_fuv = dnext();
  A.zmet = dnext();
  A.n_euv_out = absorb ? dnext() : nullptr;
  A.n_fuv_out = absorb ? dnext() : nullptr;
  A.nsub = inext();
  A.niter = inext();
  A.flags = reinterpret_cast<uint32_t*>(inext());
  s->core = new (std::nothrow)
      sfsched::Core(s->cap, s->ring, sfk::kClasses, env_num("SFC_SERVE_LEVEL_CLAIMS", 0.0) != 0.0);
  if (!s->core) return fail(s, SFC_E_NOMEM, "scheduler allocation");

  // Every stream carries a CU mask (all CUs): a masked stream gets a
  // hardware queue of its own.  Plain streams share the few hardware queues
  // round-robin, and a copy kernel that lands on the drain's queue waits
  // until the persistent drain kernel ends, so admission (copy-in) and
  // completion (copy-out) would stall behind it.
  std::vector<uint32_t> all_cus(size_t((cfg.cus + 31) / 32), 0u);
  for (int c = 0; c < cfg.cus; ++c) all_cus[size_t(c / 32)] |= 1u << (c % 32);
  const uint32_t mw = uint32_t(all_cus.size());
  if (hipExtStreamCreateWithCUMask(&s->copy_stream, mw, all_cus.data()) != hipSuccess ||
      hipExtStreamCreateWithCUMask(&s->drain_stream[0], mw, all_cus.data()) != hipSuccess ||
      hipExtStreamCreateWithCUMask(&s->drain_stream[1], mw, all_cus.data()) != hipSuccess ||
      hipEventCreateWithFlags(&s->drain_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->drain_ev[1], hipEventDisableTiming) != hipSuccess)
    return fail(s, SFC_E_DEVICE, "stream/event creation");
  {
    const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
    if (hipHostMalloc(reinterpret_cast<void**>(&s->gen), 256, fl) != hipSuccess)
      return fail(s, SFC_E_NOMEM, "pinned host allocation");
    std::memset(s->gen, 0, 256);
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_gen), s->gen, 0) != hipSuccess)
      return fail(s, SFC_E_DEVICE, "host pointer mapping");
    s->left = s->gen + 8;  // its own 64-byte line of the 256-byte block
    s->d_left = s->d_gen + 8;
  }

  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, cfg.device) != hipSuccess ||
      khz <= 0)
    khz = 100000;  // 100 MHz constant clock
  const double tps = double(khz) * 1e3;
  const int reserve = int(env_num("SFC_SERVE_RESERVE_CUS", 8));
  const int cus = cfg.cus - (reserve >= 0 && reserve < cfg.cus ? reserve : 0);
  const size_t slots = size_t(sfk::kClasses) * s->ring;

  for (int prec = 0; prec < 2; ++prec) {
    Queue& q = s->q[prec];
    const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
    if (hipHostMalloc(reinterpret_cast<void**>(&q.published), 256, fl) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&q.done), sizeof(uint64_t) * slots, fl) !=
            hipSuccess)
      return fail(s, SFC_E_NOMEM, "pinned host allocation");
    std::memset(q.published, 0, sizeof(uint64_t) * sfk::kClasses);
    std::memset(q.done, 0, sizeof(uint64_t) * slots);
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&q.d_published), q.published, 0) !=
            hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&q.d_done), q.done, 0) != hipSuccess)
      return fail(s, SFC_E_DEVICE, "host pointer mapping");
    const size_t nctr = 3 * sfk::kClasses + 1;
    if (hipMalloc(&q.ctr, sizeof(unsigned long long) * nctr) != hipSuccess ||
        hipMalloc(&q.claimed, sizeof(unsigned long long) * slots) != hipSuccess ||
        hipMalloc(&q.remaining, sizeof(int32_t) * slots) != hipSuccess ||
        hipMalloc(&q.meta, sizeof(sfk::SlotMeta) * slots) != hipSuccess)
      return fail(s, SFC_E_NOMEM, "served counters");
    // one-time initialisation at creation (nothing here is captured)
    if (hipMemset(q.ctr, 0, sizeof(unsigned long long) * nctr) != hipSuccess ||
        hipMemset(q.claimed, 0, sizeof(unsigned long long) * slots) != hipSuccess ||
        hipMemset(q.remaining, 0, sizeof(int32_t) * slots) != hipSuccess ||
        hipMemset(q.meta, 0xff, sizeof(sfk::SlotMeta) * slots) != hipSuccess)
      return fail(s, SFC_E_DEVICE, "served counters");

    sfk::ServedArgs a{};
    a.net = cfg.net;
    a.par = cfg.par;
    a.arena = s->arena;
    a.meta = q.meta;
    a.claimed = q.claimed;
    a.remaining = q.remaining;
    a.published = q.d_published;
    a.head = q.ctr;
    a.seen = q.ctr + sfk::kClasses;
    a.staged = q.ctr + 2 * sfk::kClasses;
    a.newest = q.ctr + 3 * sfk::kClasses;
    a.gen = s->d_gen;
    a.left = s->d_left;
    a.done = q.d_done;
    a.ring = s->ring;
    a.idle_ticks = uint64_t(env_num("SFC_SERVE_IDLE_MS", 100.0) * 1e-3 * tps);
    a.life_ticks = uint64_t(env_num("SFC_SERVE_LIFE_S", 120.0) * tps);
    a.backoff_ticks = uint64_t(10e-6 * tps);
    a.backoff_max_ticks = uint64_t(500e-6 * tps);
    a.refill_min = cfg.refill_min;
    a.level_prio = env_num("SFC_SERVE_LEVEL_PRIO", 1.0) != 0.0 ? 1 : 0;
    a.netc = cfg.netc;
    a.parc = cfg.parc;
    q.grid = cus * sfk::served_blocks_per_cu(prec, sfk::stand_ins(cfg.net));
    for (int i = 0; i < 2; ++i) {
      a.slot = i;
      if (hipStreamBeginCapture(s->drain_stream[0], hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(s, SFC_E_DEVICE, "graph capture");
      const hipError_t le = sfk::launch_served(a, prec, q.grid, s->drain_stream[0]);
      const hipError_t ce = hipStreamEndCapture(s->drain_stream[0], &q.graph[i]);
      if (le != hipSuccess || ce != hipSuccess)
        return fail(s, SFC_E_DEVICE, "graph capture of the drain kernel");
      if (hipGraphInstantiate(&q.exec[i], q.graph[i], nullptr, nullptr, 0) != hipSuccess)
        return fail(s, SFC_E_DEVICE, "graph instantiation");
    }
  }
  if (hipDeviceSynchronize() != hipSuccess) return fail(s, SFC_E_DEVICE, "device sync");
  s->th = std::thread(run, s);
  return s;
}

int64_t capacity(const Server* s) { return s->cap; }

int submit(Server* s, const sfc_request& req, uint64_t* ticket, std::string* err) {
  sfsched::Req* r = new (std::nothrow) sfsched::Req();
  ReqDev* d = new (std::nothrow) ReqDev();
  if (!r || !d) {
    delete r;
    delete d;
    return SFC_E_NOMEM;
  }
  r->prec = req.precision;
  r->level = req.level;
  r->n = req.cells.n;
  r->dt = req.dt_seconds;
  r->key = req.block_key;
  r->resume = (req.flags & SFC_REQ_RESUME) != 0;
  r->writeback = (req.flags & SFC_REQ_WRITEBACK) != 0;
  r->tag = req.tag;
  d->cells = req.cells;
  r->dev = d;
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->fatal.empty()) {
    delete r;
    delete d;
    if (err) *err = s->fatal;
    return SFC_E_DEVICE;
  }
  if (req.hip_stream) {
    d->in_ev = s->get_event();
    if (!d->in_ev ||
        hipEventRecord(d->in_ev, reinterpret_cast<hipStream_t>(req.hip_stream)) != hipSuccess) {
      s->put_event(d->in_ev);
      delete r;
      delete d;
      if (err) *err = "event record on the producer stream";
      return SFC_E_DEVICE;
    }
  }
  const int rc = s->core->submit(r, now(), err);
  if (rc != SFC_OK) {
    s->put_event(d->in_ev);
    delete d;
    delete r;
    return rc;
  }
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return SFC_OK;
}

int poll(Server* s, uint64_t ticket, sfc_result* out) {
  std::lock_guard<std::mutex> lk(s->mu);
  sfsched::Req r;
  const int rc = s->core->poll(ticket, &r);
  if (rc == SFC_E_INVAL || rc == SFC_E_PENDING) return rc;
  out->status = r.status;
  out->level = r.level;
  out->tag = r.tag;
  out->cells = r.n;
  out->t_submit = r.t_submit;
  out->t_admit = r.t_admit;
  out->t_done = r.t_done;
  return r.status;
}

int fetch(Server* s, uint64_t ticket, const sfc_cells& dst, void* hip_stream, std::string* err) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->fatal.empty()) {
    if (err) *err = s->fatal;
    return SFC_E_DEVICE;
  }
  int64_t off = -1, n = 0;
  const int rc = s->core->fetch_range(ticket, &off, &n, err);
  if (rc != SFC_OK) return rc;
  if (dst.n != n) {
    if (err) *err = "fetch: destination holds " + std::to_string(dst.n) + " cells, the block " +
                    std::to_string(n);
    return SFC_E_INVAL;
  }
  sfsched::Req r;
  r.n = n;
  r.off = off;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  hipEvent_t ev = nullptr;
  hipError_t e = sfk::launch_copy_out(s->copy_args(r, dst), st);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev, st);
  // the block's next substep (and any later use of its range) is staged on
  // the copy stream, after this copy
  if (e == hipSuccess) e = hipStreamWaitEvent(s->copy_stream, ev, 0);
  if (ev) (void)hipEventDestroy(ev);
  if (e != hipSuccess) {
    if (err) *err = std::string("fetch: ") + hipGetErrorString(e);
    return SFC_E_DEVICE;
  }
  return SFC_OK;
}

int release(Server* s, uint64_t key, std::string* err) {
  std::lock_guard<std::mutex> lk(s->mu);
  const int rc = s->core->release(key, err);
  s->cv_work.notify_one();
  return rc;
}

int drain(Server* s, std::string* err) {
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->core->outstanding() == 0 || !s->fatal.empty(); });
  if (!s->fatal.empty()) {
    if (err) *err = s->fatal;
    return SFC_E_DEVICE;
  }
  return SFC_OK;
}

void destroy(Server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->core->outstanding() == 0 || !s->fatal.empty(); });
    s->quit = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  (void)hipSetDevice(s->cfg.device);
  for (auto& d : s->drain_stream)
    if (d) (void)hipStreamSynchronize(d);
  if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
  free_all(s);
  delete s;
}

double now() {
  using C = std::chrono::steady_clock;
  return std::chrono::duration<double>(C::now().time_since_epoch()).count();
}

}  // namespace sfserve
