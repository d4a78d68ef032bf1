// sfserve.cpp -- served form: continuous batching of cell requests (AMR
// blocks of any level, each with its own dt) on one GPU.
//
// Flow of a request:
//   submit   -> incoming queue (caller thread; descriptor copied)
//   admit    -> arena range reserved against the HBM budget, cells copied
//               from the caller's buffers into the arena (copy stream)
//   publish  -> ring entry written into coherent pinned host memory, then
//               the published count is raised (release); each precision has
//               one ring per claim class: one class for all requests
//               (admission order, the default) or one per AMR level, the
//               drain then serving the highest level with work first
//   drain    -> the persistent drain kernel, replayed from a HIP graph on
//               the drain stream whenever it is not running and published
//               work is left, claims cells lane by lane; the lane storing a
//               request's last cell raises that request's done word
//   copy-out -> results copied back into the caller's buffers (copy stream);
//               the arena range is released and the request is complete.
// One scheduler thread owns every stage after submit.  The drain streams are
// masked to fewer CUs than the device has, so the copy kernels of newly
// admitted and finished requests always find a free CU.
#include "sfserve.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace sfserve {

namespace {

enum class St { Incoming, Staging, Running, CopyOut, Done };

struct Req {
  uint64_t ticket = 0;
  sfc_request r{};
  int prec = 0;
  int cls = 0;           // claim class (AMR level clamped to the class range)
  uint64_t seq = 0;      // sequence number in its class's ring
  int64_t off = -1;      // first arena cell
  double t_submit = 0, t_admit = 0, t_done = 0;
  hipEvent_t ev = nullptr;
  St st = St::Incoming;
  int status = SFC_E_PENDING;
  bool done_seen = false;
};

// First-fit allocator of contiguous arena cell ranges.
class Ranges {
 public:
  void reset(int64_t cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  int64_t alloc(int64_t n) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<int64_t, int64_t> free_;
};

constexpr int kSlots = sfk::kClasses * sfk::kRing;

size_t slot_of(const Req* r) { return size_t(r->cls) * sfk::kRing + size_t(r->seq % sfk::kRing); }

// One set of rings (and one drain graph) per precision; every array below
// is class-major, kRing slots per class.
struct Queue {
  sfk::RingEntry* ring = nullptr;      // coherent pinned host memory, kSlots entries
  uint64_t* published = nullptr;       // coherent pinned host memory, kClasses words
  uint64_t* done = nullptr;            // coherent pinned host memory, kSlots words
  sfk::RingEntry* d_ring = nullptr;    // device views of the three above
  uint64_t* d_published = nullptr;
  uint64_t* d_done = nullptr;
  unsigned long long* ctr = nullptr;   // device, 3 x kClasses + 1: head | seen | staged | newest
  uint32_t* claimed = nullptr;         // device, kSlots: cells handed out per slot
  int32_t* remaining = nullptr;        // device, kSlots: cells not yet stored per slot
  uint64_t next_seq[sfk::kClasses] = {};
  std::deque<Req*> inflight[sfk::kClasses];  // admitted, done not yet seen; seq order
  uint64_t pub_total = 0;              // requests published, all classes
  int64_t running = 0;                 // published, done not yet seen
  hipGraph_t graph[2] = {nullptr, nullptr};     // one per drain slot (its slot is an argument)
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int grid = 0;
};

}  // namespace

struct Server {
  Config cfg;
  sfk::Cells arena{};
  void* arena_mem = nullptr;
  int64_t cap = 0;
  bool evolve = false;
  Queue q[2];
  hipStream_t copy_stream = nullptr;
  // Two drain slots, each a CU-masked stream (its own hardware queue).  A
  // drain kernel's waves leave once idle, but the kernel lives on while a
  // few of them finish long cells; a second kernel launched meanwhile takes
  // the freed slots, so newly published requests find a full complement of
  // waves instead of the few survivors.  Once the newer kernel's waves
  // start, the older kernel's waves stop claiming and leave as their cells
  // finish, so its slot frees up for the next launch.
  hipStream_t drain_stream[2] = {nullptr, nullptr};
  hipEvent_t drain_ev[2] = {nullptr, nullptr};
  bool drain_live[2] = {false, false};
  int drain_prec[2] = {0, 0};
  uint64_t drain_pub[2] = {0, 0};  // requests of its precision published at its launch
  uint64_t* gen = nullptr;         // coherent pinned host memory, per slot: latest launch generation
  uint64_t* d_gen = nullptr;
  uint64_t gen_count = 0;
  bool fifo = true;                // every request in class 0 (admission order only)
  int last_prec = 1;
  Ranges ranges;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> incoming;                   // guarded by mu
  std::unordered_map<uint64_t, Req*> tickets;  // guarded by mu
  uint64_t next_ticket = 1;                    // guarded by mu
  int64_t outstanding = 0;                     // guarded by mu
  bool quit = false;                           // guarded by mu
  std::string fatal;                           // guarded by mu
  std::thread th;

  // scheduler thread only
  std::deque<Req*> pending, staging, copyout;
  std::vector<hipEvent_t> events;
};

namespace {

int64_t cell_bytes(bool evolve) {
  // 12 float64 arrays (13 with E_IR) and 3 int32 arrays per arena cell
  return 8 * (evolve ? 13 : 12) + 4 * 3;
}

hipEvent_t get_event(Server* s) {
  if (!s->events.empty()) {
    hipEvent_t e = s->events.back();
    s->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void put_event(Server* s, hipEvent_t e) {
  if (e) s->events.push_back(e);
}

sfk::CopyArgs copy_args(Server* s, const Req* r) {
  sfk::CopyArgs a{};
  const sfc_cells& c = r->r.cells;
  a.user.n = c.n;
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
  a.arena = s->arena;
  a.off = r->off;
  a.z_default = s->cfg.par.z_default;
  Queue& q = s->q[r->prec];
  a.remaining_slot = q.remaining + slot_of(r);
  a.claimed_slot = q.claimed + slot_of(r);
  a.staged = q.ctr + 2 * sfk::kClasses + r->cls;
  a.ir_evolve = s->evolve ? 1 : 0;
  return a;
}

// Called with s->mu NOT held.
void finish(Server* s, Req* r, int status) {
  std::lock_guard<std::mutex> lk(s->mu);
  r->status = status;
  r->t_done = now();
  r->st = St::Done;
  s->outstanding -= 1;
  s->cv_done.notify_all();
}

void set_fatal(Server* s, const std::string& msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fatal.empty()) s->fatal = msg;
  s->cv_done.notify_all();
}

bool hip_ok(Server* s, hipError_t e, const char* where) {
  if (e == hipSuccess) return true;
  set_fatal(s, std::string(where) + ": " + hipGetErrorString(e));
  return false;
}

// One pass of the scheduler; returns true if anything moved.
bool step_once(Server* s) {
  bool moved = false;
  // 1. finished copy-outs -> complete (copy stream is in order)
  while (!s->copyout.empty()) {
    Req* r = s->copyout.front();
    const hipError_t e = hipEventQuery(r->ev);
    if (e == hipErrorNotReady) break;
    if (!hip_ok(s, e, "copy-out")) return false;
    s->copyout.pop_front();
    put_event(s, r->ev);
    r->ev = nullptr;
    s->ranges.release(r->off, r->r.cells.n);
    finish(s, r, SFC_OK);
    moved = true;
  }
  // 2. done words raised by the drain kernel -> copy results back
  for (int p = 0; p < 2; ++p) {
    Queue& q = s->q[p];
    for (auto& fl : q.inflight) {
    for (Req* r : fl) {
      if (r->st != St::Running || r->done_seen) continue;
      const uint64_t d = __atomic_load_n(q.done + slot_of(r), __ATOMIC_ACQUIRE);
      if (d != r->seq + 1) continue;
      r->done_seen = true;
      q.running -= 1;
      r->ev = get_event(s);
      if (!r->ev) return set_fatal(s, "event pool"), false;
      const sfk::CopyArgs a = copy_args(s, r);
      if (!hip_ok(s, sfk::launch_copy_out(a, s->copy_stream), "copy-out launch")) return false;
      if (!hip_ok(s, hipEventRecord(r->ev, s->copy_stream), "event record")) return false;
      r->st = St::CopyOut;
      s->copyout.push_back(r);
      moved = true;
    }
    while (!fl.empty() && fl.front()->done_seen) fl.pop_front();
    }
  }
  // 3. finished copy-ins -> publish, in admission order
  while (!s->staging.empty()) {
    Req* r = s->staging.front();
    const hipError_t e = hipEventQuery(r->ev);
    if (e == hipErrorNotReady) break;
    if (!hip_ok(s, e, "copy-in")) return false;
    s->staging.pop_front();
    put_event(s, r->ev);
    r->ev = nullptr;
    Queue& q = s->q[r->prec];
    sfk::RingEntry& re = q.ring[slot_of(r)];
    re.arena_off = uint64_t(r->off);
    re.n = uint64_t(r->r.cells.n);
    re.dt = r->r.dt_seconds;
    re.level = uint64_t(r->r.level < 0 ? 0 : r->r.level > 255 ? 255 : r->r.level);
    __atomic_store_n(&re.seq, r->seq, __ATOMIC_RELEASE);
    __atomic_store_n(q.published + r->cls, r->seq + 1, __ATOMIC_RELEASE);
    r->st = St::Running;
    q.running += 1;
    q.pub_total += 1;
    moved = true;
  }
  // 4. admission: arrival order, while the arena and the ring have room
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->incoming.empty()) {
      s->pending.push_back(s->incoming.front());
      s->incoming.pop_front();
    }
  }
  while (!s->pending.empty()) {
    Req* r = s->pending.front();
    Queue& q = s->q[r->prec];
    auto& fl = q.inflight[r->cls];
    if (!fl.empty() && q.next_seq[r->cls] - fl.front()->seq >= uint64_t(sfk::kRing)) break;
    const int64_t off = s->ranges.alloc(r->r.cells.n);
    if (off < 0) break;
    s->pending.pop_front();
    r->off = off;
    r->seq = q.next_seq[r->cls]++;
    r->ev = get_event(s);
    if (!r->ev) return set_fatal(s, "event pool"), false;
    const sfk::CopyArgs a = copy_args(s, r);
    if (!hip_ok(s, sfk::launch_copy_in(a, s->copy_stream), "copy-in launch")) return false;
    if (!hip_ok(s, hipEventRecord(r->ev, s->copy_stream), "event record")) return false;
    r->t_admit = now();
    r->st = St::Staging;
    fl.push_back(r);
    s->staging.push_back(r);
    moved = true;
  }
  // 5. keep drain kernels running while published work is left: a free
  //    slot takes a precision that has published work and no live kernel
  //    (alternating when both wait), else a second kernel for a precision
  //    whose live kernel was launched before its latest publications
  for (int i = 0; i < 2; ++i) {
    if (!s->drain_live[i]) continue;
    const hipError_t e = hipEventQuery(s->drain_ev[i]);
    if (e == hipSuccess) s->drain_live[i] = false;
    else if (e != hipErrorNotReady && !hip_ok(s, e, "drain kernel")) return false;
  }
  for (int i = 0; i < 2; ++i) {
    if (s->drain_live[i]) continue;
    const int o = 1 - i;
    int pick = -1;
    for (int k = 1; k <= 2 && pick < 0; ++k) {
      const int p = (s->last_prec + k) % 2;
      const bool covered = s->drain_live[o] && s->drain_prec[o] == p;
      if (s->q[p].running > 0 && !covered) pick = p;
    }
    if (pick < 0 && s->drain_live[o]) {
      const int p = s->drain_prec[o];
      if (s->q[p].running > 0 && s->q[p].pub_total > s->drain_pub[o]) pick = p;
    }
    if (pick < 0) continue;
    Queue& q = s->q[pick];
    // a launch's waves read its generation when they start; older waves of
    // the same precision stop claiming once a newer launch has started
    __atomic_store_n(s->gen + i, ++s->gen_count, __ATOMIC_RELEASE);
    if (!hip_ok(s, hipGraphLaunch(q.exec[i], s->drain_stream[i]), "graph launch")) return false;
    if (!hip_ok(s, hipEventRecord(s->drain_ev[i], s->drain_stream[i]), "event record")) return false;
    s->drain_live[i] = true;
    s->drain_prec[i] = pick;
    s->drain_pub[i] = q.pub_total;
    s->last_prec = pick;
    moved = true;
  }
  return moved;
}

void run(Server* s) {
  (void)hipSetDevice(s->cfg.device);
  for (;;) {
    bool failed;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      failed = !s->fatal.empty();
    }
    if (failed) break;
    const bool moved = step_once(s);
    std::unique_lock<std::mutex> lk(s->mu);
    const bool idle = s->outstanding == 0 && s->incoming.empty();
    const bool live = s->drain_live[0] || s->drain_live[1];
    if (s->quit && idle && !live) break;
    if (!moved) {
      if (idle && !live)
        s->cv_work.wait(lk, [&] { return s->quit || !s->incoming.empty(); });
      else
        s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }
  // after a device error every request still outstanding fails
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->fatal.empty()) {
    for (auto& kv : s->tickets) {
      if (kv.second->st != St::Done) {
        kv.second->st = St::Done;
        kv.second->status = SFC_E_DEVICE;
        kv.second->t_done = now();
      }
    }
    s->outstanding = 0;
    s->cv_done.notify_all();
  }
}

void free_all(Server* s) {
  for (auto& q : s->q) {
    for (auto& x : q.exec)
      if (x) (void)hipGraphExecDestroy(x);
    for (auto& g : q.graph)
      if (g) (void)hipGraphDestroy(g);
    if (q.ring) (void)hipHostFree(q.ring);
    if (q.published) (void)hipHostFree(q.published);
    if (q.done) (void)hipHostFree(q.done);
    if (q.ctr) (void)hipFree(q.ctr);
    if (q.claimed) (void)hipFree(q.claimed);
    if (q.remaining) (void)hipFree(q.remaining);
  }
  if (s->gen) (void)hipHostFree(s->gen);
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  for (auto& e : s->drain_ev)
    if (e) (void)hipEventDestroy(e);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  for (auto& d : s->drain_stream)
    if (d) (void)hipStreamDestroy(d);
  if (s->arena_mem) (void)hipFree(s->arena_mem);
}

double env_num(const char* name, double dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  char* end = nullptr;
  const double x = std::strtod(v, &end);
  return (end && *end == 0) ? x : dflt;
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
  const int64_t cb = cell_bytes(s->evolve);
  s->cap = int64_t(cfg.budget_bytes / uint64_t(cb));
  s->cap = (s->cap / 64) * 64;
  if (s->cap < 64) return fail(s, SFC_E_INVAL, "served budget below 64 cells");
  // arena: one allocation, each array 256-byte aligned
  const int64_t nd = s->evolve ? 13 : 12;
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
  A.nsub = inext();
  A.niter = inext();
  A.flags = reinterpret_cast<uint32_t*>(inext());
  s->ranges.reset(s->cap);

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
  }

  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, cfg.device) != hipSuccess ||
      khz <= 0)
    khz = 100000;  // 100 MHz constant clock
  const double tps = double(khz) * 1e3;
  const int reserve = int(env_num("SFC_SERVE_RESERVE_CUS", 8));
  const int cus = cfg.cus - (reserve >= 0 && reserve < cfg.cus ? reserve : 0);
  s->fifo = env_num("SFC_SERVE_LEVEL_CLAIMS", 0.0) == 0.0;

  for (int prec = 0; prec < 2; ++prec) {
    Queue& q = s->q[prec];
    const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
    if (hipHostMalloc(reinterpret_cast<void**>(&q.ring), sizeof(sfk::RingEntry) * kSlots, fl) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&q.published), 256, fl) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&q.done), sizeof(uint64_t) * kSlots, fl) !=
            hipSuccess)
      return fail(s, SFC_E_NOMEM, "pinned host allocation");
    std::memset(q.ring, 0xff, sizeof(sfk::RingEntry) * kSlots);
    std::memset(q.published, 0, sizeof(uint64_t) * sfk::kClasses);
    std::memset(q.done, 0, sizeof(uint64_t) * kSlots);
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&q.d_ring), q.ring, 0) != hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&q.d_published), q.published, 0) !=
            hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&q.d_done), q.done, 0) != hipSuccess)
      return fail(s, SFC_E_DEVICE, "host pointer mapping");
    const size_t nctr = 3 * sfk::kClasses + 1;
    if (hipMalloc(&q.ctr, sizeof(unsigned long long) * nctr) != hipSuccess ||
        hipMalloc(&q.claimed, sizeof(uint32_t) * kSlots) != hipSuccess ||
        hipMalloc(&q.remaining, sizeof(int32_t) * kSlots) != hipSuccess)
      return fail(s, SFC_E_NOMEM, "served counters");
    if (hipMemset(q.ctr, 0, sizeof(unsigned long long) * nctr) != hipSuccess ||
        hipMemset(q.claimed, 0, sizeof(uint32_t) * kSlots) != hipSuccess ||
        hipMemset(q.remaining, 0, sizeof(int32_t) * kSlots) != hipSuccess)
      return fail(s, SFC_E_DEVICE, "served counters");

    sfk::ServedArgs a{};
    a.net = cfg.net;
    a.par = cfg.par;
    a.arena = s->arena;
    a.ring = q.d_ring;
    a.published = q.d_published;
    a.head = q.ctr;
    a.seen = q.ctr + sfk::kClasses;
    a.staged = q.ctr + 2 * sfk::kClasses;
    a.newest = q.ctr + 3 * sfk::kClasses;
    a.gen = s->d_gen;
    a.claimed = q.claimed;
    a.remaining = q.remaining;
    a.done = q.d_done;
    a.idle_ticks = uint64_t(env_num("SFC_SERVE_IDLE_MS", 100.0) * 1e-3 * tps);
    a.life_ticks = uint64_t(env_num("SFC_SERVE_LIFE_S", 120.0) * tps);
    a.backoff_ticks = uint64_t(10e-6 * tps);
    a.backoff_max_ticks = uint64_t(500e-6 * tps);
    a.refill_min = cfg.refill_min;
    a.level_prio = env_num("SFC_SERVE_LEVEL_PRIO", 1.0) != 0.0 ? 1 : 0;
    a.netc = cfg.netc;
    a.parc = cfg.parc;
    q.grid = cus * sfk::served_blocks_per_cu(prec);
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
  if (req.cells.n > s->cap) {
    if (err) *err = "request of " + std::to_string(req.cells.n) + " cells exceeds the arena (" +
                    std::to_string(s->cap) + " cells)";
    return SFC_E_BUDGET;
  }
  Req* r = new (std::nothrow) Req();
  if (!r) return SFC_E_NOMEM;
  r->r = req;
  r->prec = req.precision;
  r->cls = s->fifo ? 0 : (req.level < 0 ? 0 : req.level >= sfk::kClasses ? sfk::kClasses - 1 : req.level);
  r->t_submit = now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->fatal.empty()) {
    delete r;
    if (err) *err = s->fatal;
    return SFC_E_DEVICE;
  }
  r->ticket = s->next_ticket++;
  s->tickets[r->ticket] = r;
  s->incoming.push_back(r);
  s->outstanding += 1;
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return SFC_OK;
}

int poll(Server* s, uint64_t ticket, sfc_result* out) {
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return SFC_E_INVAL;
  Req* r = it->second;
  if (r->st != St::Done) return SFC_E_PENDING;
  out->status = r->status;
  out->level = r->r.level;
  out->tag = r->r.tag;
  out->cells = r->r.cells.n;
  out->t_submit = r->t_submit;
  out->t_admit = r->t_admit;
  out->t_done = r->t_done;
  const int st = r->status;
  s->tickets.erase(it);
  delete r;
  return st;
}

int drain(Server* s, std::string* err) {
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->outstanding == 0 || !s->fatal.empty(); });
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
    s->cv_done.wait(lk, [&] { return s->outstanding == 0 || !s->fatal.empty(); });
    s->quit = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  (void)hipSetDevice(s->cfg.device);
  for (auto& d : s->drain_stream)
    if (d) (void)hipStreamSynchronize(d);
  if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
  for (auto& kv : s->tickets) delete kv.second;
  free_all(s);
  delete s;
}

double now() {
  using C = std::chrono::steady_clock;
  return std::chrono::duration<double>(C::now().time_since_epoch()).count();
}

}  // namespace sfserve
