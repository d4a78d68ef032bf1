// sfk_serve.hip -- served-form kernels: the persistent drain that claims
// cells of published requests from the per-class rings, and the copy
// kernels that move a request between the caller's buffers and the arena.
// The per-lane method code is in sfk_lane.h.
#include "sfk_lane.h"
#include "sfk_served.h"

namespace sfk {
namespace {

// ------------------------------------------------------------------ served
__device__ inline uint64_t agent_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The slot descriptor a wave last claimed from; every lane holds the same copy.
struct WaveCache {
  uint64_t k = ~0ull;  // request sequence number of the cached descriptor
  int cls = -1;        // its class
  uint64_t n = 0, off = 0, lvl = 0;
  double dt = 0.0;
};

// A lane's request: class in the top byte, AMR level (clamped to 0..255)
// in the next, sequence number below.
constexpr int kClassShift = 56;
constexpr int kLevelShift = 48;
constexpr uint64_t kSeqMask = (1ull << kLevelShift) - 1;

struct Claim {
  uint64_t tk;  // class << kClassShift | level << kLevelShift | seq
  uint64_t first, off;
  double dt;
  int take;
};

// Read the descriptor of ring slot m into c if it belongs to the request
// whose sequence number has the low 32 bits `tag` (seqlock: the arm kernel
// writes ~0, the fields, then the sequence number, with release fences
// between).  Returns false if the slot holds another request, or is being
// rewritten for one.
__device__ inline bool read_meta(const SlotMeta* m, uint32_t tag, int cls, WaveCache& c) {
  const uint64_t s1 = agent_load(&m->seq);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const uint64_t n = agent_load(&m->n);
  const uint64_t off = agent_load(&m->off);
  const uint64_t lvl = agent_load(&m->level);
  const uint64_t dtb = agent_load(reinterpret_cast<const uint64_t*>(&m->dt));
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const uint64_t s2 = agent_load(&m->seq);
  if (s1 != s2 || s1 == ~0ull || uint32_t(s1) != tag) return false;
  c.k = s1;
  c.cls = cls;
  c.n = n;
  c.off = off;
  c.lvl = lvl;
  c.dt = __longlong_as_double((long long)dtb);
  return true;
}

// Claim up to `want` cells for one wave.  Wave-uniform call: every lane
// takes part and gets the same result.  Lane l < kClasses inspects class l,
// so one round of loads covers every class, and the wave takes cells of the
// oldest request of the highest class with unclaimed cells.  The host's
// published count of a class is read only when the class looks exhausted
// and a request was armed since the largest count read so far, which is
// kept in device memory for every wave.  The cells come from one atomicAdd
// on the slot's claim word, so concurrent waves never retry; a request
// found exhausted moves its class head on (compare-and-swap; a failure
// means another wave already did).  If the claim word carries another
// request's tag, the slot was armed again, so the head's request is done:
// the head moves on and the cells handed out are the newer request's.
// Lane kClasses reads the newest launch generation of this precision:
// take = -1 when it is newer than `gen`.
__device__ Claim claim_cells(const ServedArgs& a, int want, WaveCache& c, int lane,
                             uint64_t gen) {
  Claim r{0, 0, 0, 0.0, 0};
  for (int attempt = 0; attempt < 16; ++attempt) {
    uint64_t k = 0, p = 0;
    if (lane == kClasses) {
      k = __hip_atomic_load(a.newest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (lane < kClasses) {
      k = __hip_atomic_load(a.head + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      p = __hip_atomic_load(a.seen + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (k >= p &&
          __hip_atomic_load(a.staged + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > p) {
        p = __hip_atomic_load(a.published + lane, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_fetch_max(a.seen + lane, (unsigned long long)p, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (__ballot(lane == kClasses && k > gen)) {
      r.take = -1;  // a newer launch runs: stop claiming
      return r;
    }
    const unsigned long long avail = __ballot(lane < kClasses && k < p);
    if (avail == 0ull) return r;
    const int cls = 63 - __clzll((long long)avail);
    const uint64_t kc = __shfl(k, cls);
    const size_t slot = size_t(cls) * a.ring + size_t(kc & (a.ring - 1));
    uint64_t first = 0;
    int take = 0;
    if (lane == 0) {
      const unsigned long long w = __hip_atomic_fetch_add(
          a.claimed + slot, (unsigned long long)want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const uint32_t tag = uint32_t(w >> 32);
      const uint64_t o = w & 0xffffffffull;
      bool have;
      if (tag == uint32_t(kc)) {
        have = (c.k == kc && c.cls == cls) || read_meta(a.meta + slot, tag, cls, c);
      } else {
        // the slot holds a newer request of this class: kc is done
        unsigned long long expect = kc;
        __hip_atomic_compare_exchange_strong(a.head + cls, &expect, kc + 1, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        have = (uint32_t(c.k) == tag && c.cls == cls && c.k != ~0ull) ||
               read_meta(a.meta + slot, tag, cls, c);
      }
      if (have && o < c.n) {
        const uint64_t left = c.n - o;
        first = o;
        take = int(left < uint64_t(want) ? left : uint64_t(want));
      } else if (tag == uint32_t(kc)) {
        unsigned long long expect = kc;
        __hip_atomic_compare_exchange_strong(a.head + cls, &expect, kc + 1, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    c.k = __shfl(c.k, 0);
    c.cls = __shfl(c.cls, 0);
    c.n = __shfl(c.n, 0);
    c.off = __shfl(c.off, 0);
    c.lvl = __shfl(c.lvl, 0);
    c.dt = __shfl(c.dt, 0);
    take = __shfl(take, 0);
    if (take > 0) {
      r.tk = (uint64_t(cls) << kClassShift) | (c.lvl << kLevelShift) | (c.k & kSeqMask);
      r.first = __shfl(first, 0);
      r.off = c.off;
      r.dt = c.dt;
      r.take = take;
      return r;
    }
  }
  return r;
}

// Count off the cells the wave's lanes have stored since the last flush:
// one release fence for all of them, then one decrement per cell; the lane
// that takes a request's count to zero raises its done word (system scope).
// pend is the lane's request token (class, level, sequence number) + 1, or 0.
// Wave-uniform call.
__device__ inline void flush_done(const ServedArgs& a, uint64_t& pend) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (pend) {
    const uint64_t tk = pend - 1;
    const uint64_t seq = tk & kSeqMask;
    const size_t slot = size_t(tk >> kClassShift) * a.ring + size_t(seq & (a.ring - 1));
    const int left = __hip_atomic_fetch_add(a.remaining + slot, -1, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    if (left == 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(a.done + slot, seq + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    pend = 0;
  }
}

// Issue priority of the wave from the finest AMR level among its lanes'
// cells: level >= 5 -> 3, 4 -> 2, 3 -> 1, else 0.  A level-L block is
// advanced 2^L times per coarse step, one substep after the other, so the
// finest levels form the longest chains of dependent requests, and each
// substep lasts as long as its slowest cell; with priority the waves holding
// those cells lose fewer issue cycles to the other waves of their SIMD.
// Wave-uniform call; prio is the wave's current setting.
__device__ inline void set_level_prio(int lvl, int& prio) {
  const int want = __ballot(lvl >= 5) ? 3 : __ballot(lvl == 4) ? 2 : __ballot(lvl == 3) ? 1 : 0;
  if (want == prio) return;
  prio = want;
  switch (want) {
    case 3: __builtin_amdgcn_s_setprio(3); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    default: __builtin_amdgcn_s_setprio(0); break;
  }
}

// Persistent drain: lanes refill from the request rings as they finish;
// every cell is advanced by its own request's dt with the same per-lane
// code as the plain step, so a cell's result does not depend on which
// requests share the device with it.  Idle waves back off (doubling waits)
// and leave after idle_ticks without work.  After life_ticks, or once a
// newer launch of the same precision has started (its generation, read
// from the host at each wave's start, is larger), waves stop claiming and
// leave when their lanes are done (each cell is bounded by n_sub_max
// subcycles), so every wave reaches an exit and the newer launch, whose
// waves take the freed slots, serves all new work.  An exiting wave raises
// its slot's left word, which tells the host that the launch has begun to
// shrink.
template <class R, bool kS>
__global__ __launch_bounds__(kBlock) void served_drain_kernel(ServedArgs) {
  stage_tables();
  const int lane = threadIdx.x & 63;
  int64_t cell = -1;
  uint64_t tk = 0, pend = 0;  // the lane's request token; pend = tk + 1 once stored
  double cdt = 0.0;           // the lane's request dt (photon absorption at the store)
  Lane L;
  WaveCache wc;
  const uint64_t t0 = (uint64_t)wall_clock64();
  uint64_t next_try = t0, last_work = t0, backoff = kargs<ServedArgs>().backoff_ticks;
  int since_flush = 0;
  int prio = 0;
  bool closing = false;
  uint64_t gen = 0;
  {
    const ServedArgs& a = kargs<ServedArgs>();
    gen = __hip_atomic_load(a.gen + a.slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (lane == 0)
      __hip_atomic_fetch_max(a.newest, (unsigned long long)gen, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
  for (;;) {
    const ServedArgs& a = kargs<ServedArgs>();
    const unsigned long long idle = __ballot(cell < 0);
    const unsigned long long busy = __ballot(cell >= 0);
    const bool pending = __ballot(pend != 0) != 0ull;
    const int nidle = __popcll(idle);
    const uint64_t now = (uint64_t)wall_clock64();
    if (now - t0 > a.life_ticks) closing = true;
    if (pending && (busy == 0 || nidle >= a.refill_min || ++since_flush >= 64)) {
      flush_done(a, pend);
      since_flush = 0;
    }
    if (!closing && nidle > 0 && (nidle >= a.refill_min || busy == 0) && now >= next_try) {
      const Claim c = claim_cells(a, nidle, wc, lane, gen);
      if (c.take < 0) {
        closing = true;
        continue;
      }
      if (c.take == 0) {
        next_try = now + backoff;
        backoff = backoff * 2 < a.backoff_max_ticks ? backoff * 2 : a.backoff_max_ticks;
        if (busy == 0) {
          if (now - last_work > a.idle_ticks) break;
          __builtin_amdgcn_s_sleep(64);
        }
        continue;
      }
      last_work = now;
      backoff = a.backoff_ticks;
      // order the arena reads after the request's publication
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
      if (cell < 0) {
        const unsigned r = lanes_below(idle);
        if (r < unsigned(c.take)) {
          cell = int64_t(c.off + c.first + r);
          tk = c.tk;
          cdt = c.dt;
          if (!load_cell<R>(fresh(a.netc), fresh(a.parc), a.arena, cell, c.dt, L)) {
            cell = -1;
            pend = tk + 1;
          }
        }
      }
      continue;
    }
    if (busy == 0) {
      if (closing || now - last_work > a.idle_ticks) break;
      if (prio != 0) set_level_prio(-1, prio);
      __builtin_amdgcn_s_sleep(64);
      continue;
    }
    if (a.level_prio) set_level_prio(cell >= 0 ? int((tk >> kLevelShift) & 0xff) : -1, prio);
    if (cell >= 0) {
      if (subcycle<R, kS>(fresh(a.netc), fresh(a.parc), L)) {
        store_cell<R>(fresh(a.netc), fresh(a.parc), a.arena, cell, L, cdt);
        cell = -1;
        pend = tk + 1;
      }
    }
  }
  if (__ballot(pend != 0)) flush_done(kargs<ServedArgs>(), pend);
  // tell the host that this launch no longer holds all its waves
  if (lane == 0) {
    const ServedArgs& a = kargs<ServedArgs>();
    __hip_atomic_store(a.left + a.slot, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ __launch_bounds__(256) void copy_in_kernel(CopyArgs a) {
  const int64_t n = a.user.n;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = a.off + i;
    a.arena.y_h2[j] = a.user.y_h2[i];
    a.arena.y_e[j] = a.user.y_e[i];
    a.arena.eint[j] = a.user.eint[i];
    a.arena.tdust[j] = a.user.tdust[i];
    if (a.ir_evolve) a.arena.eir[j] = a.user.eir[i];
    const_cast<double*>(a.arena.nh)[j] = a.user.nh[i];
    const_cast<double*>(a.arena.n_euv)[j] = a.user.n_euv[i];
    const_cast<double*>(a.arena.n_fuv)[j] = a.user.n_fuv[i];
    const_cast<double*>(a.arena.zmet)[j] = a.user.zmet ? a.user.zmet[i] : a.z_default;
  }
}

// Results of a request (or a resident block) into the caller's buffers;
// arrays the caller passes as NULL are skipped.
__global__ __launch_bounds__(256) void copy_out_kernel(CopyArgs a) {
  const int64_t n = a.user.n;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = a.off + i;
    if (a.user.y_h2) a.user.y_h2[i] = a.arena.y_h2[j];
    if (a.user.y_e) a.user.y_e[i] = a.arena.y_e[j];
    if (a.user.eint) a.user.eint[i] = a.arena.eint[j];
    if (a.user.tdust) a.user.tdust[i] = a.arena.tdust[j];
    if (a.ir_evolve && a.user.eir) a.user.eir[i] = a.arena.eir[j];
    if (a.user.y_h) a.user.y_h[i] = a.arena.y_h[j];
    if (a.user.y_hp) a.user.y_hp[i] = a.arena.y_hp[j];
    if (a.user.y_hm) a.user.y_hm[i] = a.arena.y_hm[j];
    if (a.user.tgas) a.user.tgas[i] = a.arena.tgas[j];
    if (a.user.nsub) a.user.nsub[i] = a.arena.nsub[j];
    if (a.user.niter) a.user.niter[i] = a.arena.niter[j];
    if (a.user.flags) a.user.flags[i] = a.arena.flags[j];
    if (a.user.n_euv_out && a.arena.n_euv_out) a.user.n_euv_out[i] = a.arena.n_euv_out[j];
    if (a.user.n_fuv_out && a.arena.n_fuv_out) a.user.n_fuv_out[i] = a.arena.n_fuv_out[j];
  }
}

// Arm one ring slot: descriptor, remaining count, then the claim word
// (the request's tag, nothing handed out), then the class's armed count.
// Runs after the request's copy-in on the same stream, so a wave that sees
// the new claim word also sees the request's cells.
__global__ __launch_bounds__(64) void arm_kernel(ArmArgs a) {
  if (threadIdx.x != 0) return;
  __hip_atomic_store(&a.meta->seq, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __hip_atomic_store(&a.meta->off, a.off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&a.meta->n, a.n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&a.meta->level, a.level, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(reinterpret_cast<uint64_t*>(&a.meta->dt),
                     (uint64_t)__double_as_longlong(a.dt), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(a.remaining, int32_t(a.n), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __hip_atomic_store(&a.meta->seq, a.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(a.claimed, (unsigned long long)(a.seq & 0xffffffffull) << 32,
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __hip_atomic_fetch_add(a.staged, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

namespace {
template <class K>
int drain_blocks_per_cu(K kernel) {
  int nb = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0);
  return nb > 0 ? nb : 1;
}
}  // namespace

int served_blocks_per_cu(int precision, bool si) {
  if (precision == 1)
    return si ? drain_blocks_per_cu(served_drain_kernel<float, true>)
              : drain_blocks_per_cu(served_drain_kernel<float, false>);
  return si ? drain_blocks_per_cu(served_drain_kernel<double, true>)
            : drain_blocks_per_cu(served_drain_kernel<double, false>);
}

hipError_t launch_served(const ServedArgs& a, int precision, int grid, hipStream_t s) {
  const bool si = stand_ins(a.net);
  if (precision == 1 && si)
    hipLaunchKernelGGL((served_drain_kernel<float, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else if (precision == 1)
    hipLaunchKernelGGL((served_drain_kernel<float, false>), dim3(grid), dim3(kBlock), 0, s, a);
  else if (si)
    hipLaunchKernelGGL((served_drain_kernel<double, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((served_drain_kernel<double, false>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

namespace {
int copy_grid(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return int(g < 512 ? (g > 0 ? g : 1) : 512);
}
}  // namespace

hipError_t launch_copy_in(const CopyArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(copy_in_kernel, dim3(copy_grid(a.user.n)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_copy_out(const CopyArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(copy_out_kernel, dim3(copy_grid(a.user.n)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_arm(const ArmArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(arm_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace sfk
