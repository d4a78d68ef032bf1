// sfk_li.hip -- the plain step: the persistent lane-refill kernel over a
// caller's cells (LI binary64, mixed, and the Newton-Raphson comparator)
// and the density and two-phase progress dispatch kernels.  The per-lane
// method code is in sfk_lane.h.
#include "sfk_lane.h"

namespace sfk {
namespace {

// ------------------------------------------------------------------ kernels
// Persistent lane-refill driver.  cell: >= 0 working, -1 idle, -2 retired
// (the counter passed the end).  Every lane either works on a cell, whose
// subcycles are bounded by n_sub_max, or retires; the wave leaves once all
// its lanes have retired.
// Past the density-ordered head, work positions are claimed 64 at a time
// per wave (one atomicAdd) into a wave-local stash that idle lanes draw
// from in order: the cells behind 64 consecutive positions (four cache
// lines per array in index order) are then all read and written through
// the L2 of the XCD the wave runs on.
constexpr unsigned kStash = 64;

// Estimated cost bucket of a cell suspended after its first pass: the
// subcycles it still needs at the larger of two paces, the average over
// the pass (nsub steps covered dt - rem) and that of its last subcycle
// (hlast), at most what the subcycle cap leaves; half-octave buckets.
// The last step catches cells whose steps have begun to shrink: at the
// average pace they would be claimed last and run alone at the end.
__device__ inline int progress_bucket(double dt, double rem, int32_t nsub, int32_t nmax,
                                      double hlast) {
  double est = double(nmax - nsub);
  const double done = dt - rem;
  if (done > 0.0) {
    double g = double(nsub) * (rem / done);
    if (hlast > 0.0) g = fmax(g, rem / hlast);
    if (g < est) est = g;
  }
  if (!(est > 0.0)) est = 0.0;
  const float l2 = __builtin_amdgcn_logf(float(est) + 1.0f);  // log2
  const int b = int(floorf(2.0f * l2));
  return b < 0 ? 0 : (b >= kOrderBuckets ? kOrderBuckets - 1 : b);
}

// kNR selects the Newton-Raphson comparator instead of the LI subcycle
// (binary64 only); both share the lane refill, stash and dispatch.
template <class R, bool kNR, bool kS>
__device__ __attribute__((always_inline)) inline void step_loop() {
  stage_tables();
  const int lane = threadIdx.x & 63;
  int64_t cell = -1;
  Lane L;
  double tsub = 0.0;  // NR driver state
  int lev = 0, attempts = 0;
  unsigned long long sbase = 0;  // wave-uniform stash: positions [sbase, sbase + sleft)
  const int32_t budget = kargs<Args>().budget_dev ? int32_t(*kargs<Args>().budget_dev)
                                                   : kargs<Args>().budget;
  unsigned sleft = 0;
  for (;;) {
    const Args& a = kargs<Args>();
    const unsigned long long idle = __ballot(cell == -1);
    const unsigned long long busy = __ballot(cell >= 0);
    const int nidle = __popcll(idle);
    if (nidle > 0 && (nidle >= a.refill_min || busy == 0)) {
      if (sleft == 0) {
        // inside the density-ordered head claim only what the idle lanes
        // take now (those cells are long and must not wait in a stash)
        const int leader = __ffsll((long long)idle) - 1;
        unsigned long long base = 0;
        unsigned want = kStash;
        if (lane == leader) {
          const unsigned long long head = a.dense ? (unsigned long long)(*a.dense) : 0ull;
          if (a.fine ||
              __hip_atomic_load(a.counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < head)
            want = unsigned(nidle);
          base = atomicAdd(a.counter, (unsigned long long)want);
        }
        sbase = __shfl(base, leader);
        sleft = unsigned(__shfl(int(want), leader));
      }
      const unsigned take = unsigned(nidle) < sleft ? unsigned(nidle) : sleft;
      if (cell == -1) {
        const unsigned r = lanes_below(idle);
        if (r < take) {
          const unsigned long long idx = sbase + r;
          const unsigned long long lim = a.limit ? *a.limit : (unsigned long long)a.c.n;
          if (idx < lim) {
            if (!kNR && a.resume) {
              cell = resume_cell(fresh(a.netc), fresh(a.parc), a.c, a.sus, a.order[idx], L);
            } else {
              cell = a.order ? int64_t(a.order[idx]) : int64_t(idx);
              if (!load_cell<R>(fresh(a.netc), fresh(a.parc), a.c, cell, a.dt, L)) cell = -1;
            }
            tsub = 0.0;
            lev = 0;
            attempts = 0;
          } else {
            cell = -2;
          }
        }
      }
      sbase += take;
      sleft -= take;
      continue;
    }
    if (busy == 0) break;
    if (cell >= 0) {
      const double rem_before = L.rem;
      const bool done = kNR ? nr_attempt<kS>(fresh(a.netc), fresh(a.parc), L, tsub, lev, attempts)
                            : subcycle<R, kS>(fresh(a.netc), fresh(a.parc), L);
      if (done) {
        store_cell<R>(fresh(a.netc), fresh(a.parc), a.c, cell, L, a.dt);
        cell = -1;
      } else if (!kNR && budget > 0 && L.nsub >= budget) {
        // first pass over: one slot counter update per wave
        const unsigned long long m = __ballot(true);
        const int leader = __ffsll((long long)m) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(a.sus.count, (unsigned long long)__popcll(m));
        base = __shfl(base, leader);
        const unsigned long long slot = base + lanes_below(m);
        suspend_cell(fresh(a.parc), a.c, a.sus, cell, slot, L);
        a.sus.bucket[slot] =
            progress_bucket(a.dt, L.rem, L.nsub, fresh(a.parc).n_sub_max, rem_before - L.rem);
        cell = -1;
      }
    }
  }
}

// The LI kernels at two waves per SIMD at least (binary64 peaks at ~220
// registers; mixed fits three waves without the stand-in pieces).  kS: the
// network's stand-in pieces compiled in (stand_ins()).
template <class R, bool kS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
void li_step_kernel(Args) { step_loop<R, false, kS>(); }

// The NR comparator: its inner solve (nr_inner) is a called function, so
// the register budget is left to the compiler (it settles at two waves per
// SIMD without spills); one wave per SIMD is allowed rather than a spill.
template <bool kS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1)))
void nr_step_kernel(Args) { step_loop<double, true, kS>(); }

__global__ void reset_kernel(unsigned long long* counter) { *counter = 0ull; }

// ------------------------------------------------------------------ dispatch
// Density dispatch.  The densest cells (those in the top half-octave
// buckets of n_H that together hold at most a quarter of the cells, or all
// cells) go first, bucket by bucket, densest first; all other cells follow
// in index order, so that most lanes still read consecutive cells.  Each block owns
// one contiguous chunk of cells.  Invalid densities (non-positive, NaN) go
// to the lowest bucket.  Work buffer (uint32): hist[B] | offs[B] | plan[4]
// | blockcnt[kOrderBlocks] | blockoff[kOrderBlocks].
__device__ inline int density_bucket(double nh) {
  if (!(nh > 0.0) || !(nh < 1.0e300)) return 0;
  const float l2 = __builtin_amdgcn_logf(float(nh));  // log2, binary32 is plenty
  int b = int(floorf(2.0f * l2)) + kOrderBuckets / 2;
  return b < 0 ? 0 : (b >= kOrderBuckets ? kOrderBuckets - 1 : b);
}

__global__ __launch_bounds__(256) void order_zero_kernel(uint32_t* work) {
  for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x) work[t] = 0u;
}

struct OrderWork {
  uint32_t *hist, *offs, *plan, *blockcnt, *blockoff;
};
__device__ inline OrderWork order_work(uint32_t* w) {
  return {w, w + kOrderBuckets, w + 2 * kOrderBuckets, w + 2 * kOrderBuckets + 4,
          w + 2 * kOrderBuckets + 4 + kOrderBlocks};
}
// [begin, end) of block b's chunk (chunk is a multiple of 256)
__device__ inline void chunk_of(int64_t n, int64_t chunk, int b, int64_t& begin, int64_t& end) {
  begin = int64_t(b) * chunk;
  end = begin + chunk < n ? begin + chunk : n;
}

__global__ __launch_bounds__(256) void order_count_kernel(const double* nh, int64_t n,
                                                          int64_t chunk, uint32_t* work) {
  __shared__ uint32_t h[kOrderBuckets];
  for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x) h[t] = 0u;
  __syncthreads();
  int64_t begin, end;
  chunk_of(n, chunk, blockIdx.x, begin, end);
  for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x)
    atomicAdd(&h[density_bucket(nh[i])], 1u);
  __syncthreads();
  const OrderWork w = order_work(work);
  for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x)
    if (h[t]) atomicAdd(&w.hist[t], h[t]);
}

// One thread: the cut bucket, the dense buckets' offsets (densest first)
// and the number of dense cells; all_dense puts every cell in the head.
__global__ void order_plan_kernel(int64_t n, int all_dense, int64_t lanes, int32_t budget,
                                  uint32_t* work) {
  if (threadIdx.x != 0) return;
  const OrderWork w = order_work(work);
  const uint64_t cap = all_dense ? uint64_t(n) : uint64_t(n) / 4;
  uint64_t sum = 0;
  int cut = kOrderBuckets;
  for (int b = kOrderBuckets - 1; b >= 0; --b) {
    if (sum + w.hist[b] > cap) break;
    sum += w.hist[b];
    cut = b;
  }
  uint32_t off = 0u;
  for (int b = kOrderBuckets - 1; b >= 0; --b) {
    w.offs[b] = b >= cut ? off : 0u;
    if (b >= cut) off += w.hist[b];
  }
  w.plan[0] = uint32_t(cut);
  w.plan[1] = off;
  if (all_dense) {
    // Progress dispatch pays off when the long (dense) cells outnumber the
    // lanes: the resumed pass then starts the longest first.  With fewer,
    // suspending them at the budget only postpones their rest until the
    // whole first pass is over, so the first pass runs every cell to its end.
    uint64_t dense = 0;
    for (int b = density_bucket(1.0e6); b < kOrderBuckets; ++b) dense += w.hist[b];
    w.plan[2] = dense >= uint64_t(lanes) ? uint32_t(budget) : 0u;
  }
}

__global__ __launch_bounds__(256) void order_blockcount_kernel(const double* nh, int64_t n,
                                                               int64_t chunk, uint32_t* work) {
  __shared__ uint32_t c;
  if (threadIdx.x == 0) c = 0u;
  __syncthreads();
  const OrderWork w = order_work(work);
  const int cut = int(w.plan[0]);
  int64_t begin, end;
  chunk_of(n, chunk, blockIdx.x, begin, end);
  uint32_t mine = 0u;
  for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x)
    mine += density_bucket(nh[i]) < cut ? 1u : 0u;
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) w.blockcnt[blockIdx.x] = c;
}

// One thread: where each block's index-ordered cells start.
__global__ void order_blockscan_kernel(int nblocks, uint32_t* work) {
  if (threadIdx.x != 0) return;
  const OrderWork w = order_work(work);
  uint32_t off = w.plan[1];
  for (int b = 0; b < nblocks; ++b) {
    w.blockoff[b] = off;
    off += w.blockcnt[b];
  }
}

// Dense cells take a range reserved per bucket (any order inside a bucket);
// the others are placed in index order: the chunk is walked in tiles of
// 256, each wave ranks its lanes with a ballot and the waves stack up in
// order.
__global__ __launch_bounds__(256) void order_scatter_kernel(const double* nh, int64_t n,
                                                            int64_t chunk, uint32_t* work,
                                                            int32_t* order) {
  __shared__ uint32_t cnt[kOrderBuckets], base[kOrderBuckets];
  __shared__ uint32_t wtot[4];
  __shared__ uint32_t running;
  const OrderWork w = order_work(work);
  const int cut = int(w.plan[0]);
  int64_t begin, end;
  chunk_of(n, chunk, blockIdx.x, begin, end);
  for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x) cnt[t] = 0u;
  if (threadIdx.x == 0) running = 0u;
  __syncthreads();
  for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
    const int b = density_bucket(nh[i]);
    if (b >= cut) atomicAdd(&cnt[b], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x) {
    base[t] = cnt[t] ? atomicAdd(&w.offs[t], cnt[t]) : 0u;
    cnt[t] = 0u;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const uint32_t boff = w.blockoff[blockIdx.x];
  for (int64_t t0 = begin; t0 < end; t0 += blockDim.x) {
    const int64_t i = t0 + threadIdx.x;
    const int b = i < end ? density_bucket(nh[i]) : kOrderBuckets;
    const bool rest = i < end && b < cut;
    const unsigned long long m = __ballot(rest);
    const uint32_t rank = lanes_below(m);
    if ((threadIdx.x & 63) == 0) wtot[wave] = uint32_t(__popcll(m));
    __syncthreads();
    uint32_t before = running;
    for (int v = 0; v < wave; ++v) before += wtot[v];
    if (rest) order[boff + before + rank] = int32_t(i);
    if (i < end && b >= cut) {
      const uint32_t r = atomicAdd(&cnt[b], 1u);
      order[base[b] + r] = int32_t(i);
    }
    __syncthreads();
    if (threadIdx.x == 0) running += wtot[0] + wtot[1] + wtot[2] + wtot[3];
    __syncthreads();
  }
}

// Second phase of two-phase dispatch: the suspended cells, longest
// estimated remainder first, in decreasing half-octave buckets of the
// estimate (any order inside a bucket), the bucket taken at suspension
// (progress_bucket).  Slots [0, *count) are split into one contiguous
// share per block.
__device__ inline void slot_share(unsigned long long used, int b, int nb, int64_t& begin,
                                  int64_t& end) {
  const int64_t per = (int64_t(used) + nb - 1) / nb;
  begin = int64_t(b) * per;
  end = begin + per < int64_t(used) ? begin + per : int64_t(used);
  if (begin > end) begin = end;
}

__global__ __launch_bounds__(256) void progress_count_kernel(Suspended sus, uint32_t* work) {
  __shared__ uint32_t h[kOrderBuckets];
  for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x) h[t] = 0u;
  __syncthreads();
  int64_t begin, end;
  slot_share(*sus.count, blockIdx.x, gridDim.x, begin, end);
  for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x) atomicAdd(&h[sus.bucket[i]], 1u);
  __syncthreads();
  const OrderWork w = order_work(work);
  for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x)
    if (h[t]) atomicAdd(&w.hist[t], h[t]);
}

// One thread: bucket offsets, longest bucket first.
__global__ void progress_plan_kernel(uint32_t* work) {
  if (threadIdx.x != 0) return;
  const OrderWork w = order_work(work);
  uint32_t off = 0u;
  for (int b = kOrderBuckets - 1; b >= 0; --b) {
    w.offs[b] = off;
    off += w.hist[b];
  }
}

__global__ __launch_bounds__(256) void progress_scatter_kernel(Suspended sus, uint32_t* work,
                                                               int32_t* order) {
  __shared__ uint32_t cnt[kOrderBuckets], base[kOrderBuckets];
  const OrderWork w = order_work(work);
  int64_t begin, end;
  slot_share(*sus.count, blockIdx.x, gridDim.x, begin, end);
  for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x) cnt[t] = 0u;
  __syncthreads();
  for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x)
    atomicAdd(&cnt[sus.bucket[i]], 1u);
  __syncthreads();
  for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x) {
    base[t] = cnt[t] ? atomicAdd(&w.offs[t], cnt[t]) : 0u;
    cnt[t] = 0u;
  }
  __syncthreads();
  for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
    const int b = sus.bucket[i];
    order[base[b] + atomicAdd(&cnt[b], 1u)] = int32_t(i);
  }
}

// Arena <-> caller copies of one request (grid-stride over its cells).

}  // namespace

hipError_t launch_step(const Args& a, int precision, int grid, hipStream_t s) {
  const bool si = stand_ins(a.net);
  if (precision == 1 && si)
    hipLaunchKernelGGL((li_step_kernel<float, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else if (precision == 1)
    hipLaunchKernelGGL((li_step_kernel<float, false>), dim3(grid), dim3(kBlock), 0, s, a);
  else if (si)
    hipLaunchKernelGGL((li_step_kernel<double, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((li_step_kernel<double, false>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_step_nr(const Args& a, int grid, hipStream_t s) {
  if (stand_ins(a.net))
    hipLaunchKernelGGL((nr_step_kernel<true>), dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((nr_step_kernel<false>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reset(unsigned long long* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

namespace {
template <class K>
int blocks_per_cu(K kernel) {
  int nb = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0);
  return nb > 0 ? nb : 1;
}
}  // namespace

int max_blocks_per_cu(int precision, bool si) {
  if (precision == 2) return si ? blocks_per_cu(nr_step_kernel<true>) : blocks_per_cu(nr_step_kernel<false>);
  if (precision == 1)
    return si ? blocks_per_cu(li_step_kernel<float, true>) : blocks_per_cu(li_step_kernel<float, false>);
  return si ? blocks_per_cu(li_step_kernel<double, true>) : blocks_per_cu(li_step_kernel<double, false>);
}

hipError_t launch_order(const double* nh, int64_t n, bool all_dense, int32_t* order,
                        uint32_t* work, hipStream_t s, int64_t lanes, int32_t budget) {
  const int64_t tiles = (n + 255) / 256;
  const int grid = int(tiles < kOrderBlocks ? (tiles > 0 ? tiles : 1) : kOrderBlocks);
  const int64_t chunk = ((tiles + grid - 1) / grid) * 256;
  hipLaunchKernelGGL(order_zero_kernel, dim3(1), dim3(256), 0, s, work);
  hipLaunchKernelGGL(order_count_kernel, dim3(grid), dim3(256), 0, s, nh, n, chunk, work);
  hipLaunchKernelGGL(order_plan_kernel, dim3(1), dim3(64), 0, s, n, int(all_dense), lanes, budget,
                     work);
  hipLaunchKernelGGL(order_blockcount_kernel, dim3(grid), dim3(256), 0, s, nh, n, chunk, work);
  hipLaunchKernelGGL(order_blockscan_kernel, dim3(1), dim3(64), 0, s, grid, work);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(grid), dim3(256), 0, s, nh, n, chunk, work,
                     order);
  return hipGetLastError();
}

hipError_t launch_progress_order(const Suspended& sus, int64_t cap, uint32_t* work,
                                 int32_t* order, hipStream_t s) {
  const int64_t tiles = (cap + 255) / 256;
  const int grid = int(tiles < kOrderBlocks ? (tiles > 0 ? tiles : 1) : kOrderBlocks);
  hipLaunchKernelGGL(order_zero_kernel, dim3(1), dim3(256), 0, s, work);
  hipLaunchKernelGGL(progress_count_kernel, dim3(grid), dim3(256), 0, s, sus, work);
  hipLaunchKernelGGL(progress_plan_kernel, dim3(1), dim3(64), 0, s, work);
  hipLaunchKernelGGL(progress_scatter_kernel, dim3(grid), dim3(256), 0, s, sus, work, order);
  return hipGetLastError();
}

}  // namespace sfk
