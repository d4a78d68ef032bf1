// sfk_served.h -- internal interface between the served-form scheduler
// (sfserve.cpp) and its kernels (sfk_serve.hip).
#pragma once
#include "sfk.h"

namespace sfk {

// Served form.  Requests are published by the host into rings that live in
// coherent pinned host memory, one ring per claim class (the AMR level,
// clamped to 0..kClasses-1).  Waves claim cells of the oldest request of the
// highest class that has unclaimed cells: a device head index per class
// names that request, and a per-slot device counter hands out its cells with
// one atomicAdd.  A slot is reused only kRing requests of its class later,
// long after every wave has moved past it.  The lane that stores a request's
// last cell raises its done word.
constexpr int kRing = 16384;   // ring slots per class
constexpr int kClasses = 8;    // claim classes; finer AMR levels are served first

struct RingEntry {            // written by the host before publication
  uint64_t arena_off;         // first arena cell of the request
  uint64_t n;                 // cells (> 0)
  double dt;                  // interval [s]
  uint64_t level;             // AMR level, clamped to 0..255
  uint64_t seq;               // request sequence number in its class (written last)
};

struct ServedArgs {
  Net net;
  Par par;
  Cells arena;                        // arena SoA arrays (n = capacity)
  const RingEntry* ring;              // host-mapped, kClasses * kRing entries, class-major
  const uint64_t* published;          // host-mapped, kClasses: requests published per class
  unsigned long long* head;           // device, kClasses: oldest request that may have unclaimed cells
  unsigned long long* seen;           // device, kClasses: largest published count read so far
  const unsigned long long* staged;   // device, kClasses: requests whose copy-in was launched
  unsigned long long* newest;         // device: largest launch generation started (this precision)
  const uint64_t* gen;                // host-mapped, per drain slot: generation of its latest launch
  uint32_t* claimed;                  // device, per ring slot: cells handed out
  int32_t* remaining;                 // device, per ring slot: cells not yet stored
  uint64_t* done;                     // host-mapped, per ring slot: seq + 1 when complete
  uint64_t idle_ticks;                // a wave with no work for this long exits
  uint64_t life_ticks;                // no claims after this long (wall-clock ticks)
  uint64_t backoff_ticks;             // first wait after a claim that found nothing
  uint64_t backoff_max_ticks;         // waits double up to this
  int32_t refill_min;
  int32_t level_prio;                 // waves holding finer-level cells issue first (0: off)
  int32_t slot;                       // drain slot this launch runs on
  const Net* netc;                    // device copies of net and par (read-only)
  const Par* parc;
};

// Copy of one request between caller buffers and the arena.
struct CopyArgs {
  Cells user;        // caller buffers (n = request cells)
  Cells arena;       // arena arrays
  int64_t off;       // first arena cell
  double z_default;  // zmet when the caller passes none
  int32_t* remaining_slot;  // copy-in: set to n (may be null)
  uint32_t* claimed_slot;   // copy-in: set to 0 (may be null)
  unsigned long long* staged;  // copy-in: incremented once (may be null)
  int32_t ir_evolve;
};

// host-callable launchers (defined in sfk_serve.hip)
int served_blocks_per_cu(int precision);
hipError_t launch_served(const ServedArgs& a, int precision, int grid, hipStream_t s);
hipError_t launch_copy_in(const CopyArgs& a, hipStream_t s);
hipError_t launch_copy_out(const CopyArgs& a, hipStream_t s);

}  // namespace sfk
