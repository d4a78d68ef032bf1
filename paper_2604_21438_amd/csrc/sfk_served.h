// sfk_served.h -- internal interface between the served-form scheduler
// (sfserve.cpp) and its kernels (sfk_serve.hip).
#pragma once
#include "sfk.h"

namespace sfk {

// Served form.  A request is staged on the copy stream: its cells are
// copied into the arena (unless it continues a resident block), then an arm
// kernel writes the request's descriptor into its ring slot in device
// memory and arms the slot's claim word.  The host then raises the published
// count of the request's claim class (coherent pinned host memory), one
// request at a time in sequence order.  Waves claim cells of the oldest
// request of the highest class that has unclaimed cells: a device head index
// per class names that request, and the slot's claim word hands out its
// cells with one atomicAdd.  The claim word carries the low 32 bits of the
// request's sequence number beside the count, so a wave that still holds an
// older request of the same slot (the host arms a slot again only once its
// previous request is done) sees the mismatch in the word it got back, and
// the cells it was handed are the newer request's, which it serves.  The
// lane that stores a request's last cell raises its done word.
constexpr int kClasses = 8;    // claim classes; finer AMR levels are served first
constexpr int kRingMax = 16384;  // largest ring (slots per class)

struct SlotMeta {             // written by the arm kernel, read by the drain
  uint64_t seq;               // request sequence number in its class; ~0 while rewritten
  uint64_t off;               // first arena cell
  uint64_t n;                 // cells (> 0, < 2^31)
  double dt;                  // interval [s]
  uint64_t level;             // AMR level, clamped to 0..255
};

struct ServedArgs {
  Net net;
  Par par;
  Cells arena;                        // arena SoA arrays (n = capacity)
  const SlotMeta* meta;               // device, kClasses * ring, class-major
  unsigned long long* claimed;        // device, per slot: seq tag << 32 | cells handed out
  int32_t* remaining;                 // device, per slot: cells not yet stored
  const uint64_t* published;          // host-mapped, kClasses: requests published per class
  unsigned long long* head;           // device, kClasses: oldest request that may have unclaimed cells
  unsigned long long* seen;           // device, kClasses: largest published count read so far
  const unsigned long long* staged;   // device, kClasses: requests armed
  unsigned long long* newest;         // device: largest launch generation started (this precision)
  const uint64_t* gen;                // host-mapped, per drain slot: generation of its latest launch
  uint64_t* left;                     // host-mapped, per drain slot: 1 once a wave of its latest launch has exited
  uint64_t* done;                     // host-mapped, per ring slot: seq + 1 when complete
  uint64_t ring;                      // slots per class, a power of two
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

// Copy of cells between caller buffers and the arena (copy-in, copy-out,
// fetch).  Caller arrays that are NULL are skipped.
struct CopyArgs {
  Cells user;        // caller buffers (n = request cells)
  Cells arena;       // arena arrays
  int64_t off;       // first arena cell
  double z_default;  // zmet when the caller passes none
  int32_t ir_evolve;
};

// Arming of one ring slot for a staged request.
struct ArmArgs {
  SlotMeta* meta;
  unsigned long long* claimed;
  int32_t* remaining;
  unsigned long long* staged;  // the class's armed-request count
  uint64_t seq, off, n, level;
  double dt;
};

// host-callable launchers (defined in sfk_serve.hip)
int served_blocks_per_cu(int precision, bool stand_ins);
hipError_t launch_served(const ServedArgs& a, int precision, int grid, hipStream_t s);
hipError_t launch_copy_in(const CopyArgs& a, hipStream_t s);
hipError_t launch_copy_out(const CopyArgs& a, hipStream_t s);
hipError_t launch_arm(const ArmArgs& a, hipStream_t s);

}  // namespace sfk
