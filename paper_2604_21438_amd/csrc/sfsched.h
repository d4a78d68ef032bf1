// sfsched.h -- host-side core of the served form: request bookkeeping,
// admission against the HBM budget into ranges of the device arena, ring
// slots, resident block keys, publication order and completion.
//
// No HIP here.  Every device action goes through the Ops interface, which
// the library implements with HIP kernels and events (sfserve.cpp) and the
// CPU tests with a simulated device, so the admission logic is exercised on
// the host alone.  The Core is not thread-safe: its owner serialises calls.
#pragma once
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

namespace sfsched {

// status codes (the values of sfchem.h)
constexpr int kOk = 0, kInval = -1, kNomem = -2, kBudget = -3, kDevice = -4, kPending = -5,
              kState = -7;

enum class St { Pending, Staging, Running, CopyOut, Done };

struct Req {
  // set by the caller before submit
  int prec = 0;          // 0 binary64, 1 mixed
  int level = 0;         // AMR level (claim class when classes are by level)
  int64_t n = 0;         // cells; for a continued key 0 means the key's count
  double dt = 0.0;
  uint64_t key = 0;      // block key, 0 = none
  bool resume = false;   // continue from the key's resident state (no upload)
  bool writeback = false;  // keyed: copy results back into the caller's buffers too
  uint64_t tag = 0;      // the caller's, returned unchanged
  void* dev = nullptr;   // owned by the Ops implementation (caller buffers, events)
  // set by the core
  uint64_t ticket = 0;
  int cls = 0;           // claim class
  uint64_t seq = 0;      // sequence number in its (precision, class) ring
  int64_t off = -1;      // first arena cell
  bool copy_in = true, copy_out = true;
  St st = St::Pending;
  int status = kPending;
  bool done_seen = false;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
};

class Ops {
 public:
  virtual ~Ops() = default;
  // Upload r's cells into its arena range when r.copy_in, then arm ring
  // slot `slot` for r (its descriptor and counters); queued work, 0 or an
  // error code.
  virtual int stage(Req& r, size_t slot) = 0;
  virtual int staged(Req& r) = 0;      // 1 complete, 0 not yet, < 0 error
  // requests of (prec, cls) published so far; raised in sequence order
  virtual void publish(int prec, int cls, uint64_t count) = 0;
  virtual bool done(const Req& r, size_t slot) = 0;  // the device finished r
  virtual int copy_out(Req& r) = 0;    // results into the caller's buffers
  virtual int copied_out(Req& r) = 0;  // 1 complete, 0 not yet, < 0 error
  virtual void retire(Req& r) = 0;     // r is done: release per-request resources
  virtual double now() = 0;
};

// First-fit allocator of contiguous arena cell ranges.
class Ranges {
 public:
  void reset(int64_t cap);
  int64_t alloc(int64_t n);  // first cell, or -1
  void release(int64_t off, int64_t n);
  int64_t free_cells() const;

 private:
  std::map<int64_t, int64_t> free_;
};

struct Key {
  int64_t off = -1;           // arena range (allocated at the first admission)
  int64_t n = 0;
  std::deque<Req*> chain;     // requests of the key not yet done, in submit order
  uint64_t last_ticket = 0;   // the key's latest request (fetch target)
  bool releasing = false;
};

class Core {
 public:
  // capacity: arena cells; ring: slots per (precision, class) ring, a
  // power of two >= 2; classes: claim classes per precision; by_level:
  // class = AMR level (clamped), else every request in class 0.
  Core(int64_t capacity, uint32_t ring, int classes, bool by_level);
  ~Core();

  int64_t capacity() const { return cap_; }
  uint32_t ring() const { return ring_; }
  int classes() const { return classes_; }
  size_t slot_of(const Req& r) const {
    return size_t(r.cls) * ring_ + size_t(r.seq & (ring_ - 1));
  }

  // ---- caller side ----
  // Validates and queues r (the core owns it from here); sets r->ticket.
  int submit(Req* r, double now, std::string* err);
  // Done: fills *out (a copy) and frees the request; kPending if not done;
  // kInval for an unknown ticket.
  int poll(uint64_t ticket, Req* out);
  // The arena range holding the results of a keyed request that is done
  // and is still its key's latest request.
  int fetch_range(uint64_t ticket, int64_t* off, int64_t* n, std::string* err) const;
  // Give a key's range back once its requests are done.
  int release(uint64_t key, std::string* err);
  int64_t outstanding() const { return outstanding_; }
  bool idle() const { return outstanding_ == 0 && pending_.empty(); }

  // ---- scheduler side ----
  // One pass: completions, publication, admission.  Returns true if
  // anything moved; on a device error returns false with *fatal set.
  bool step(Ops& ops, std::string* fatal);
  // After a device error: every request still outstanding fails.
  void fail_all(int status, double now);
  int64_t running(int prec) const { return running_[prec]; }
  uint64_t published_total(int prec) const { return pub_total_[prec]; }
  int64_t resident_cells() const;  // cells held by keys (admitted or done)

 private:
  bool admit(Ops& ops, std::string* fatal);
  void finish(Ops& ops, Req* r, int status);

  int64_t cap_;
  uint32_t ring_;
  int classes_;
  bool by_level_;
  Ranges ranges_;
  uint64_t next_ticket_ = 1;
  int64_t outstanding_ = 0;
  std::unordered_map<uint64_t, Req*> tickets_;
  std::unordered_map<uint64_t, Key> keys_;
  std::unordered_map<uint64_t, uint64_t> key_of_ticket_;  // latest ticket of each key
  std::deque<Req*> pending_, staging_, copyout_;
  // per precision: next sequence number and in-flight requests per class
  std::vector<uint64_t> next_seq_[2];
  std::vector<std::deque<Req*>> inflight_[2];
  int64_t running_[2] = {0, 0};
  uint64_t pub_total_[2] = {0, 0};
};

}  // namespace sfsched
