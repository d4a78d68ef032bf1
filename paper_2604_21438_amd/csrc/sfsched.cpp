// sfsched.cpp -- host-side core of the served form (see sfsched.h).
#include "sfsched.h"

#include <iterator>

namespace sfsched {

void Ranges::reset(int64_t cap) {
  free_.clear();
  if (cap > 0) free_[0] = cap;
}

int64_t Ranges::alloc(int64_t n) {
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

void Ranges::release(int64_t off, int64_t n) {
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

int64_t Ranges::free_cells() const {
  int64_t s = 0;
  for (const auto& kv : free_) s += kv.second;
  return s;
}

Core::Core(int64_t capacity, uint32_t ring, int classes, bool by_level)
    : cap_(capacity), ring_(ring), classes_(classes), by_level_(by_level) {
  ranges_.reset(cap_);
  for (int p = 0; p < 2; ++p) {
    next_seq_[p].assign(size_t(classes_), 0);
    inflight_[p].resize(size_t(classes_));
  }
}

Core::~Core() {
  for (auto& kv : tickets_) delete kv.second;
}

int Core::submit(Req* r, double now, std::string* err) {
  auto bad = [&](int code, const char* msg) {
    if (err) *err = msg;
    return code;
  };
  if (r->prec != 0 && r->prec != 1) return bad(kInval, "unknown precision");
  if (r->n < 0 || r->n >= (int64_t(1) << 31))
    return bad(kInval, "a request holds between 1 and 2^31 - 1 cells");
  Key* k = nullptr;
  if (r->key == 0) {
    if (r->resume) return bad(kInval, "continuing a block needs its block key");
    if (r->n == 0) return bad(kInval, "empty request");
    r->copy_in = true;
    r->copy_out = true;
  } else {
    auto it = keys_.find(r->key);
    if (it != keys_.end()) {
      k = &it->second;
      if (k->releasing) return bad(kState, "block key is being released");
      if (r->resume && r->n == 0) r->n = k->n;
      if (r->n != k->n) return bad(kInval, "a block key keeps its cell count (release it first)");
    } else {
      if (r->resume) return bad(kState, "no resident state for this block key");
      if (r->n == 0) return bad(kInval, "empty request");
    }
    r->copy_in = !r->resume;
    r->copy_out = r->writeback;
  }
  if (r->n > cap_) return bad(kBudget, "request larger than the whole arena");
  if (r->key != 0 && !k) {
    k = &keys_[r->key];
    k->n = r->n;
  }
  r->cls = by_level_ ? (r->level < 0 ? 0 : r->level >= classes_ ? classes_ - 1 : r->level) : 0;
  r->ticket = next_ticket_++;
  r->st = St::Pending;
  r->status = kPending;
  r->done_seen = false;
  r->off = -1;
  r->t_submit = now;
  tickets_[r->ticket] = r;
  outstanding_ += 1;
  pending_.push_back(r);
  if (k) {
    k->chain.push_back(r);
    if (k->last_ticket) key_of_ticket_.erase(k->last_ticket);
    k->last_ticket = r->ticket;
    key_of_ticket_[r->ticket] = r->key;
  }
  return kOk;
}

int Core::poll(uint64_t ticket, Req* out) {
  auto it = tickets_.find(ticket);
  if (it == tickets_.end()) return kInval;
  Req* r = it->second;
  if (r->st != St::Done) return kPending;
  *out = *r;
  tickets_.erase(it);
  delete r;
  return out->status;
}

int Core::fetch_range(uint64_t ticket, int64_t* off, int64_t* n, std::string* err) const {
  auto kt = key_of_ticket_.find(ticket);
  if (kt == key_of_ticket_.end()) {
    if (err) *err = "not the latest request of a resident block key";
    return tickets_.count(ticket) || ticket < next_ticket_ ? kState : kInval;
  }
  auto rt = tickets_.find(ticket);
  if (rt != tickets_.end() && rt->second->st != St::Done) return kPending;
  if (rt != tickets_.end() && rt->second->status != kOk) {
    if (err) *err = "the request failed";
    return kState;
  }
  const Key& k = keys_.at(kt->second);
  *off = k.off;
  *n = k.n;
  return kOk;
}

int Core::release(uint64_t key, std::string* err) {
  auto it = keys_.find(key);
  if (it == keys_.end() || it->second.releasing) {
    if (err) *err = "unknown block key";
    return kInval;
  }
  Key& k = it->second;
  k.releasing = true;
  if (k.last_ticket) key_of_ticket_.erase(k.last_ticket);
  if (k.chain.empty()) {
    if (k.off >= 0) ranges_.release(k.off, k.n);
    keys_.erase(it);
  }
  return kOk;
}

int64_t Core::resident_cells() const {
  int64_t s = 0;
  for (const auto& kv : keys_)
    if (kv.second.off >= 0) s += kv.second.n;
  return s;
}

void Core::finish(Ops& ops, Req* r, int status) {
  r->st = St::Done;
  r->status = status;
  r->t_done = ops.now();
  outstanding_ -= 1;
  if (r->key == 0) {
    ranges_.release(r->off, r->n);
  } else {
    auto it = keys_.find(r->key);
    Key& k = it->second;
    if (!k.chain.empty() && k.chain.front() == r) k.chain.pop_front();
    if (k.releasing && k.chain.empty()) {
      if (k.off >= 0) ranges_.release(k.off, k.n);
      keys_.erase(it);
    }
  }
  ops.retire(*r);
}

bool Core::admit(Ops& ops, std::string* fatal) {
  bool moved = false;
  bool alloc_blocked = false;  // an earlier request waits for arena room
  for (auto it = pending_.begin(); it != pending_.end();) {
    Req* r = *it;
    auto& fl = inflight_[r->prec][size_t(r->cls)];
    // a ring slot is reused only after the request that held it is done
    if (!fl.empty() && next_seq_[r->prec][size_t(r->cls)] - fl.front()->seq >= ring_) {
      ++it;
      continue;
    }
    int64_t off = -1;
    if (r->key != 0) {
      Key& k = keys_.at(r->key);
      if (k.chain.front() != r) {  // an earlier request of this block is not done
        ++it;
        continue;
      }
      if (k.off < 0) {
        if (alloc_blocked || (k.off = ranges_.alloc(k.n)) < 0) {
          alloc_blocked = true;
          ++it;
          continue;
        }
      }
      off = k.off;
    } else {
      // requests that need arena room are admitted in arrival order
      if (alloc_blocked || (off = ranges_.alloc(r->n)) < 0) {
        alloc_blocked = true;
        ++it;
        continue;
      }
    }
    r->off = off;
    r->seq = next_seq_[r->prec][size_t(r->cls)]++;
    r->t_admit = ops.now();
    r->st = St::Staging;
    const int rc = ops.stage(*r, slot_of(*r));
    if (rc != kOk) {
      if (fatal) *fatal = "stage: device error";
      return false;
    }
    fl.push_back(r);
    staging_.push_back(r);
    it = pending_.erase(it);
    moved = true;
  }
  return moved;
}

bool Core::step(Ops& ops, std::string* fatal) {
  bool moved = false;
  // 1. finished copy-outs (the copy stream is in order)
  while (!copyout_.empty()) {
    Req* r = copyout_.front();
    const int q = ops.copied_out(*r);
    if (q < 0) {
      if (fatal) *fatal = "copy-out: device error";
      return false;
    }
    if (q == 0) break;
    copyout_.pop_front();
    finish(ops, r, kOk);
    moved = true;
  }
  // 2. requests the device finished
  for (int p = 0; p < 2; ++p) {
    for (auto& fl : inflight_[p]) {
      for (Req* r : fl) {
        if (r->st != St::Running || r->done_seen) continue;
        if (!ops.done(*r, slot_of(*r))) continue;
        r->done_seen = true;
        running_[p] -= 1;
        moved = true;
        if (r->copy_out) {
          if (ops.copy_out(*r) != kOk) {
            if (fatal) *fatal = "copy-out launch: device error";
            return false;
          }
          r->st = St::CopyOut;
          copyout_.push_back(r);
        } else {
          finish(ops, r, kOk);
        }
      }
      while (!fl.empty() && fl.front()->done_seen) fl.pop_front();
    }
  }
  // 3. staged requests are published in admission order
  while (!staging_.empty()) {
    Req* r = staging_.front();
    const int q = ops.staged(*r);
    if (q < 0) {
      if (fatal) *fatal = "copy-in: device error";
      return false;
    }
    if (q == 0) break;
    staging_.pop_front();
    r->st = St::Running;
    running_[r->prec] += 1;
    pub_total_[r->prec] += 1;
    ops.publish(r->prec, r->cls, r->seq + 1);
    moved = true;
  }
  // 4. admission
  std::string f;
  const bool admitted = admit(ops, &f);
  if (!f.empty()) {
    if (fatal) *fatal = f;
    return false;
  }
  return moved || admitted;
}

void Core::fail_all(int status, double now) {
  for (auto& kv : tickets_) {
    Req* r = kv.second;
    if (r->st != St::Done) {
      r->st = St::Done;
      r->status = status;
      r->t_done = now;
    }
  }
  outstanding_ = 0;
  pending_.clear();
  staging_.clear();
  copyout_.clear();
}

}  // namespace sfsched
