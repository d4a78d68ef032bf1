// sched_sim.cpp -- the served form's host scheduler core (sfsched) driven
// against a simulated device on the CPU.
//
// The simulated device keeps one value per arena cell.  A copy-in writes
// the caller's values into the request's range, the drain replaces every
// cell x of a published request by x / 2 + dt, a copy-out or fetch reads
// the range back.  Every result can therefore be predicted exactly, and the
// simulation checks, at each device action:
//   - no two requests in flight share an arena cell, and the arena is never
//     over-committed;
//   - a ring slot is armed again only after the request that held it is
//     done, and publication follows staging, one request at a time in
//     sequence order per (precision, class);
//   - a block key keeps its range across its requests, and its requests
//     run one after the other;
// and at the end that every request completed with the predicted values.
// Scenarios: queued admission under a tight budget with a small ring, claim
// classes by level, resident block keys (continue, write back, fetch,
// release), keys that hold the whole arena, and the API's error cases.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "sfsched.h"

using namespace sfsched;

#define CHECK(c)                                                             \
  do {                                                                       \
    if (!(c)) {                                                              \
      std::fprintf(stderr, "CHECK failed at %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                          \
    }                                                                        \
  } while (0)

struct User {            // a caller's request buffers
  std::vector<double> buf;
};

struct SimReq {          // what the device knows of a request
  Req* r = nullptr;
  long t_staged = -1, t_done = -1, t_copied = -1;
  bool published = false, done = false;
  User* user = nullptr;
};

class Sim : public Ops {
 public:
  Sim(int64_t cap, uint32_t ring, int classes, unsigned seed)
      : arena(size_t(cap), std::nan("")), owner(size_t(cap), 0), ring_(ring), rng(seed) {
    slot_owner.resize(2);
    for (auto& v : slot_owner) v.assign(size_t(classes) * ring, 0);
    published.assign(2, std::vector<uint64_t>(size_t(classes), 0));
  }
  std::vector<double> arena;
  std::vector<uint64_t> owner;  // ticket of the request in flight on each cell, 0 if none
  uint32_t ring_;
  std::mt19937 rng;
  long tick = 0;
  std::map<uint64_t, SimReq> reqs;                 // by ticket
  std::vector<std::vector<uint64_t>> slot_owner;   // ticket that armed each slot last
  std::vector<std::vector<uint64_t>> published;
  std::map<std::pair<int, uint64_t>, uint64_t> by_seq;  // (prec*64 + cls, seq) -> ticket
  int64_t busy_cells = 0;
  std::map<uint64_t, int64_t> key_off;             // first range seen per block key

  int delay(int lo, int hi) { return std::uniform_int_distribution<int>(lo, hi)(rng); }

  int stage(Req& r, size_t slot) override {
    SimReq& s = reqs[r.ticket];
    s.r = &r;
    s.user = static_cast<User*>(r.dev);
    // the slot's previous request must be done before it is armed again
    const uint64_t prev = slot_owner[size_t(r.prec)][slot];
    if (prev) CHECK(reqs.count(prev) && reqs[prev].done);
    slot_owner[size_t(r.prec)][slot] = r.ticket;
    CHECK(slot == size_t(r.cls) * ring_ + (r.seq & (ring_ - 1)));
    by_seq[{r.prec * 64 + r.cls, r.seq}] = r.ticket;
    // exclusive use of the range while in flight; a key keeps its range
    CHECK(r.off >= 0 && r.off + r.n <= int64_t(arena.size()));
    for (int64_t i = 0; i < r.n; ++i) {
      CHECK(owner[size_t(r.off + i)] == 0);
      owner[size_t(r.off + i)] = r.ticket;
    }
    busy_cells += r.n;
    CHECK(busy_cells <= int64_t(arena.size()));
    if (r.key) {
      auto it = key_off.find(r.key);
      if (it == key_off.end()) key_off[r.key] = r.off;
      else CHECK(it->second == r.off);
    }
    CHECK(r.copy_in == (s.user != nullptr && !r.resume));
    s.t_staged = tick + delay(0, 3);
    return kOk;
  }
  int staged(Req& r) override {
    SimReq& s = reqs[r.ticket];
    if (tick < s.t_staged) return 0;
    if (r.copy_in && !s.published && s.t_staged >= 0) {
      for (int64_t i = 0; i < r.n; ++i) arena[size_t(r.off + i)] = s.user->buf[size_t(i)];
    }
    return 1;
  }
  void publish(int prec, int cls, uint64_t count) override {
    auto& p = published[size_t(prec)][size_t(cls)];
    CHECK(count == p + 1);
    p = count;
    const uint64_t t = by_seq.at({prec * 64 + cls, count - 1});
    SimReq& s = reqs[t];
    CHECK(tick >= s.t_staged);
    s.published = true;
    s.t_done = tick + delay(1, 25);
  }
  // the drain: published requests finish at their time, in any order
  void advance() {
    ++tick;
    for (auto& kv : reqs) {
      SimReq& s = kv.second;
      if (s.published && !s.done && tick >= s.t_done) {
        const Req& r = *s.r;
        for (int64_t i = 0; i < r.n; ++i) {
          double& x = arena[size_t(r.off + i)];
          x = 0.5 * x + r.dt;
        }
        s.done = true;
      }
    }
  }
  bool done(const Req& r, size_t) override { return reqs[r.ticket].done; }
  int copy_out(Req& r) override {
    SimReq& s = reqs[r.ticket];
    CHECK(s.done && s.user);
    s.t_copied = tick + delay(0, 3);
    for (int64_t i = 0; i < r.n; ++i) s.user->buf[size_t(i)] = arena[size_t(r.off + i)];
    return kOk;
  }
  int copied_out(Req& r) override { return tick >= reqs[r.ticket].t_copied ? 1 : 0; }
  void retire(Req& r) override {
    for (int64_t i = 0; i < r.n; ++i) {
      CHECK(owner[size_t(r.off + i)] == r.ticket);
      owner[size_t(r.off + i)] = 0;
    }
    busy_cells -= r.n;
  }
  double now() override { return double(tick); }
};

static double f_step(double x, double dt) { return 0.5 * x + dt; }

// Run the core until every submitted ticket is done; submissions may be
// staggered through `arrive` (tick -> requests).
struct Harness {
  Core core;
  Sim sim;
  std::vector<std::unique_ptr<User>> users;
  Harness(int64_t cap, uint32_t ring, int classes, bool by_level, unsigned seed)
      : core(cap, ring, classes, by_level), sim(cap, ring, classes, seed) {}

  uint64_t submit(Req* r, const std::vector<double>* init, int expect = kOk) {
    if (init) {
      users.push_back(std::make_unique<User>());
      users.back()->buf = *init;
      r->dev = users.back().get();
    }
    std::string err;
    const int rc = core.submit(r, sim.now(), &err);
    if (rc != expect) std::fprintf(stderr, "submit: %d (%s), expected %d\n", rc, err.c_str(), expect);
    CHECK(rc == expect);
    if (rc != kOk) delete r;
    return rc == kOk ? r->ticket : 0;
  }
  void run_until_idle(long limit = 200000) {
    std::string fatal;
    for (long i = 0; i < limit && !core.idle(); ++i) {
      core.step(sim, &fatal);
      CHECK(fatal.empty());
      sim.advance();
    }
    CHECK(core.idle());
  }
};

static std::vector<double> initial(uint64_t tag, int64_t n) {
  std::vector<double> v(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) v[size_t(i)] = double(tag) * 1000.0 + double(i);
  return v;
}

// Many unkeyed requests against a small arena and ring: queueing, arrival
// order, exact results.
static void scenario_tight_budget(bool by_level) {
  Harness h(1000, 4, 8, by_level, 7);
  std::mt19937 rng(11);
  struct Exp { uint64_t t; std::vector<double> want; User* u; };
  std::vector<Exp> ex;
  std::string fatal;
  for (int q = 0; q < 300; ++q) {
    Req* r = new Req();
    r->prec = q % 2;
    r->level = int(rng() % 6);
    r->n = 1 + int64_t(rng() % 400);
    r->dt = 1.0 + double(q % 5);
    auto init = initial(uint64_t(q + 1), r->n);
    const uint64_t t = h.submit(r, &init);
    std::vector<double> want(init.size());
    for (size_t i = 0; i < init.size(); ++i) want[i] = f_step(init[i], r->dt);
    ex.push_back({t, want, h.users.back().get()});
    // staggered arrivals
    for (int k = 0; k < int(rng() % 4); ++k) {
      h.core.step(h.sim, &fatal);
      CHECK(fatal.empty());
      h.sim.advance();
    }
  }
  h.run_until_idle();
  for (auto& e : ex) {
    Req out;
    CHECK(h.core.poll(e.t, &out) == kOk);
    CHECK(out.t_submit <= out.t_admit && out.t_admit <= out.t_done);
    CHECK(e.u->buf == e.want);
  }
  std::printf("PASS tight budget%s: 300 requests through a 1000-cell arena and 4-slot rings\n",
              by_level ? " (classes by level)" : "");
}

// Block keys: each block advanced over several substeps with its state
// resident, interleaved with unkeyed traffic; results fetched, written
// back, and the keys released.
static void scenario_keys() {
  const int nkeys = 12, nsub = 6;
  Harness h(4000, 8, 8, false, 3);
  std::mt19937 rng(5);
  std::vector<int64_t> kn(nkeys);
  std::vector<std::vector<double>> state(nkeys);
  std::vector<uint64_t> last(nkeys);
  std::string fatal;
  for (int k = 0; k < nkeys; ++k) {
    kn[size_t(k)] = 16 + int64_t(rng() % 120);
    state[size_t(k)] = initial(uint64_t(5000 + k), kn[size_t(k)]);
  }
  std::vector<std::pair<uint64_t, std::vector<double>>> unkeyed;
  std::vector<User*> unkeyed_users;
  std::vector<std::pair<User*, std::vector<double>>> written;  // write-back buffers
  for (int s = 0; s < nsub; ++s) {
    for (int k = 0; k < nkeys; ++k) {
      Req* r = new Req();
      r->key = 100 + uint64_t(k);
      r->prec = k % 2;
      r->level = k % 6;
      r->dt = 0.25 * double(s + 1);
      r->resume = s > 0;
      r->writeback = (s == nsub - 1) && (k % 3 == 0);
      r->n = r->resume ? 0 : kn[size_t(k)];
      std::vector<double> buf = state[size_t(k)];
      last[size_t(k)] = h.submit(r, (!r->resume || r->writeback) ? &buf : nullptr);
      for (auto& x : state[size_t(k)]) x = f_step(x, 0.25 * double(s + 1));
      if (r->writeback) written.push_back({h.users.back().get(), state[size_t(k)]});
    }
    // unkeyed traffic between the substeps
    for (int q = 0; q < 10; ++q) {
      Req* r = new Req();
      r->n = 1 + int64_t(rng() % 300);
      r->dt = 3.0;
      r->prec = q % 2;
      auto init = initial(uint64_t(9000 + s * 10 + q), r->n);
      const uint64_t t = h.submit(r, &init);
      std::vector<double> want(init.size());
      for (size_t i = 0; i < init.size(); ++i) want[i] = f_step(init[i], 3.0);
      unkeyed.push_back({t, want});
      unkeyed_users.push_back(h.users.back().get());
    }
    for (int k = 0; k < 30; ++k) {
      h.core.step(h.sim, &fatal);
      CHECK(fatal.empty());
      h.sim.advance();
    }
  }
  h.run_until_idle();
  for (size_t i = 0; i < unkeyed.size(); ++i) CHECK(unkeyed_users[i]->buf == unkeyed[i].second);
  for (int k = 0; k < nkeys; ++k) {
    int64_t off = -1, n = 0;
    std::string err;
    CHECK(h.core.fetch_range(last[size_t(k)], &off, &n, &err) == kOk);
    CHECK(n == kn[size_t(k)] && off == h.sim.key_off.at(100 + uint64_t(k)));
    for (int64_t i = 0; i < n; ++i) CHECK(h.sim.arena[size_t(off + i)] == state[size_t(k)][size_t(i)]);
    Req out;
    CHECK(h.core.poll(last[size_t(k)], &out) == kOk);
    // still fetchable after the poll, until the key moves on or is released
    CHECK(h.core.fetch_range(last[size_t(k)], &off, &n, &err) == kOk);
  }
  // write-back requests put the final state into the caller's buffers
  CHECK(!written.empty());
  for (auto& w : written) CHECK(w.first->buf == w.second);
  CHECK(h.core.resident_cells() > 0);
  for (int k = 0; k < nkeys; ++k) {
    std::string err;
    CHECK(h.core.release(100 + uint64_t(k), &err) == kOk);
    int64_t off, n;
    CHECK(h.core.fetch_range(last[size_t(k)], &off, &n, &err) == kState);
  }
  CHECK(h.core.resident_cells() == 0);
  std::printf("PASS block keys: %d blocks x %d substeps resident, %zu unkeyed requests between\n",
              nkeys, nsub, unkeyed.size());
}

// Resident keys fill most of the arena: a request that cannot fit waits,
// the keys' continued substeps still run (they need no room), and after the
// keys are released the waiting request runs.
static void scenario_keys_hold_arena() {
  Harness h(1000, 4, 8, false, 9);
  std::string fatal;
  std::vector<uint64_t> t0;
  for (int k = 0; k < 3; ++k) {
    Req* r = new Req();
    r->key = 1 + uint64_t(k);
    r->n = 300;
    r->dt = 1.0;
    auto init = initial(uint64_t(k + 1), 300);
    t0.push_back(h.submit(r, &init));
  }
  h.run_until_idle();
  Req* big = new Req();
  big->n = 500;
  big->dt = 1.0;
  auto init = initial(77, 500);
  const uint64_t tb = h.submit(big, &init);
  // continued substeps of every key behind the waiting request
  std::vector<uint64_t> t1;
  for (int k = 0; k < 3; ++k) {
    Req* r = new Req();
    r->key = 1 + uint64_t(k);
    r->resume = true;
    r->dt = 2.0;
    t1.push_back(h.submit(r, nullptr));
  }
  for (int i = 0; i < 2000; ++i) {
    h.core.step(h.sim, &fatal);
    h.sim.advance();
  }
  Req out;
  for (uint64_t t : t1) CHECK(h.core.poll(t, &out) == kOk);
  CHECK(h.core.poll(tb, &out) == kPending);
  std::string err;
  CHECK(h.core.release(1, &err) == kOk);
  for (int i = 0; i < 200; ++i) {
    h.core.step(h.sim, &fatal);
    h.sim.advance();
  }
  CHECK(h.core.poll(tb, &out) == kPending);  // 300 and 100 free cells apart: no room yet
  CHECK(h.core.release(2, &err) == kOk);
  h.run_until_idle();
  CHECK(h.core.poll(tb, &out) == kOk);
  std::printf("PASS keys holding the arena: continued substeps run while a larger request waits\n");
}

static void scenario_errors() {
  Harness h(1000, 4, 8, false, 1);
  std::string err;
  std::vector<double> ten(10, 1.0);
  Req* r = new Req();
  r->key = 5;
  r->resume = true;
  h.submit(r, nullptr, kState);  // nothing resident under key 5
  r = new Req();
  r->resume = true;
  r->n = 10;
  h.submit(r, &ten, kInval);  // continuing needs a key
  r = new Req();
  r->n = int64_t(1) << 31;
  h.submit(r, nullptr, kInval);  // beyond the 32-bit claim counters
  r = new Req();
  r->n = 1001;
  h.submit(r, nullptr, kBudget);  // larger than the arena
  r = new Req();
  r->n = 0;
  h.submit(r, nullptr, kInval);
  r = new Req();
  r->prec = 2;
  r->n = 4;
  h.submit(r, nullptr, kInval);
  r = new Req();
  r->key = 5;
  r->n = 10;
  r->dt = 1.0;
  const uint64_t t1 = h.submit(r, &ten);
  int64_t off, n;
  CHECK(h.core.fetch_range(t1, &off, &n, &err) == kPending);
  r = new Req();
  r->key = 5;
  r->n = 11;
  h.submit(r, nullptr, kInval);  // a key keeps its cell count
  h.run_until_idle();
  CHECK(h.core.fetch_range(t1, &off, &n, &err) == kOk && n == 10);
  r = new Req();
  r->key = 5;
  r->resume = true;
  r->dt = 1.0;
  const uint64_t t2 = h.submit(r, nullptr);
  CHECK(h.core.fetch_range(t1, &off, &n, &err) == kState);  // superseded
  CHECK(h.core.release(6, &err) == kInval);
  CHECK(h.core.release(5, &err) == kOk);                    // deferred: t2 in flight
  r = new Req();
  r->key = 5;
  r->resume = true;
  h.submit(r, nullptr, kState);                             // key being released
  h.run_until_idle();
  Req out;
  CHECK(h.core.poll(t2, &out) == kOk);
  CHECK(h.core.poll(t2, &out) == kInval);
  CHECK(h.core.resident_cells() == 0);
  std::printf("PASS errors: unknown key, missing key, 2^31 cells, over budget, empty, precision, "
              "cell count of a key, superseded fetch, release\n");
}

// A block's substeps all submitted at once: they must run one after the
// other on the same range, each on the state the previous one left.
static void scenario_key_burst() {
  Harness h(2000, 4, 8, true, 21);
  const int nkeys = 6, nsub = 8;
  std::vector<std::vector<double>> state(nkeys);
  std::vector<uint64_t> last(nkeys);
  for (int k = 0; k < nkeys; ++k) {
    state[size_t(k)] = initial(uint64_t(300 + k), 50 + 10 * k);
    for (int s = 0; s < nsub; ++s) {
      Req* r = new Req();
      r->key = 40 + uint64_t(k);
      r->level = s % 6;
      r->prec = (k + s) % 2;
      r->dt = 1.0 + s;
      r->resume = s > 0;
      r->n = r->resume ? 0 : int64_t(state[size_t(k)].size());
      std::vector<double> buf = state[size_t(k)];
      last[size_t(k)] = h.submit(r, r->resume ? nullptr : &buf);
      for (auto& x : state[size_t(k)]) x = f_step(x, 1.0 + s);
    }
  }
  h.run_until_idle();
  for (int k = 0; k < nkeys; ++k) {
    int64_t off, n;
    std::string err;
    CHECK(h.core.fetch_range(last[size_t(k)], &off, &n, &err) == kOk);
    for (int64_t i = 0; i < n; ++i) CHECK(h.sim.arena[size_t(off + i)] == state[size_t(k)][size_t(i)]);
  }
  std::printf("PASS key bursts: %d blocks with %d substeps each submitted at once\n", nkeys, nsub);
}

int main() {
  scenario_key_burst();
  scenario_tight_budget(false);
  scenario_tight_budget(true);
  scenario_keys();
  scenario_keys_hold_arena();
  scenario_errors();
  std::printf("ALL PASS\n");
  return 0;
}
