// sfserve.h -- served form (continuous batching of AMR blocks): request
// queue, HBM-budget admission into a device arena, resident block keys,
// persistent drain kernel replayed as a HIP graph, completion and latency
// bookkeeping.  The admission and bookkeeping logic is the host-only core
// of sfsched.h; this layer implements its device actions with HIP.
#pragma once
#include <stdint.h>

#include <string>

#include "sfchem.h"
#include "sfk_served.h"

namespace sfserve {

struct Config {
  int device = 0;
  uint64_t budget_bytes = 0;
  sfk::Net net{};
  sfk::Par par{};
  int cus = 0;
  int refill_min = 1;
  const sfk::Net* netc = nullptr;  // device copies owned by the context
  const sfk::Par* parc = nullptr;
};

struct Server;

// Allocates the arena (budget_bytes of device memory), the ring slots and
// the drain graphs, and starts the scheduler thread.
Server* create(const Config& cfg, std::string* err, int* code);
int64_t capacity(const Server* s);  // arena capacity in cells
int submit(Server* s, const sfc_request& req, uint64_t* ticket, std::string* err);
int poll(Server* s, uint64_t ticket, sfc_result* out);
int fetch(Server* s, uint64_t ticket, const sfc_cells& dst, void* hip_stream, std::string* err);
int release(Server* s, uint64_t key, std::string* err);
int drain(Server* s, std::string* err);
void destroy(Server* s);
double now();

}  // namespace sfserve
