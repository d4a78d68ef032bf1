// sfserve.cpp -- served form (work in progress: not started yet).
#include "sfserve.h"

#include <chrono>

namespace sfserve {

struct Server {};

Server* create(const Config&, std::string* err) {
  if (err) *err = "served form not built";
  return nullptr;
}
int submit(Server*, const sfc_request&, uint64_t*, std::string* err) {
  if (err) *err = "served form not built";
  return SFC_E_STATE;
}
int poll(Server*, uint64_t, sfc_result*) { return SFC_E_STATE; }
int drain(Server*, std::string*) { return SFC_OK; }
void destroy(Server*) {}
double now() {
  using C = std::chrono::steady_clock;
  return std::chrono::duration<double>(C::now().time_since_epoch()).count();
}

}  // namespace sfserve
