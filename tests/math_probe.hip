// math_probe.hip -- test-only library: runs the kernels' hand-written
// binary64 math (fexp, flog, frcp, fsqrt of sfk_lane.h) over an array, so
// that tests can hold each to its stated accuracy against references of
// high precision.  Built next to the tests by the package build.
#include "sfk_lane.h"

namespace sfk {
namespace {
__global__ __launch_bounds__(256) void math_probe_kernel(const double* x, double* out, int64_t n,
                                                         int fn) {
  stage_tables();  // every thread: ends with a barrier
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  double r;
  if (fn == 0) r = fexp(v);
  else if (fn == 1) r = flog(v);
  else if (fn == 2) r = frcp(v);
  else r = fsqrt(v);
  out[i] = r;
}
}  // namespace
}  // namespace sfk

// fn: 0 e^x, 1 ln x, 2 1/x, 3 sqrt x; x, out device arrays of n doubles.
// Returns 0, or -1 for a bad argument, or the HIP error of the launch.
extern "C" int sfk_math_probe(const double* x, double* out, int64_t n, int fn, void* stream) {
  if (n < 0 || fn < 0 || fn > 3 || (n > 0 && (!x || !out))) return -1;
  if (n == 0) return 0;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return -1;
  hipLaunchKernelGGL(sfk::math_probe_kernel, dim3(unsigned(blocks)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), x, out, n, fn);
  return int(hipGetLastError());
}
