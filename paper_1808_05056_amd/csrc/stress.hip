// Timing perturbation for race testing: a bounded spin on one stream, and a
// NaN fill that poisons the device arena before an operation list runs.  With
// delays of random length inserted before random operations, every ordering
// the waits of an operation list allow becomes likely; a missing wait then
// shows as a result that differs from the undelayed run (or as NaN, when a
// kernel reads a buffer before its copy arrived).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace ooc {
namespace {

// One wave waits until `ticks` of the constant 100 MHz wall clock have passed,
// or `max_iter` sleep steps, whichever comes first: it always ends.
__global__ __launch_bounds__(64) void spin(uint64_t ticks, uint32_t max_iter) {
  const uint64_t t0 = wall_clock64();
  for (uint32_t it = 0; it < max_iter; ++it) {
    if (wall_clock64() - t0 >= ticks) break;
    __builtin_amdgcn_s_sleep(8);
  }
}

__global__ __launch_bounds__(256) void fill_nan(double* __restrict__ x, int64_t n) {
  const double v = __builtin_nan("");
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] = v;
}

}  // namespace

hipError_t launch_spin(uint32_t microseconds, hipStream_t s) {
  const uint32_t us = microseconds > 5000 ? 5000 : microseconds;
  // a sleep step of 8 x 64 cycles is at least ~0.2 us at 2.4 GHz: the
  // iteration bound ends the wait within about twice its length even if the
  // clock read stalls
  hipLaunchKernelGGL(spin, dim3(1), dim3(64), 0, s, (uint64_t)us * 100u, us * 8u + 64u);
  return hipGetLastError();
}

hipError_t launch_fill_nan(double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(fill_nan, dim3((unsigned)blocks), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

}  // namespace ooc
