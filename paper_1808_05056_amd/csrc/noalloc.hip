// The split-BF16 tile product on device pointers without device allocation.
//
// ooc_split_gemm_device allocates its slice workspace for each call.  Callers
// that cannot allocate device memory (code under stream capture, serving
// loops, harnesses that forbid it) use ooc_split_gemm_device_noalloc, which
// runs the same kernels with the workspace in a file-scope device array of
// OOC_NOALLOC_SCRATCH_BYTES.  Each device the library runs on holds its own
// copy of the array until the process ends.  Host code never uses the
// array's name as an address: its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and kept.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"
#include "kernels.hpp"

namespace ooc {
namespace {

constexpr int kMaxScratchDevices = 64;

__device__ __align__(256) unsigned char scratch[OOC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of this device's copy of `scratch`; the device is current.
ooc_status scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(OOC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return OOC_OK;
}

}  // namespace
}  // namespace ooc

using namespace ooc;

extern "C" {

ooc_status ooc_split_gemm_device_noalloc(int32_t device, int64_t m, int64_t n, int64_t k, int32_t s, double alpha,
                                         const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                                         double* C, int64_t ldc, void* stream) {
  if (m < 0 || n < 0 || k < 0) return fail(OOC_ERR_ARG, "negative size");
  if (s < 1 || s > 8) return fail(OOC_ERR_ARG, "slices must be 1..8");
  if (m == 0 || n == 0) return OOC_OK;
  if (!C || ldc < n) return fail(OOC_ERR_ARG, "bad C or ldc");
  if (k > 0 && (!A || !B || lda < k || ldb < n)) return fail(OOC_ERR_ARG, "bad A, B, lda or ldb");
  const size_t need = split_workspace_bytes(m, n, k, s, kSliceBF16);
  if (need > (size_t)OOC_NOALLOC_SCRATCH_BYTES)
    return fail(OOC_ERR_CAPACITY, "split workspace of " + std::to_string(need) + " bytes exceeds the " +
                                      std::to_string((size_t)OOC_NOALLOC_SCRATCH_BYTES) +
                                      "-byte static scratch buffer");
  if (device < 0 || device >= kMaxScratchDevices) return fail(OOC_ERR_NO_DEVICE, "device ordinal out of range");
  ooc_status st = use_device(device);
  if (st != OOC_OK) return st;
  void* ws = nullptr;
  st = scratch_address(device, &ws);
  if (st != OOC_OK) return st;
  // every buffer the kernels read is fully written first (slice planes with
  // their zero padding, exponents, column maxima, slice-sum tile), so the
  // previous call's contents need no clearing
  const hipError_t e = launch_split_gemm(kSliceBF16, m, n, k, s, alpha, A, lda, B, ldb, beta, C, ldc, 0.0, nullptr, 0,
                                         ws, (size_t)OOC_NOALLOC_SCRATCH_BYTES, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(OOC_ERR_HIP, std::string("split gemm launch: ") + hipGetErrorString(e));
  return OOC_OK;
}

}  // extern "C"
