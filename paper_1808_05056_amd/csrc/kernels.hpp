// Launchers of the device kernels (all enqueue on the given stream and return
// the launch status; none synchronises).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ooc.h"

namespace ooc {

// C = alpha*A*op(B) + beta*C + gamma*D, FP64 on matrix cores (row-major; k == 0
// gives beta*C + gamma*D; C is not read when beta == 0, D not when gamma == 0).
// op(B) = B (k x n, ldb >= n) or, with transb, B^T (B stored n x k, ldb >= k).
// Elements (r, c) with r - c < tri are neither read nor written (tri =
// kNoTri: all are): a block at (i0, j0) of a lower-triangular result uses
// tri = j0 - i0.
constexpr int64_t kNoTri = INT64_MIN;
hipError_t launch_dgemm_f64(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                            const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                            double gamma, const double* D, int64_t ldd, hipStream_t stream, bool transb = false,
                            int64_t tri = kNoTri);

// Split tile product (s slices of BF16 or INT8, by bytes per slice element):
// same result contract as launch_dgemm_f64 up to the split scheme's error;
// uses `workspace` (split_workspace_bytes).  K is processed in panels of at
// most kSplitMaxK (exact int32 slice sums):
// C = alpha*S_0 + beta*C + gamma*D, then C = alpha*S_p + C.
enum SliceFormat { kSliceInt8 = 1, kSliceBF16 = 2 };
inline SliceFormat slice_format(int precision) { return precision == OOC_SPLIT_INT8 ? kSliceInt8 : kSliceBF16; }
constexpr int64_t kSplitMaxK = 8192;
size_t split_workspace_bytes(int64_t m, int64_t n, int64_t k, int s, SliceFormat f);
// Whether the INT8 slice products of an m x n block run on 256 x 256 tiles
// (else 256 x 128) on a device of `cus` compute units.
bool split_i8_wide(int64_t m, int64_t n, int cus);
// Optional timing of the slice-product kernels alone (slicing kernels
// excluded): events[2x] and events[2x+1] are recorded around the x-th
// slice-product launch, for x < count; `used` counts the launches made.
struct KernelTimer {
  hipEvent_t* events = nullptr;
  int count = 0;
  int used = 0;
};
// Number of slice-product launches a split product over k makes.
inline int64_t split_launches(int64_t k) { return k <= 0 ? 0 : (k + kSplitMaxK - 1) / kSplitMaxK; }
// With transb, B is stored transposed (n x k, ldb >= k).
hipError_t launch_split_gemm(SliceFormat f, int64_t m, int64_t n, int64_t k, int s, double alpha, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                             double gamma, const double* D, int64_t ldd, void* workspace, size_t ws_bytes,
                             hipStream_t stream, KernelTimer* timer = nullptr, bool transb = false,
                             bool reuse_a = false, bool reuse_b = false);

// The planner network (see mlp.hip): parameter count, scratch size (floats)
// for a batch of n, forward pass into y, loss and gradient, one Adam step.
int64_t mlp_param_count(int d, int H);
int64_t mlp_scratch_floats(int64_t n, int d, int H);
hipError_t launch_mlp_forward(int64_t n, int d, int H, const float* params, const float* X, float* scratch,
                              float* y_out, hipStream_t s);
hipError_t launch_mlp_grad(int64_t n, int d, int H, const float* params, const float* X, const float* t, float wd,
                           float* scratch, float* grad, float* loss, hipStream_t s);
hipError_t launch_adam(int64_t count, float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);

// Cholesky pieces on device blocks (chol.hip), row-major FP64:
// A = L L^T in place for the n x n block A (lower triangle; the strict upper
// triangle untouched); a pivot that is not positive sets *status (if still 0)
// to col_base + its column + 1.  X <- X L^{-T} (rlt) or X <- X L^{-1} (rln)
// for the m x n block X and the n x n lower-triangular L.
hipError_t launch_potrf_lower(int64_t n, double* A, int64_t lda, double* status, int64_t col_base, hipStream_t s);
hipError_t launch_trsm_rlt(int64_t m, int64_t n, double* X, int64_t ldx, const double* L, int64_t ldl,
                           hipStream_t s);
hipError_t launch_trsm_rln(int64_t m, int64_t n, double* X, int64_t ldx, const double* L, int64_t ldl,
                           hipStream_t s);

// Device-to-device copy kernel (bytes and pointers multiples of 16).
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// Race testing (stress.hip): a wait of about `microseconds` (at most 5000) on
// the stream, and a NaN fill of n doubles.
hipError_t launch_spin(uint32_t microseconds, hipStream_t s);
hipError_t launch_fill_nan(double* x, int64_t n, hipStream_t s);

}  // namespace ooc
