// Cholesky factorisation and triangular solve of device-resident blocks.
//
// The paper names dense factorisations built on the out-of-core product as
// the next use of its method (Section VII).  The out-of-core Cholesky
// factorisation moves one block column at a time through the device: the
// column's update by the columns to its left is an out-of-core product
// (C = C - A B^T with a lower-triangle mask), and the column itself is
// factored on the device by the two operations here:
//   potrf: A = L L^T in place for an n x n block (lower triangle read and
//          written; the strict upper triangle is neither);
//   trsm:  X <- X L^{-T} for an m x n block X and an n x n lower-triangular L
//          (the column's rows below its diagonal block).
// Both recurse on halves: potrf(A11); A21 <- A21 L11^{-T}; A22 <- A22 - A21 A21^T
// (lower triangle); potrf(A22), and trsm on X1 = X[:, :n1]; X2 <- X2 - X1 L21^T;
// trsm on X2, so nearly all their flops run in the FP64 matrix-core tile
// kernel; blocks of at most 64 columns are finished by the leaf kernels
// below.  Every quotient is a true division (no reciprocal), so integer
// inputs whose factor is integer give it exactly.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace ooc {
namespace {

constexpr int kLeaf = 64;   // potrf leaf: one wave, the block in LDS
constexpr int kLeafT = 64;  // trsm leaf: one thread per row of X, rows and L in LDS
constexpr int kLeafRows = 64;  // rows of X per trsm-leaf workgroup (one wave: more workgroups per leaf)

// One wave factors an n x n block (n <= 64) held in LDS, column by column:
// pivot, scale the column below it, update the trailing lower triangle.  A
// pivot that is not positive (or not finite) stops the factorisation; the
// first failing column + 1 + col_base is written to *status if it is still 0.
__global__ __launch_bounds__(64) void potrf_leaf(int n, double* __restrict__ A, int64_t lda,
                                                 double* __restrict__ status, int64_t col_base) {
  __shared__ double a[kLeaf][kLeaf + 1];
  const int l = threadIdx.x;
  for (int r = 0; r < n; ++r)
    if (l <= r) a[r][l] = A[r * lda + l];
  __syncthreads();
  int bad = -1;
  for (int j = 0; j < n && bad < 0; ++j) {
    const double d = a[j][j];
    if (!(d > 0.0) || !isfinite(d)) {
      bad = j;
      break;
    }
    const double piv = sqrt(d);
    __syncthreads();
    if (l == j) a[j][j] = piv;
    if (l > j && l < n) a[l][j] = a[l][j] / piv;
    __syncthreads();
    // row l of the trailing triangle: a[l][c] -= a[l][j] a[c][j], j < c <= l
    if (l > j && l < n) {
      const double lj = a[l][j];
      for (int c = j + 1; c <= l; ++c) a[l][c] = a[l][c] - lj * a[c][j];
    }
    __syncthreads();
  }
  if (bad >= 0) {
    if (l == 0 && *status == 0.0) *status = (double)(col_base + bad + 1);
    return;
  }
  for (int r = 0; r < n; ++r)
    if (l <= r) A[r * lda + l] = a[r][l];
}

// X <- X L^{-T} for X (m x n, n <= 64): each thread solves one row,
// x_j = (x_j - sum_{k<j} x_k L_jk) / L_jj, with L and the rows in LDS (a
// thread's row as a column of xs, so the threads read consecutive words).
__global__ __launch_bounds__(kLeafRows) void trsm_leaf(int64_t m, int n, double* __restrict__ X, int64_t ldx,
                                                       const double* __restrict__ L, int64_t ldl) {
  __shared__ double lt[kLeafT][kLeafT + 1];
  __shared__ double xs[kLeafT][kLeafRows];
  for (int e = threadIdx.x; e < kLeafT * kLeafT; e += kLeafRows) {
    const int r = e / kLeafT, c = e % kLeafT;
    lt[r][c] = (r < n && c <= r) ? L[r * ldl + c] : (r == c ? 1.0 : 0.0);
  }
  const int t = threadIdx.x;
  const int64_t row = (int64_t)blockIdx.x * kLeafRows + t;
  double* xr = X + row * ldx;
  const bool live = row < m;
  for (int j = 0; j < n; ++j) xs[j][t] = live ? xr[j] : 0.0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double s = xs[j][t];
    for (int k = 0; k < j; ++k) s = s - xs[k][t] * lt[j][k];
    xs[j][t] = s / lt[j][j];
  }
  if (live)
    for (int j = 0; j < n; ++j) xr[j] = xs[j][t];
}

// split point of n columns: a multiple of `leaf` near the middle
int64_t half_of(int64_t n, int64_t leaf) {
  const int64_t h = (n / 2 + leaf - 1) / leaf * leaf;
  return h < n ? h : n - leaf;
}

}  // namespace

hipError_t launch_trsm_rlt(int64_t m, int64_t n, double* X, int64_t ldx, const double* L, int64_t ldl,
                           hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (n <= kLeafT) {
    hipLaunchKernelGGL(trsm_leaf, dim3((unsigned)((m + kLeafRows - 1) / kLeafRows)), dim3(kLeafRows), 0, s, m,
                       (int)n, X, ldx, L, ldl);
    return hipGetLastError();
  }
  const int64_t n1 = half_of(n, kLeafT), n2 = n - n1;
  hipError_t e = launch_trsm_rlt(m, n1, X, ldx, L, ldl, s);
  // X2 <- X2 - X1 L21^T
  if (e == hipSuccess)
    e = launch_dgemm_f64(m, n2, n1, -1.0, X, ldx, L + n1 * ldl, ldl, 1.0, X + n1, ldx, 0.0, nullptr, 0, s, true);
  if (e == hipSuccess) e = launch_trsm_rlt(m, n2, X + n1, ldx, L + n1 * ldl + n1, ldl, s);
  return e;
}

hipError_t launch_potrf_lower(int64_t n, double* A, int64_t lda, double* status, int64_t col_base, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n <= kLeaf) {
    hipLaunchKernelGGL(potrf_leaf, dim3(1), dim3(64), 0, s, (int)n, A, lda, status, col_base);
    return hipGetLastError();
  }
  const int64_t n1 = half_of(n, kLeaf), n2 = n - n1;
  hipError_t e = launch_potrf_lower(n1, A, lda, status, col_base, s);
  if (e == hipSuccess) e = launch_trsm_rlt(n2, n1, A + n1 * lda, lda, A, lda, s);
  // A22 <- A22 - A21 A21^T on and below the diagonal
  if (e == hipSuccess)
    e = launch_dgemm_f64(n2, n2, n1, -1.0, A + n1 * lda, lda, A + n1 * lda, lda, 1.0, A + n1 * lda + n1, lda, 0.0,
                         nullptr, 0, s, true, 0);
  if (e == hipSuccess) e = launch_potrf_lower(n2, A + n1 * lda + n1, lda, status, col_base + n1, s);
  return e;
}

}  // namespace ooc
