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
//   trsm back: X <- X L^{-1} (the backward solve of ooc_trsm_ex and ooc_potrs).
// potrf walks blocks of 64 columns right-looking (factor the diagonal block,
// solve the rows below, A22 <- A22 - A21 A21^T on the lower triangle); the
// solves recurse on halves (forward: trsm on X1 = X[:, :n1]; X2 <- X2 - X1
// L21^T; trsm on X2; backward: trsm on X2, X1 <- X1 - X2 L21, trsm on X1).  Nearly all their flops run in the FP64 matrix-core tile kernel;
// blocks of at most 64 columns are finished by the leaf kernels below.  Every quotient is a true division (no reciprocal), so integer
// inputs whose factor is integer give it exactly.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace ooc {
namespace {

constexpr int kLeaf = 64;   // potrf leaf: one wave, row l of the block in lane l's registers
constexpr int kLeafT = 64;  // trsm leaf: 64 columns, one wave of 64 lanes
constexpr int kBatch = 16;  // L values read from LDS together by the leaves

// v from lane `lane` (wave-uniform), read into scalar registers.
__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One wave factors an n x n block (n <= 64), right-looking: lane l holds row
// l of the block in registers (rows and columns beyond n are the identity,
// which factors to itself).  For each column j: the pivot comes from lane j,
// every lane below divides its entry of the column by the pivot's square
// root, and lane l updates its row, a_lc -= a_lj L_cj for j < c <= l, with
// the column L_.j shared through LDS.  A pivot that is not positive (or not finite) stops
// the factorisation; the first failing column + 1 + col_base is written to
// *status if it is still 0.  The block moves through LDS on the way in and
// out so that the global accesses are row-contiguous.
__global__ __launch_bounds__(64) void potrf_leaf(int n, double* __restrict__ A, int64_t lda,
                                                 double* __restrict__ status, int64_t col_base) {
  __shared__ double t[kLeaf][kLeaf + 1];
  __shared__ double col[kLeaf];
  const int l = threadIdx.x;
  {
    // every lane loads from an address inside the block (clamped) and then
    // selects, so that the 64 loads are all in flight at once
    const int lc = l < n ? l : n - 1;
    double v[kLeaf];
#pragma unroll
    for (int r = 0; r < kLeaf; ++r) v[r] = A[(r < n ? r : n - 1) * lda + lc];
#pragma unroll
    for (int r = 0; r < kLeaf; ++r) t[r][l] = (r < n && l <= r) ? v[r] : (l == r ? 1.0 : 0.0);
  }
  __syncthreads();
  double a[kLeaf];
#pragma unroll
  for (int c = 0; c < kLeaf; ++c) a[c] = t[l][c];
  // a failing pivot is recorded and the (then meaningless) arithmetic runs on,
  // so that the loops stay straight-line code
  int bad = -1;
#pragma clang loop unroll(full)
  for (int j = 0; j < kLeaf; ++j) {
    const double d = lane_value(a[j], j);
    if (bad < 0 && (!(d > 0.0) || !isfinite(d))) bad = j;
    const double piv = sqrt(d);
    if (l == j) a[j] = piv;
    if (l > j) a[j] = a[j] / piv;
    // column j of L through LDS (one wave: its LDS operations run in order),
    // read back in batches of 16 words whose reads are in flight together
    col[l] = a[j];
    __syncthreads();
#pragma clang loop unroll(full)
    for (int c0 = j + 1; c0 < kLeaf; c0 += kBatch) {
      double lv[kBatch];
#pragma unroll
      for (int t = 0; t < kBatch; ++t)
        if (c0 + t < kLeaf) lv[t] = col[c0 + t];
#pragma unroll
      for (int t = 0; t < kBatch; ++t)
        if (c0 + t < kLeaf && l >= c0 + t) a[c0 + t] = a[c0 + t] - a[j] * lv[t];
    }
    __syncthreads();
  }
  if (bad >= 0) {
    if (l == 0 && *status == 0.0) *status = (double)(col_base + bad + 1);
    return;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kLeaf; ++c) t[l][c] = a[c];
  __syncthreads();
  for (int r = 0; r < n; ++r)
    if (l <= r) A[r * lda + l] = t[r][l];
}

// X <- X L^{-T} (forward, BACK false) or X <- X L^{-1} (BACK true) for X
// (m x n, n <= 64): a wave holds 16 rows of X, four lanes per row, lane q of
// a row holding its columns 16q .. 16q+15 in registers, and substitutes
// right-looking.  Forward: for k = 0, 1, ...: x_k = x_k / L_kk, then x_j =
// x_j - x_k L_jk for j > k.  Backward: for k = n-1, n-2, ...: x_k = x_k /
// L_kk, then x_j = x_j - x_k L_kj for j < k.  The lane holding column k
// divides, the quotient goes to the row's other lanes by a DPP quad
// broadcast, and every lane updates its columns (the updates of one k are
// independent).  Four lanes per row give a launch four times the waves of
// one lane per row (the chunks of a panel's rows run a few thousand rows per
// launch).  The L values of one k (column k of L forward, row k backward) sit
// in a row of LDS, identity beyond n, each 16-column segment padded by one
// word so that the four lanes of a row read distinct banks; the rows of X
// move through LDS so that the global accesses are row-contiguous.
constexpr int kLeafRows = 16;  // rows of X per trsm leaf wave
__device__ __forceinline__ int lseg(int j) { return j + (j >> 4); }

// v from lane Q of each quad of lanes, to every lane of that quad.
template <int Q>
__device__ __forceinline__ double quad_bcast(double v) {
  constexpr int ctrl = Q | (Q << 2) | (Q << 4) | (Q << 6);  // quad_perm [Q, Q, Q, Q]
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, ctrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <bool BACK>
__device__ __forceinline__ void trsm_leaf_body(int64_t m, int n, double* __restrict__ X, int64_t ldx,
                                               const double* __restrict__ L, int64_t ldl) {
  __shared__ double lt[kLeafT][kLeafT + 4];        // forward lt[k][lseg(j)] = L_jk, backward L_kj
  __shared__ double xs[kLeafRows][kLeafT + 1];     // the block's rows
  const int l = threadIdx.x, r = l >> 2, q = l & 3;
  const int64_t row0 = (int64_t)blockIdx.x * kLeafRows;
  {
    // every lane loads from an address inside L and X (clamped) and then
    // selects, so that the loads are all in flight at once; lane l reads
    // column l of L, v[j] = L_jl, and column l of the block's rows
    const int lc = l < n ? l : n - 1;
    double v[kLeafT];
#pragma unroll
    for (int j = 0; j < kLeafT; ++j) v[j] = L[(j < n ? j : n - 1) * ldl + lc];
#pragma unroll
    for (int j = 0; j < kLeafT; ++j) {
      const double e = (j < n && l <= j) ? v[j] : (j == l ? 1.0 : 0.0);
      if (BACK)
        lt[j][lseg(l)] = e;
      else
        lt[l][lseg(j)] = e;
    }
    double w[kLeafRows];
#pragma unroll
    for (int rr = 0; rr < kLeafRows; ++rr) w[rr] = X[(row0 + rr < m ? row0 + rr : m - 1) * ldx + lc];
#pragma unroll
    for (int rr = 0; rr < kLeafRows; ++rr) xs[rr][l] = (row0 + rr < m && l < n) ? w[rr] : 0.0;
  }
  __syncthreads();
  double x[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) x[t] = xs[r][16 * q + t];
#pragma clang loop unroll(full)
  for (int i = 0; i < kLeafT; ++i) {
    const int k = BACK ? kLeafT - 1 - i : i;
    const int qk = k >> 4, c = k & 15;
    const double own = x[c] / lt[k][lseg(k)];  // the quotient, in the lanes that hold column k
    double xk;
    switch (qk) {
      case 0: xk = quad_bcast<0>(own); break;
      case 1: xk = quad_bcast<1>(own); break;
      case 2: xk = quad_bcast<2>(own); break;
      default: xk = quad_bcast<3>(own); break;
    }
    if (q == qk) x[c] = xk;
    double lv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) lv[t] = lt[k][lseg(16 * q + t)];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int j = 16 * q + t;
      if (BACK ? j < k : j > k) x[t] = x[t] - xk * lv[t];
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) xs[r][16 * q + t] = x[t];
  __syncthreads();
  for (int rr = 0; rr < kLeafRows; ++rr)
    if (row0 + rr < m && l < n) X[(row0 + rr) * ldx + l] = xs[rr][l];
}

__global__ __launch_bounds__(64) void trsm_leaf(int64_t m, int n, double* __restrict__ X, int64_t ldx,
                                                const double* __restrict__ L, int64_t ldl) {
  trsm_leaf_body<false>(m, n, X, ldx, L, ldl);
}

__global__ __launch_bounds__(64) void trsm_leaf_back(int64_t m, int n, double* __restrict__ X, int64_t ldx,
                                                     const double* __restrict__ L, int64_t ldl) {
  trsm_leaf_body<true>(m, n, X, ldx, L, ldl);
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
    hipLaunchKernelGGL(trsm_leaf, dim3((unsigned)((m + kLeafRows - 1) / kLeafRows)), dim3(kLeafT), 0, s, m, (int)n, X,
                       ldx, L, ldl);
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

hipError_t launch_trsm_rln(int64_t m, int64_t n, double* X, int64_t ldx, const double* L, int64_t ldl,
                           hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (n <= kLeafT) {
    hipLaunchKernelGGL(trsm_leaf_back, dim3((unsigned)((m + kLeafRows - 1) / kLeafRows)), dim3(kLeafT), 0, s, m, (int)n,
                       X, ldx, L, ldl);
    return hipGetLastError();
  }
  // Y L = X with L = [L11 0; L21 L22]: Y2 = X2 L22^{-1}, then Y1 = (X1 - Y2 L21) L11^{-1}
  const int64_t n1 = half_of(n, kLeafT), n2 = n - n1;
  hipError_t e = launch_trsm_rln(m, n2, X + n1, ldx, L + n1 * ldl + n1, ldl, s);
  // X1 <- X1 - X2 L21
  if (e == hipSuccess)
    e = launch_dgemm_f64(m, n1, n2, -1.0, X + n1, ldx, L + n1 * ldl, ldl, 1.0, X, ldx, 0.0, nullptr, 0, s);
  if (e == hipSuccess) e = launch_trsm_rln(m, n1, X, ldx, L, ldl, s);
  return e;
}

// Right-looking over blocks of kLeaf columns: factor the diagonal block (one
// wave), solve the rows below against it (one leaf launch over all of them),
// and update the trailing lower triangle with one product.  Three launches of
// wide grids per block instead of the many narrow ones of a recursion on
// halves.
hipError_t launch_potrf_lower(int64_t n, double* A, int64_t lda, double* status, int64_t col_base, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int64_t k0 = 0; k0 < n && e == hipSuccess; k0 += kLeaf) {
    const int64_t kb = n - k0 < kLeaf ? n - k0 : kLeaf, m2 = n - k0 - kb;
    double* Akk = A + k0 * lda + k0;
    hipLaunchKernelGGL(potrf_leaf, dim3(1), dim3(64), 0, s, (int)kb, Akk, lda, status, col_base + k0);
    e = hipGetLastError();
    if (m2 == 0 || e != hipSuccess) break;
    double* A21 = Akk + kb * lda;
    e = launch_trsm_rlt(m2, kb, A21, lda, Akk, lda, s);
    // A22 <- A22 - A21 A21^T on and below the diagonal
    if (e == hipSuccess)
      e = launch_dgemm_f64(m2, m2, kb, -1.0, A21, lda, A21, lda, 1.0, A21 + kb, lda, 0.0, nullptr, 0, s, true, 0);
  }
  return e;
}

}  // namespace ooc
