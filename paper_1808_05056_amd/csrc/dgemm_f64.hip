// FP64 tile product on CDNA4 matrix cores: C = alpha*A*B + beta*C, row-major.
//
// This is the DGEMM stage of the paper's pipeline (Section V, stage
// "DGEMM" of Fig. 4), which the paper delegates to a vendor library.  Here it
// is a hand-written gfx950 kernel:
//   * a 256-thread workgroup (4 waves of 64) computes a 128 x 128 tile of C,
//     each wave a 64 x 64 quarter as 4 x 4 blocks of V_MFMA_F64_16X16X4_F64;
//   * K advances in steps of 16: the next step's A and B tiles are fetched
//     from global memory into registers (16-byte loads, coalesced along the
//     contiguous dimension) while the current step's tiles are multiplied
//     out of LDS; LDS is double-buffered so one barrier per step suffices;
//   * A is stored transposed in LDS (k-major) so that the 16 lanes feeding one
//     MFMA row read 16 consecutive doubles, like the B reads;
//   * workgroups are numbered so that each XCD (workgroups are dealt to the 8
//     XCDs round robin) receives a contiguous band of tiles, and tiles are
//     ordered in groups of rows so that concurrently running tiles share A
//     rows and B columns in that XCD's L2.
// Operand layout of V_MFMA_F64_16X16X4_F64 (one wave): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator element v of lane l is
// D[l/16 + 4v][l%16].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace ooc {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int PADA = 4, PADB = 4;
constexpr int NTHREADS = 256;
constexpr int GROUP_M = 8;

template <bool VEC>
__global__ __launch_bounds__(NTHREADS, 2) void dgemm_f64_mfma(
    int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A, int64_t lda,
    const double* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
    double gamma, const double* __restrict__ D, int64_t ldd, int tiles_m, int tiles_n) {
  __shared__ __attribute__((aligned(16))) double As[2][BK][BM + PADA];
  __shared__ __attribute__((aligned(16))) double Bs[2][BK][BN + PADB];

  // ---- tile selection: XCD bands, then row groups -------------------------------
  const int ntiles = tiles_m * tiles_n;
  const int b = blockIdx.x;
  const int xcd = b & 7, local = b >> 3;
  const int q = ntiles >> 3, r = ntiles & 7;
  const int lin = xcd * q + (xcd < r ? xcd : r) + local;
  const int group = lin / (GROUP_M * tiles_n);
  const int first_m = group * GROUP_M;
  const int gm = (tiles_m - first_m) < GROUP_M ? (tiles_m - first_m) : GROUP_M;
  const int in_group = lin - group * GROUP_M * tiles_n;
  const int tm = first_m + in_group % gm;
  const int tn = in_group / gm;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;

  // global-load assignment: A row ar, k offset ak (8 doubles); B k-row bk, column offset bn (8 doubles)
  const int ar = tid >> 1, ak = (tid & 1) * 8;
  const int bk = tid >> 4, bn = (tid & 15) * 8;

  const bool full_mn = (m0 + BM <= M) && (n0 + BN <= N);
  double ra[8], rb[8];

  auto gload = [&](int64_t k0) {
    const bool fast = full_mn && (k0 + BK <= K);
    const int64_t arow = m0 + ar;
    const int64_t brow = k0 + bk;
    if (fast) {
      const double* pa = A + arow * lda + k0 + ak;
      const double* pb = B + brow * ldb + n0 + bn;
      if (VEC) {
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          double2 va = *reinterpret_cast<const double2*>(pa + e);
          double2 vb = *reinterpret_cast<const double2*>(pb + e);
          ra[e] = va.x; ra[e + 1] = va.y;
          rb[e] = vb.x; rb[e + 1] = vb.y;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) { ra[e] = pa[e]; rb[e] = pb[e]; }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t kk = k0 + ak + e;
        ra[e] = (arow < M && kk < K) ? A[arow * lda + kk] : 0.0;
        const int64_t nn = n0 + bn + e;
        rb[e] = (brow < K && nn < N) ? B[brow * ldb + nn] : 0.0;
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) As[buf][ak + e][ar] = ra[e];
#pragma unroll
    for (int e = 0; e < 8; e += 2) *reinterpret_cast<double2*>(&Bs[buf][bk][bn + e]) = make_double2(rb[e], rb[e + 1]);
  };

  dbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (K + BK - 1) / BK;
  if (nk > 0) {
    gload(0);
    lstore(0);
    __syncthreads();
  }
  const int lrow = lane & 15, lk = lane >> 4;
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const int kk = s * 4 + lk;
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][kk][wm * 64 + i * 16 + lrow];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[buf][kk][wn * 64 + j * 16 + lrow];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: C = alpha*acc + beta*C + gamma*D (C, D not read when their weight is 0)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + wn * 64 + j * 16 + lrow;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 64 + i * 16 + lk + 4 * v;
        if (row < M && col < N) {
          double* pc = C + row * ldc + col;
          double val = alpha * acc[i][j][v];
          if (beta != 0.0) val += beta * *pc;
          if (gamma != 0.0) val += gamma * D[row * ldd + col];
          *pc = val;
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_dgemm_f64(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                            const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                            double gamma, const double* D, int64_t ldd, hipStream_t stream) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int tiles_m = (int)((m + BM - 1) / BM), tiles_n = (int)((n + BN - 1) / BN);
  const int64_t nt = (int64_t)tiles_m * tiles_n;
  if (nt > 0x7fffffff) return hipErrorInvalidValue;
  const bool vec = ((lda & 1) == 0) && ((ldb & 1) == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
  if (k <= 0) { A = nullptr; B = nullptr; }
  if (gamma == 0.0) D = nullptr;
  dim3 grid((unsigned)nt), block(NTHREADS);
  if (vec)
    hipLaunchKernelGGL(dgemm_f64_mfma<true>, grid, block, 0, stream, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                       gamma, D, ldd, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL(dgemm_f64_mfma<false>, grid, block, 0, stream, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                       gamma, D, ldd, tiles_m, tiles_n);
  return hipGetLastError();
}

}  // namespace ooc
