// FP64-accurate tile product from BF16 slices on CDNA4 matrix cores.
//
// The paper's DGEMM stage computes each tile in FP64 (Section V).  This is an
// alternative for the same stage: the error-free splitting of a matrix
// product into exactly computable slice products (Ozaki, Ogita, Oishi and
// Rump, Numer. Algorithms 59, 2012), with slices small enough that every
// slice product is exact on BF16 matrix cores with FP32 accumulation.
//
// For one K panel, A (m x k) and B (k x n):
//  1. e_i = smallest integer with max_k |A_ik| < 2^e_i; f_j likewise per column of B.
//  2. r = A_ik; for p = 1..s: m_p = rint(r * 2^(8p - e_i)), r -= m_p * 2^(e_i - 8p).
//     Each step is exact; |m_1| <= 256 and |m_p| <= 128 (p >= 2) are integers that
//     BF16 holds exactly.  Same for B with f_j.
//  3. For each weight t = p + q (2 <= t <= s+1), U_t = sum over p + q = t of
//     sum_k mA_p[i,k] mB_q[k,j].  Inside a chunk of 64 k every partial sum is an
//     integer below 2^24 (at most 64 * (2*2^15 + 6*2^14) for t <= 9, or
//     64 * 2^16 for t = 2), so the FP32 MFMA accumulation is exact; chunk sums
//     are added into U_t in FP64, also exactly.
//  4. S = sum over t from s+1 down to 2 of U_t * 2^(e_i + f_j - 8t), accumulated
//     in FP64 from the smallest weight to the largest.
//  5. C = alpha*S + beta*C + gamma*D with separate roundings (no fused
//     multiply-add), C not read when beta == 0, D not read when gamma == 0.
// A row or column holding a non-finite value gives NaN in its output row or
// column.
//
// Workspace layout (bytes): A planes [s][mpad][kpad] bf16, B planes
// [s][npad][kpad] bf16 (B transposed so MFMA operands are contiguous in k),
// row exponents [mpad] int32, column exponents [npad] int32, where mpad,
// npad and kpad are m, n and k rounded up to 64 and the padding is zero.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace ooc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int32_t kBad = 0x7fffffff;  // exponent marking a non-finite row or column

__device__ inline uint16_t bf16_bits_exact(double v) {
  // v is an integer of magnitude <= 256: exact in FP32, whose low 16 bits are then zero
  return (uint16_t)(__float_as_uint((float)v) >> 16);
}

__device__ inline int32_t exponent_of(double mx) {
  if (mx == 0.0) return 0;
  int ex = 0;
  (void)frexp(mx, &ex);  // mx = f * 2^ex with 0.5 <= f < 1, so mx < 2^ex and 2^(ex-1) <= mx
  return ex;
}

// One wave per row of A: exponent, then s slices of the row into the planes.
__global__ __launch_bounds__(256) void split_rows(int64_t m, int64_t k, const double* __restrict__ A, int64_t lda,
                                                  int s, int64_t mpad, int64_t kpad, uint16_t* __restrict__ planes,
                                                  int32_t* __restrict__ ex_out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= mpad) return;
  const bool live = row < m;
  double mx = 0.0;
  int bad = 0;
  if (live) {
    for (int64_t kk = lane; kk < k; kk += 64) {
      const double v = A[row * lda + kk];
      if (!isfinite(v)) bad = 1;
      mx = fmax(mx, fabs(v));
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off));
    bad |= __shfl_xor(bad, off);
  }
  const int32_t ex = bad ? kBad : exponent_of(mx);
  if (lane == 0) ex_out[row] = ex;
  for (int64_t kk = lane; kk < kpad; kk += 64) {
    double r = (live && !bad && kk < k) ? A[row * lda + kk] : 0.0;
    for (int p = 1; p <= s; ++p) {
      double mp = 0.0;
      if (r != 0.0) {
        mp = rint(ldexp(r, 8 * p - ex));
        r = r - ldexp(mp, ex - 8 * p);
      }
      planes[((int64_t)(p - 1) * mpad + row) * kpad + kk] = bf16_bits_exact(mp);
    }
  }
}

// Column maxima of |B| (k x n, row-major) as IEEE bit patterns, which order
// like the values for non-negative doubles (and put Inf and NaN above every
// finite value): a 2-D grid of 256 columns x 256 rows, combined with atomicMax.
__global__ __launch_bounds__(256) void zero_u64(uint64_t* __restrict__ x, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) x[i] = 0;
}

__global__ __launch_bounds__(256) void col_absmax(int64_t k, int64_t n, const double* __restrict__ B, int64_t ldb,
                                                  unsigned long long* __restrict__ mx) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.y * 256;
  if (j >= n) return;
  const int64_t k1 = k0 + 256 < k ? k0 + 256 : k;
  unsigned long long best = 0;
  for (int64_t kk = k0; kk < k1; ++kk) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(B[kk * ldb + j]));
    best = bits > best ? bits : best;
  }
  atomicMax(mx + j, best);
}

__global__ __launch_bounds__(256) void col_exponents(int64_t npad, const unsigned long long* __restrict__ mx,
                                                     int32_t* __restrict__ ex_out) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= npad) return;
  const unsigned long long bits = mx[j];
  ex_out[j] = bits >= 0x7ff0000000000000ull ? kBad : exponent_of(__longlong_as_double((long long)bits));
}

// Slices of B into transposed planes [p][j][k]: a 64 (k) x 64 (j) tile per workgroup.
__global__ __launch_bounds__(256) void split_cols(int64_t k, int64_t n, const double* __restrict__ B, int64_t ldb,
                                                  int s, int64_t npad, int64_t kpad, const int32_t* __restrict__ ex,
                                                  uint16_t* __restrict__ planes) {
  __shared__ double tile[64][65];
  const int t = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  // load: 16 rows of k per pass, 64 consecutive columns (coalesced)
  for (int rep = 0; rep < 16; ++rep) {
    const int kl = rep * 4 + (t >> 6), jl = t & 63;
    const int64_t kk = k0 + kl, j = j0 + jl;
    tile[jl][kl] = (kk < k && j < n) ? B[kk * ldb + j] : 0.0;
  }
  __syncthreads();
  const int jl = t >> 2, ks = (t & 3) * 16;
  const int64_t j = j0 + jl;
  const int32_t e = ex[j];
  for (int q = 0; q < 16; ++q) {
    const int kl = ks + q;
    double r = (e == kBad) ? 0.0 : tile[jl][kl];
    for (int p = 1; p <= s; ++p) {
      double mp = 0.0;
      if (r != 0.0) {
        mp = rint(ldexp(r, 8 * p - e));
        r = r - ldexp(mp, e - 8 * p);
      }
      planes[((int64_t)(p - 1) * npad + j) * kpad + k0 + kl] = bf16_bits_exact(mp);
    }
  }
}

// Slice products: 4 waves in 2 x 2, each a 32 x 32 output block (one MFMA block).
// Operand layout of V_MFMA_F32_32X32X16_BF16: lane l supplies A[l%32][8*(l/32) .. +8]
// and B[8*(l/32) .. +8][l%32]; accumulator element v of lane l is
// D[8*(v/4) + 4*(l/32) + v%4][l%32].
__global__ __launch_bounds__(256) void split_gemm(int64_t m, int64_t n, int64_t kpad, int s,
                                                  const uint16_t* __restrict__ Ap, const uint16_t* __restrict__ Bp,
                                                  int64_t mpad, int64_t npad, const int32_t* __restrict__ ea,
                                                  const int32_t* __restrict__ fb, double alpha, double beta,
                                                  double* __restrict__ C, int64_t ldc, double gamma,
                                                  const double* __restrict__ D, int64_t ldd) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.y * 64 + (w >> 1) * 32;
  const int64_t col0 = (int64_t)blockIdx.x * 64 + (w & 1) * 32;
  const int64_t arow = row0 + (lane & 31), bcol = col0 + (lane & 31);
  const int koff = 8 * (lane >> 5);
  double S[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) S[v] = 0.0;
  int32_t er[16], fc;
#pragma unroll
  for (int v = 0; v < 16; ++v) er[v] = ea[row0 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4)];
  fc = fb[bcol];
  for (int t = s + 1; t >= 2; --t) {
    double U[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) U[v] = 0.0;
    const int plo = t - s > 1 ? t - s : 1, phi = t - 1 < s ? t - 1 : s;
    for (int64_t kc = 0; kc < kpad; kc += 64) {
      f32x16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.f;
      for (int p = plo; p <= phi; ++p) {
        const int q = t - p;
        const uint16_t* pa = Ap + ((int64_t)(p - 1) * mpad + arow) * kpad + kc + koff;
        const uint16_t* pb = Bp + ((int64_t)(q - 1) * npad + bcol) * kpad + kc + koff;
#pragma unroll
        for (int kk = 0; kk < 64; kk += 16) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(pa + kk);
          const bf16x8 b = *reinterpret_cast<const bf16x8*>(pb + kk);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) U[v] += (double)acc[v];
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int32_t ee = er[v];
      if (ee != kBad && fc != kBad) S[v] = S[v] + ldexp(U[v], ee + fc - 8 * t);
    }
  }
  const int64_t col = bcol;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t row = row0 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
    if (row < m && col < n) {
      double val;
      if (er[v] == kBad || fc == kBad) {
        val = __builtin_nan("");
      } else {
        val = __dmul_rn(alpha, S[v]);
        if (beta != 0.0) val = __dadd_rn(val, __dmul_rn(beta, C[row * ldc + col]));
        if (gamma != 0.0) val = __dadd_rn(val, __dmul_rn(gamma, D[row * ldd + col]));
      }
      C[row * ldc + col] = val;
    }
  }
}

inline int64_t pad64(int64_t x) { return (x + 63) / 64 * 64; }

}  // namespace

size_t split_workspace_bytes(int64_t m, int64_t n, int64_t k, int s) {
  const int64_t mp = pad64(m), np = pad64(n), kp = pad64(k);
  return (size_t)(2 * s * (mp + np) * kp + 4 * (mp + np) + 8 * np);
}

hipError_t launch_split_gemm(int64_t m, int64_t n, int64_t k, int s, double alpha, const double* A, int64_t lda,
                             const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double gamma,
                             const double* D, int64_t ldd, void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (s < 1 || s > 8) return hipErrorInvalidValue;
  if (k <= 0) return launch_dgemm_f64(m, n, 0, alpha, nullptr, 1, nullptr, 1, beta, C, ldc, gamma, D, ldd, stream);
  const int64_t mp = pad64(m), np = pad64(n), kp = pad64(k);
  if (split_workspace_bytes(m, n, k, s) > ws_bytes) return hipErrorInvalidValue;
  uint16_t* Ap = static_cast<uint16_t*>(workspace);
  uint16_t* Bp = Ap + (size_t)s * mp * kp;
  int32_t* ea = reinterpret_cast<int32_t*>(Bp + (size_t)s * np * kp);
  int32_t* fb = ea + mp;
  unsigned long long* bmax = reinterpret_cast<unsigned long long*>(fb + np);  // 8-byte aligned: mp, np even
  if (gamma == 0.0) D = nullptr;
  hipLaunchKernelGGL(split_rows, dim3((unsigned)(mp / 4)), dim3(256), 0, stream, m, k, A, lda, s, mp, kp, Ap, ea);
  hipLaunchKernelGGL(zero_u64, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, stream,
                     reinterpret_cast<uint64_t*>(bmax), np);
  hipLaunchKernelGGL(col_absmax, dim3((unsigned)((n + 255) / 256), (unsigned)((k + 255) / 256)), dim3(256), 0, stream,
                     k, n, B, ldb, bmax);
  hipLaunchKernelGGL(col_exponents, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, stream, np, bmax, fb);
  hipLaunchKernelGGL(split_cols, dim3((unsigned)(kp / 64), (unsigned)(np / 64)), dim3(256), 0, stream, k, n, B, ldb, s,
                     np, kp, fb, Bp);
  hipLaunchKernelGGL(split_gemm, dim3((unsigned)(np / 64), (unsigned)(mp / 64)), dim3(256), 0, stream, m, n, kp, s, Ap,
                     Bp, mp, np, ea, fb, alpha, beta, C, ldc, gamma, D, ldd);
  return hipGetLastError();
}

}  // namespace ooc
