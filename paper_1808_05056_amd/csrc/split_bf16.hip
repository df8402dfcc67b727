// FP64-accurate tile product from BF16 or INT8 slices on CDNA4 matrix cores.
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
//     sum_k mA_p[i,k] mB_q[k,j].  A product of slices is at most 2^16 (t = 2),
//     2^15 (t = 3) or 2^14 in magnitude, so inside a window of 256, 128 or 64 k
//     of all pairs of the weight every partial sum is an integer below 2^24 and
//     the FP32 MFMA accumulation is exact; window sums are added into an int32
//     U_t, exact for K panels of at most 8192.
//  4. S = sum over t from s+1 down to 2 of U_t * 2^(e_i + f_j - 8t), accumulated
//     in FP64 from the smallest weight to the largest.
//  5. C = alpha*S + beta*C + gamma*D with separate roundings (no fused
//     multiply-add), C not read when beta == 0, D not read when gamma == 0.
// A row or column holding a non-finite value gives NaN in its output row or
// column.
//
// The INT8 form runs the same steps with digits m_p = trunc(r * 2^(7p - e_i))
// (|m_p| <= 127, a signed byte) and weights 2^(e_i + f_j - 7t); its slice
// products run on INT8 matrix cores with exact INT32 sums and need no
// accumulation windows (split_gemm_i8).
//
// Workspace layout: see split_workspace_bytes (B planes are stored transposed
// so MFMA operands are contiguous in k; all padding is zero).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Slice formats, by bytes per slice element EB: 2 = BF16 digits m_p =
// rint(r 2^(8p-e)) (|m_1| <= 256, |m_p| <= 128), 1 = INT8 digits m_p =
// trunc(r 2^(7p-e)) (|m_p| <= 127); in both r -= m_p 2^(e - bits p), exactly.
template <int EB>
struct SliceFmt;
template <>
struct SliceFmt<2> {
  static constexpr int kBits = 8;
  __device__ static double digit(double x) { return rint(x); }
  __device__ static uint32_t pattern(double m) { return bf16_bits_exact(m); }
};
template <>
struct SliceFmt<1> {
  static constexpr int kBits = 7;
  __device__ static double digit(double x) { return trunc(x); }
  __device__ static uint32_t pattern(double m) { return (uint32_t)(uint8_t)(int8_t)(int)m; }
};

// The S slices of r (exponent e) as bit patterns of the format.
template <int S, int EB>
__device__ __forceinline__ void slices_of(double r, int32_t e, uint32_t (&bits)[S]) {
  constexpr int b = SliceFmt<EB>::kBits;
#pragma unroll
  for (int p = 1; p <= S; ++p) {
    double mp = 0.0;
    if (r != 0.0) {
      mp = SliceFmt<EB>::digit(ldexp(r, b * p - e));
      r = r - ldexp(mp, e - b * p);
    }
    bits[p - 1] = SliceFmt<EB>::pattern(mp);
  }
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// One wave per row of A: exponent, then the S slices of the row into the
// planes, 8 consecutive k per lane and step (one 8 * EB-byte store per plane).
template <int S, int EB>
__global__ __launch_bounds__(256) void split_rows(int64_t m, int64_t k, const double* __restrict__ A, int64_t lda,
                                                  int64_t mpad, int64_t kpad, uint8_t* __restrict__ planes,
                                                  int32_t* __restrict__ ex_out) {
  constexpr int E = 8, PER = 4 / EB, NW = E / PER;  // elements per lane and step, per 32-bit word; words
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
  // kpad is a multiple of 64, so a lane's E values never cross it
  for (int64_t k0 = (int64_t)lane * E; k0 < kpad; k0 += 64 * E) {
    uint32_t w[S][NW];
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int x = 0; x < NW; ++x) w[p][x] = 0;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int64_t kk = k0 + q;
      const double r = (live && !bad && kk < k) ? A[row * lda + kk] : 0.0;
      uint32_t b[S];
      slices_of<S, EB>(r, ex, b);
#pragma unroll
      for (int p = 0; p < S; ++p) w[p][q / PER] |= b[p] << (8 * EB * (q % PER));
    }
#pragma unroll
    for (int p = 0; p < S; ++p) {
      uint8_t* dst = planes + (((int64_t)p * mpad + row) * kpad + k0) * EB;
      if constexpr (EB == 2)
        *reinterpret_cast<u32x4*>(dst) = u32x4{w[p][0], w[p][1], w[p][2], w[p][3]};
      else
        *reinterpret_cast<u32x2*>(dst) = u32x2{w[p][0], w[p][1]};
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

// Slices of B into transposed planes [p][j][k]: a 64 (k) x 64 (j) tile per
// workgroup; each thread slices 16 consecutive k of one column and stores them
// as EB 16-byte vectors per plane.
template <int S, int EB>
__global__ __launch_bounds__(256) void split_cols(int64_t k, int64_t n, const double* __restrict__ B, int64_t ldb,
                                                  int64_t npad, int64_t kpad, const int32_t* __restrict__ ex,
                                                  uint8_t* __restrict__ planes) {
  constexpr int PER = 4 / EB, NW = 16 / PER;  // elements per 32-bit word, words per thread and plane
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
  uint32_t w[S][NW];
#pragma unroll
  for (int p = 0; p < S; ++p)
#pragma unroll
    for (int x = 0; x < NW; ++x) w[p][x] = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double r = (e == kBad) ? 0.0 : tile[jl][ks + q];
    uint32_t b[S];
    slices_of<S, EB>(r, e, b);
#pragma unroll
    for (int p = 0; p < S; ++p) w[p][q / PER] |= b[p] << (8 * EB * (q % PER));
  }
#pragma unroll
  for (int p = 0; p < S; ++p) {
    u32x4* dst = reinterpret_cast<u32x4*>(planes + (((int64_t)p * npad + j) * kpad + k0 + ks) * EB);
#pragma unroll
    for (int v = 0; v < EB; ++v) dst[v] = u32x4{w[p][4 * v], w[p][4 * v + 1], w[p][4 * v + 2], w[p][4 * v + 3]};
  }
}

// Slice products.  A workgroup of 4 waves (2 x 2) computes a 128 x 128 block
// of C; each wave a 64 x 64 block as 2 x 2 tiles of V_MFMA_F32_32X32X16_BF16.
// For each weight t (from s+1 down to 2) the kernel walks the K range in
// chunks of 64; every chunk of every pair (p, t-p) is staged in LDS (A plane
// rows and transposed B plane rows, k contiguous), double-buffered with the
// next chunk prefetched into registers without a break at window or weight
// boundaries.  FP32 accumulators are folded into
// integer sums U_t after windows of 256 (t <= 3), 128 (t <= 7) or 64 k, the
// longest windows whose partial sums provably stay below 2^24; with at most
// 8192 k per launch |U_t| < 8192 * 10 * 2^14 < 2^31, so int32 holds U_t
// exactly.  Between weights the FP64 slice sum S lives in a workspace tile;
// the last weight's pass finishes S and writes C.
// Operand layout of V_MFMA_F32_32X32X16_BF16: lane l supplies A[l%32][8*(l/32) .. +8]
// and B[8*(l/32) .. +8][l%32]; accumulator element v of lane l is
// D[8*(v/4) + 4*(l/32) + v%4][l%32].
constexpr int SBM = 128, SBN = 128, SKC = 64, SPAD = 8;  // tile, k chunk, LDS row padding (bf16)

// S = S + U_t 2^(e_i + f_j - bits t) for one 128 x 128 tile whose integer sums
// U_t sit in LDS (row-major), walked row by row with consecutive threads on
// consecutive columns; the last weight (t = 2) finishes S and writes
// C = alpha*S + beta*C + gamma*D with separate roundings.
__device__ __forceinline__ void slice_sum_update(const int32_t* Ul, int t, int s, int bits, int tid, int64_t m0,
                                                 int64_t n0, int64_t m, int64_t n, int64_t npad,
                                                 const int32_t* __restrict__ ea, const int32_t* __restrict__ fb,
                                                 double* __restrict__ Sws, double alpha, double beta,
                                                 double* __restrict__ C, int64_t ldc, double gamma,
                                                 const double* __restrict__ D, int64_t ldd) {
  // separate roundings: the products and sums below are not fused (the pragma
  // covers operations written in this function; HIP's __dmul_rn / __dadd_rn
  // inline plain operations from a header compiled with contraction on)
#pragma clang fp contract(off)
  const int c = tid & (SBN - 1);
  const int64_t col = n0 + c;
  const int32_t ff = fb[col];
#pragma unroll 4
  for (int r = tid / SBN; r < SBM; r += 256 / SBN) {
    const int64_t row = m0 + r;
    const int32_t ee = ea[row];
    const bool bad = ee == kBad || ff == kBad;
    double* ps = Sws + row * npad + col;
    const double term = bad ? 0.0 : ldexp((double)Ul[r * SBN + c], ee + ff - bits * t);
    const double S = (t == s + 1) ? term : (*ps + term);
    if (t > 2) {
      *ps = S;
    } else if (row < m && col < n) {
      double val;
      if (bad) {
        val = __builtin_nan("");
      } else {
        val = alpha * S;
        if (beta != 0.0) val = val + beta * C[row * ldc + col];
        if (gamma != 0.0) val = val + gamma * D[row * ldd + col];
      }
      C[row * ldc + col] = val;
    }
  }
}

constexpr int kBandRows = 4;  // tile rows per group in the XCD bands of the slice-product kernels

// Tile of workgroup b in a 1-D grid of tiles_m x tiles_n tiles: workgroups are
// dealt to the 8 XCDs round robin, so b & 7 names the XCD; each XCD takes a
// contiguous band of the tiles, walked in groups of gm_rows tile rows
// (column by column inside a group), so the tiles running together on one
// XCD share A and B plane rows in its L2.  The slice planes are re-read once
// per pair and tile; groups of 4 rows measured best (INT8 kernel at 8192^3:
// 1633 TOP/s against 1530 with the plain 2-D grid; groups of 8 gain nothing).
__device__ inline void xcd_band_tile(int b, int tiles_m, int tiles_n, int gm_rows, int* tm, int* tn) {
  const int ntiles = tiles_m * tiles_n;
  const int xcd = b & 7, local = b >> 3;
  const int q = ntiles >> 3, r = ntiles & 7;
  const int lin = xcd * q + (xcd < r ? xcd : r) + local;
  const int group = lin / (gm_rows * tiles_n);
  const int first_m = group * gm_rows;
  const int gm = (tiles_m - first_m) < gm_rows ? (tiles_m - first_m) : gm_rows;
  const int in_group = lin - group * gm_rows * tiles_n;
  *tm = first_m + in_group % gm;
  *tn = in_group / gm;
}

__device__ inline int fold_window_chunks(int t) { return t <= 3 ? 4 : (t <= 7 ? 2 : 1); }

__global__ __launch_bounds__(256, 2) void split_gemm(int64_t m, int64_t n, int64_t kpad, int s,
                                                     const uint16_t* __restrict__ Ap, const uint16_t* __restrict__ Bp,
                                                     int64_t mpad, int64_t npad, const int32_t* __restrict__ ea,
                                                     const int32_t* __restrict__ fb, double* __restrict__ Sws,
                                                     double alpha, double beta, double* __restrict__ C, int64_t ldc,
                                                     double gamma, const double* __restrict__ D, int64_t ldd) {
  // staging buffers for two chunks of A and B, or the tile's integer sums during a fold
  __shared__ __attribute__((aligned(16))) union {
    struct {
      uint16_t A[2][SBM][SKC + SPAD];
      uint16_t B[2][SBN][SKC + SPAD];
    } st;
    int32_t U[SBM * SBN];
  } sm;
  static_assert(sizeof(int32_t) * SBM * SBN <= 2 * (SBM + SBN) * (SKC + SPAD) * sizeof(uint16_t), "fold buffer");
  auto& As = sm.st.A;
  auto& Bs = sm.st.B;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  int tm, tn;
  xcd_band_tile((int)blockIdx.x, (int)(mpad / SBM), (int)(npad / SBN), kBandRows, &tm, &tn);
  const int64_t m0 = (int64_t)tm * SBM, n0 = (int64_t)tn * SBN;
  // global -> register staging: each thread moves 4 x 16 bytes of A and of B per
  // chunk: a 16-element quarter lq of rows lr and lr + 64 of the 64-k chunk
  const int lr = tid >> 2, lq = (tid & 3) * 16;
  // (named registers, not arrays: an array here was placed in scratch memory,
  // which serialised every global load behind its store)
  uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
  const int nchunks = (int)(kpad / SKC);

  auto gload = [&](int p, int q, int cc) {
    const uint16_t* pa = Ap + ((int64_t)(p - 1) * mpad + m0) * kpad + (int64_t)cc * SKC + lq;
    const uint16_t* pb = Bp + ((int64_t)(q - 1) * npad + n0) * kpad + (int64_t)cc * SKC + lq;
    const uint4* a0 = reinterpret_cast<const uint4*>(pa + (int64_t)lr * kpad);
    const uint4* a1 = reinterpret_cast<const uint4*>(pa + (int64_t)(lr + 64) * kpad);
    const uint4* b0 = reinterpret_cast<const uint4*>(pb + (int64_t)lr * kpad);
    const uint4* b1 = reinterpret_cast<const uint4*>(pb + (int64_t)(lr + 64) * kpad);
    ra0 = a0[0]; ra1 = a0[1]; ra2 = a1[0]; ra3 = a1[1];
    rb0 = b0[0]; rb1 = b0[1]; rb2 = b1[0]; rb3 = b1[1];
  };
  auto lstore = [&](int buf) {
    *reinterpret_cast<uint4*>(&As[buf][lr][lq]) = ra0;
    *reinterpret_cast<uint4*>(&As[buf][lr][lq + 8]) = ra1;
    *reinterpret_cast<uint4*>(&As[buf][lr + 64][lq]) = ra2;
    *reinterpret_cast<uint4*>(&As[buf][lr + 64][lq + 8]) = ra3;
    *reinterpret_cast<uint4*>(&Bs[buf][lr][lq]) = rb0;
    *reinterpret_cast<uint4*>(&Bs[buf][lr][lq + 8]) = rb1;
    *reinterpret_cast<uint4*>(&Bs[buf][lr + 64][lq]) = rb2;
    *reinterpret_cast<uint4*>(&Bs[buf][lr + 64][lq + 8]) = rb3;
  };

  const int fr = lane & 31, fk = 8 * (lane >> 5);
  // The steps of one weight t run window by window; inside a window over the
  // pairs (p, t-p), each over the window's chunks.  The next step is always
  // prefetched, also across window boundaries (a window only folds the FP32
  // accumulators into the integer sums) and across weights (the next weight's
  // first step is loaded into registers before the slice-sum update).
  struct Step { int c0, wlen, pi, ci; };
  auto first_step = [&](int t) { return Step{0, nchunks < fold_window_chunks(t) ? nchunks : fold_window_chunks(t), 0, 0}; };
  auto plo_of = [&](int t) { return t - s > 1 ? t - s : 1; };
  {
    const int t0 = s + 1;
    gload(plo_of(t0), t0 - plo_of(t0), 0);
    lstore(0);
    __syncthreads();
  }
  for (int t = s + 1; t >= 2; --t) {
    const int plo = plo_of(t), phi = t - 1 < s ? t - 1 : s;
    const int np = phi - plo + 1;
    const int wc = fold_window_chunks(t);
    int32_t U[2][2][16];  // exact: |U_t| < 8192 * 10 * 2^14 < 2^31 for K panels of at most 8192
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) U[i][j][v] = 0;
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
    const int nsteps = np * nchunks;
    Step cur = first_step(t);
    for (int st = 0; st < nsteps; ++st) {
      const int buf = st & 1;
      // the step after this one (within weight t)
      Step nx = cur;
      bool window_end = false;
      if (++nx.ci == nx.wlen) {
        nx.ci = 0;
        if (++nx.pi == np) {
          nx.pi = 0;
          window_end = true;
          nx.c0 += nx.wlen;
          nx.wlen = (nchunks - nx.c0) < wc ? (nchunks - nx.c0) : wc;
        }
      }
      const bool more = st + 1 < nsteps;
      if (more) gload(plo + nx.pi, t - (plo + nx.pi), nx.c0 + nx.ci);
#pragma unroll
      for (int kk = 0; kk < SKC; kk += 16) {
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * 64 + i * 32 + fr][kk + fk]);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn * 64 + j * 32 + fr][kk + fk]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      if (window_end || !more) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              U[i][j][v] += (int32_t)acc[i][j][v];
              acc[i][j][v] = 0.f;
            }
      }
      if (more) lstore(buf ^ 1);
      __syncthreads();
      cur = nx;
    }
    // prefetch the next weight's first step while the slice sums are added
    if (t > 2) gload(plo_of(t - 1), (t - 1) - plo_of(t - 1), 0);
    // S = S + U_t 2^(e_i + f_j - 8t), from the smallest weight up.  The sums go
    // through LDS (the staging buffers are idle now) so that the update below
    // walks the tile row by row with consecutive threads on consecutive columns.
    int32_t* Ul = sm.U;  // [SBM][SBN]
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          Ul[(wm * 64 + i * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4)) * SBN + wn * 64 + j * 32 + (lane & 31)] =
              U[i][j][v];
    __syncthreads();
    slice_sum_update(Ul, t, s, 8, tid, m0, n0, m, n, npad, ea, fb, Sws, alpha, beta, C, ldc, gamma, D, ldd);
    __syncthreads();  // LDS is staging space again
    if (t > 2) {
      lstore(0);
      __syncthreads();
    }
  }
}

// INT8 slice products on V_MFMA_I32_32X32X32_I8 (lane l supplies A[l%32][16*(l/32) .. +16]
// and B[16*(l/32) .. +16][l%32]; accumulator layout as for the BF16 form).  The
// same tiling and staging as split_gemm, byte for byte: a 128-k chunk of INT8
// planes is the 128 bytes of a 64-k BF16 chunk, and tiles are dealt to the
// XCDs in the same bands (xcd_band_tile).  A product of two INT8 slices is
// below 2^14 and the INT32 accumulation is exact, so no windows: one weight's
// sum over every pair and the whole K panel (at most 8192 k:
// |U_t| < 8 * 8192 * 2^14 = 2^30) stays in the accumulators.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
constexpr int SKC8 = 128;  // k per chunk (INT8)

__global__ __launch_bounds__(256, 2) void split_gemm_i8(int64_t m, int64_t n, int64_t kpad, int s,
                                                        const uint8_t* __restrict__ Ap, const uint8_t* __restrict__ Bp,
                                                        int64_t mpad, int64_t npad, const int32_t* __restrict__ ea,
                                                        const int32_t* __restrict__ fb, double* __restrict__ Sws,
                                                        double alpha, double beta, double* __restrict__ C, int64_t ldc,
                                                        double gamma, const double* __restrict__ D, int64_t ldd) {
  constexpr int LD = SKC8 + 2 * SPAD;  // bytes per LDS row: the BF16 kernel's 64 + 8 elements
  __shared__ __attribute__((aligned(16))) union {
    struct {
      uint8_t A[2][SBM][LD];
      uint8_t B[2][SBN][LD];
    } st;
    int32_t U[SBM * SBN];
  } sm;
  static_assert(sizeof(int32_t) * SBM * SBN <= 2 * (SBM + SBN) * LD, "fold buffer");
  auto& As = sm.st.A;
  auto& Bs = sm.st.B;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  int tm, tn;
  xcd_band_tile((int)blockIdx.x, (int)(mpad / SBM), (int)(npad / SBN), kBandRows, &tm, &tn);
  const int64_t m0 = (int64_t)tm * SBM, n0 = (int64_t)tn * SBN;
  // each thread moves 64 bytes of A and of B per chunk: a 32-byte quarter lq of rows lr and lr + 64
  const int lr = tid >> 2, lq = (tid & 3) * 32;
  uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
  const int nchunks = (int)(kpad / SKC8);
  auto gload = [&](int p, int q, int cc) {
    const uint8_t* pa = Ap + ((int64_t)(p - 1) * mpad + m0) * kpad + (int64_t)cc * SKC8 + lq;
    const uint8_t* pb = Bp + ((int64_t)(q - 1) * npad + n0) * kpad + (int64_t)cc * SKC8 + lq;
    const uint4* a0 = reinterpret_cast<const uint4*>(pa + (int64_t)lr * kpad);
    const uint4* a1 = reinterpret_cast<const uint4*>(pa + (int64_t)(lr + 64) * kpad);
    const uint4* b0 = reinterpret_cast<const uint4*>(pb + (int64_t)lr * kpad);
    const uint4* b1 = reinterpret_cast<const uint4*>(pb + (int64_t)(lr + 64) * kpad);
    ra0 = a0[0]; ra1 = a0[1]; ra2 = a1[0]; ra3 = a1[1];
    rb0 = b0[0]; rb1 = b0[1]; rb2 = b1[0]; rb3 = b1[1];
  };
  auto lstore = [&](int buf) {
    *reinterpret_cast<uint4*>(&As[buf][lr][lq]) = ra0;
    *reinterpret_cast<uint4*>(&As[buf][lr][lq + 16]) = ra1;
    *reinterpret_cast<uint4*>(&As[buf][lr + 64][lq]) = ra2;
    *reinterpret_cast<uint4*>(&As[buf][lr + 64][lq + 16]) = ra3;
    *reinterpret_cast<uint4*>(&Bs[buf][lr][lq]) = rb0;
    *reinterpret_cast<uint4*>(&Bs[buf][lr][lq + 16]) = rb1;
    *reinterpret_cast<uint4*>(&Bs[buf][lr + 64][lq]) = rb2;
    *reinterpret_cast<uint4*>(&Bs[buf][lr + 64][lq + 16]) = rb3;
  };
  const int fr = lane & 31, fk = 16 * (lane >> 5);
  auto plo_of = [&](int t) { return t - s > 1 ? t - s : 1; };
  {
    const int t0 = s + 1;
    gload(plo_of(t0), t0 - plo_of(t0), 0);
    lstore(0);
    __syncthreads();
  }
  for (int t = s + 1; t >= 2; --t) {
    const int plo = plo_of(t), phi = t - 1 < s ? t - 1 : s;
    const int np = phi - plo + 1;
    i32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = 0;
    // steps: the pairs (p, t-p) in turn, each over every chunk; the next step
    // is prefetched into registers while this one multiplies
    const int nsteps = np * nchunks;
    int pi = 0, ci = 0;
    for (int st = 0; st < nsteps; ++st) {
      const int buf = st & 1;
      int npi = pi, nci = ci + 1;
      if (nci == nchunks) {
        nci = 0;
        ++npi;
      }
      const bool more = st + 1 < nsteps;
      if (more) gload(plo + npi, t - (plo + npi), nci);
#pragma unroll
      for (int kk = 0; kk < SKC8; kk += 32) {
        i32x4 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const i32x4*>(&As[buf][wm * 64 + i * 32 + fr][kk + fk]);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const i32x4*>(&Bs[buf][wn * 64 + j * 32 + fr][kk + fk]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      if (more) lstore(buf ^ 1);
      __syncthreads();
      pi = npi;
      ci = nci;
    }
    // prefetch the next weight's first step while the slice sums are added
    if (t > 2) gload(plo_of(t - 1), (t - 1) - plo_of(t - 1), 0);
    int32_t* Ul = sm.U;  // [SBM][SBN]
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          Ul[(wm * 64 + i * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4)) * SBN + wn * 64 + j * 32 + (lane & 31)] =
              acc[i][j][v];
    __syncthreads();
    slice_sum_update(Ul, t, s, 7, tid, m0, n0, m, n, npad, ea, fb, Sws, alpha, beta, C, ldc, gamma, D, ldd);
    __syncthreads();  // LDS is staging space again
    if (t > 2) {
      lstore(0);
      __syncthreads();
    }
  }
}

inline int64_t pad64(int64_t x) { return (x + 63) / 64 * 64; }
inline int64_t pad128(int64_t x) { return (x + 127) / 128 * 128; }

}  // namespace

// Workspace: A planes [s][mp][kp], B planes [s][np][kp] (BF16 or INT8),
// row and column exponents (int32), column maxima (uint64), slice-sum tile
// [mp][np] (FP64), with mp, np = m, n rounded up to 128 and kp = k rounded up
// to a whole number of 128-byte chunks (64 BF16 or 128 INT8 elements).
static int64_t pad_k(int64_t k, SliceFormat f) { return f == kSliceInt8 ? pad128(k) : pad64(k); }

size_t split_workspace_bytes(int64_t m, int64_t n, int64_t k, int s, SliceFormat f) {
  const int64_t mp = pad128(m), np = pad128(n), kp = pad_k(k < kSplitMaxK ? k : kSplitMaxK, f);
  return (size_t)((int64_t)f * s * (mp + np) * kp + 4 * (mp + np) + 8 * np + 8 * mp * np);
}

static hipError_t split_panel(SliceFormat f, int64_t m, int64_t n, int64_t k, int s, double alpha, const double* A,
                              int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                              double gamma, const double* D, int64_t ldd, void* workspace, size_t ws_bytes,
                              hipStream_t stream, KernelTimer* timer);

hipError_t launch_split_gemm(SliceFormat f, int64_t m, int64_t n, int64_t k, int s, double alpha, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                             double gamma, const double* D, int64_t ldd, void* workspace, size_t ws_bytes,
                             hipStream_t stream, KernelTimer* timer) {
  // K panels of at most kSplitMaxK: C = alpha*S_0 + beta*C + gamma*D, then C = alpha*S_p + C
  if (m <= 0 || n <= 0) return hipSuccess;
  if (f != kSliceBF16 && f != kSliceInt8) return hipErrorInvalidValue;
  if (k <= kSplitMaxK)
    return split_panel(f, m, n, k, s, alpha, A, lda, B, ldb, beta, C, ldc, gamma, D, ldd, workspace, ws_bytes, stream,
                       timer);
  for (int64_t k0 = 0; k0 < k; k0 += kSplitMaxK) {
    const int64_t kk = (k - k0) < kSplitMaxK ? (k - k0) : kSplitMaxK;
    const bool first = k0 == 0;
    hipError_t e = split_panel(f, m, n, kk, s, alpha, A + k0, lda, B + k0 * ldb, ldb, first ? beta : 1.0, C, ldc,
                               first ? gamma : 0.0, D, ldd, workspace, ws_bytes, stream, timer);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t split_panel(SliceFormat f, int64_t m, int64_t n, int64_t k, int s, double alpha, const double* A,
                              int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                              double gamma, const double* D, int64_t ldd, void* workspace, size_t ws_bytes,
                              hipStream_t stream, KernelTimer* timer) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (s < 1 || s > 8) return hipErrorInvalidValue;
  if (k <= 0) return launch_dgemm_f64(m, n, 0, alpha, nullptr, 1, nullptr, 1, beta, C, ldc, gamma, D, ldd, stream);
  const int64_t mp = pad128(m), np = pad128(n), kp = pad_k(k, f);
  if (split_workspace_bytes(m, n, k, s, f) > ws_bytes) return hipErrorInvalidValue;
  const int eb = (int)f;
  uint8_t* Ap = static_cast<uint8_t*>(workspace);
  uint8_t* Bp = Ap + (size_t)eb * s * mp * kp;
  int32_t* ea = reinterpret_cast<int32_t*>(Bp + (size_t)eb * s * np * kp);
  int32_t* fb = ea + mp;
  unsigned long long* bmax = reinterpret_cast<unsigned long long*>(fb + np);  // 8-byte aligned: mp, np even
  double* Sws = reinterpret_cast<double*>(bmax + np);
  if (gamma == 0.0) D = nullptr;
  const dim3 rows_grid((unsigned)(mp / 4)), cols_grid((unsigned)(kp / 64), (unsigned)(np / 64));
  auto slice_a = [&](auto S) {
    constexpr int sv = decltype(S)::value;
    if (f == kSliceInt8)
      hipLaunchKernelGGL((split_rows<sv, 1>), rows_grid, dim3(256), 0, stream, m, k, A, lda, mp, kp, Ap, ea);
    else
      hipLaunchKernelGGL((split_rows<sv, 2>), rows_grid, dim3(256), 0, stream, m, k, A, lda, mp, kp, Ap, ea);
  };
  auto slice_b = [&](auto S) {
    constexpr int sv = decltype(S)::value;
    if (f == kSliceInt8)
      hipLaunchKernelGGL((split_cols<sv, 1>), cols_grid, dim3(256), 0, stream, k, n, B, ldb, np, kp, fb, Bp);
    else
      hipLaunchKernelGGL((split_cols<sv, 2>), cols_grid, dim3(256), 0, stream, k, n, B, ldb, np, kp, fb, Bp);
  };
  auto with_s = [&](auto fn) {
    switch (s) {
      case 1: fn(std::integral_constant<int, 1>{}); break;
      case 2: fn(std::integral_constant<int, 2>{}); break;
      case 3: fn(std::integral_constant<int, 3>{}); break;
      case 4: fn(std::integral_constant<int, 4>{}); break;
      case 5: fn(std::integral_constant<int, 5>{}); break;
      case 6: fn(std::integral_constant<int, 6>{}); break;
      case 7: fn(std::integral_constant<int, 7>{}); break;
      default: fn(std::integral_constant<int, 8>{}); break;
    }
  };
  with_s(slice_a);
  hipLaunchKernelGGL(zero_u64, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, stream,
                     reinterpret_cast<uint64_t*>(bmax), np);
  hipLaunchKernelGGL(col_absmax, dim3((unsigned)((n + 255) / 256), (unsigned)((k + 255) / 256)), dim3(256), 0, stream,
                     k, n, B, ldb, bmax);
  hipLaunchKernelGGL(col_exponents, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, stream, np, bmax, fb);
  with_s(slice_b);
  // one-dimensional grids: the kernels map workgroups to tiles in XCD bands
  const dim3 grid((unsigned)((np / SBN) * (mp / SBM)));
  const bool timed = timer && timer->used < timer->count;
  if (timed) {
    const hipError_t e = hipEventRecord(timer->events[2 * timer->used], stream);
    if (e != hipSuccess) return e;
  }
  if (f == kSliceInt8)
    hipLaunchKernelGGL(split_gemm_i8, grid, dim3(256), 0, stream, m, n, kp, s, Ap, Bp, mp, np, ea, fb, Sws, alpha,
                       beta, C, ldc, gamma, D, ldd);
  else
    hipLaunchKernelGGL(split_gemm, grid, dim3(256), 0, stream, m, n, kp, s, reinterpret_cast<const uint16_t*>(Ap),
                       reinterpret_cast<const uint16_t*>(Bp), mp, np, ea, fb, Sws, alpha, beta, C, ldc, gamma, D, ldd);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (timed) {
    const hipError_t er = hipEventRecord(timer->events[2 * timer->used + 1], stream);
    if (er != hipSuccess) return er;
    ++timer->used;
  }
  return hipSuccess;
}

}  // namespace ooc
