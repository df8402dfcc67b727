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
//     sum_k mA_p[i,k] mB_q[k,j].  |m_1| <= 2^8 and |m_p| <= 2^7 (p >= 2), so a
//     product of slices p and q is at most 2^16 (p = q = 1), 2^15 (one of them
//     1) or 2^14, and the products of one k over all pairs of weight t sum to
//     at most B(t) = 2^16 (t <= 3) or 2^16 + (t-3) 2^14 (t >= 4).  Inside a
//     window of W(t) = 256 (t <= 3), 128 (t <= 7) or 64 (t >= 8) k every
//     partial sum is an integer of magnitude at most W(t) B(t) <= 2^24 (equal
//     at t = 2, 3 and 7: no margin), so the FP32 MFMA accumulation is exact
//     (kWindowsExact checks every t up to 9); window sums are added into an
//     int32 U_t, exact for K panels of at most 8192.
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

#include <cmath>
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

// One workgroup per row of A, read from memory once: each thread holds up to
// kRowChunks chunks of 8 consecutive k in registers (chunk c of thread t at k =
// 8 (256 c + t)), the row's exponent comes from a workgroup reduction of the
// maximum, and the S slices are written from the registers, one 8 * EB-byte
// store per chunk and plane.  Every load reads an address inside the row
// (clamped) and the value is then selected, so the loads are in flight
// together.
constexpr int kRowThreads = 256, kRowE = 8;
constexpr int kRowChunks = (int)(kSplitMaxK / (kRowThreads * kRowE));
template <int S, int EB>
__global__ __launch_bounds__(kRowThreads) void split_rows(int64_t m, int64_t k, const double* __restrict__ A,
                                                          int64_t lda, int64_t mpad, int64_t kpad,
                                                          uint8_t* __restrict__ planes, int32_t* __restrict__ ex_out) {
  constexpr int E = kRowE, PER = 4 / EB, NW = E / PER;  // elements per chunk, per 32-bit word; words
  __shared__ double wmx[kRowThreads / 64];
  __shared__ int wbad[kRowThreads / 64];
  const int t = threadIdx.x, lane = t & 63;
  const int64_t row = blockIdx.x;
  const bool live = row < m;
  const double* src = A + (live ? row : m - 1) * lda;
  double v[kRowChunks][E];
  double mx = 0.0;
  int bad = 0;
#pragma unroll
  for (int c = 0; c < kRowChunks; ++c) {
    const int64_t k0 = ((int64_t)c * kRowThreads + t) * E;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int64_t kk = k0 + q;
      const double x = src[kk < k ? kk : k - 1];
      v[c][q] = (live && kk < k) ? x : 0.0;
      if (!isfinite(v[c][q])) bad = 1;
      mx = fmax(mx, fabs(v[c][q]));
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off));
    bad |= __shfl_xor(bad, off);
  }
  if (lane == 0) {
    wmx[t >> 6] = mx;
    wbad[t >> 6] = bad;
  }
  __syncthreads();
#pragma unroll
  for (int x = 0; x < kRowThreads / 64; ++x) {
    mx = fmax(mx, wmx[x]);
    bad |= wbad[x];
  }
  const int32_t ex = bad ? kBad : exponent_of(mx);
  if (t == 0) ex_out[row] = ex;
  // kpad is a multiple of 64, so a chunk never crosses it
#pragma unroll
  for (int c = 0; c < kRowChunks; ++c) {
    const int64_t k0 = ((int64_t)c * kRowThreads + t) * E;
    if (k0 >= kpad) break;
    uint32_t w[S][NW];
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int x = 0; x < NW; ++x) w[p][x] = 0;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      uint32_t bits[S];
      slices_of<S, EB>(bad ? 0.0 : v[c][q], ex, bits);
#pragma unroll
      for (int p = 0; p < S; ++p) w[p][q / PER] |= bits[p] << (8 * EB * (q % PER));
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


// The exactness windows of the BF16 slice products (k per window), and the
// bound on the sum over all pairs of weight t of one k's slice products.
__host__ __device__ constexpr int window_k(int t) { return t <= 3 ? 256 : (t <= 7 ? 128 : 64); }
__host__ __device__ constexpr int64_t pair_sum_bound(int t) {
  int64_t b = 0;
  for (int p = 1; p < t; ++p) {
    const int q = t - p;
    b += (int64_t)(p == 1 ? 256 : 128) * (q == 1 ? 256 : 128);
  }
  return b;
}
__host__ __device__ constexpr bool windows_exact() {
  for (int t = 2; t <= 9; ++t)
    if (window_k(t) * pair_sum_bound(t) > (int64_t(1) << 24)) return false;
  return true;
}
constexpr bool kWindowsExact = windows_exact();
static_assert(kWindowsExact, "an exactness window lets an FP32 partial sum exceed 2^24");

// S = S + U_t 2^(e_i + f_j - bits t) for one TBM x TBN tile whose integer
// sums U_t sit in LDS (row-major), walked row by row with consecutive threads
// on consecutive columns (NT threads); ea and fb hold the tile's row and
// column exponents (tile-relative).  The last weight (t = 2) finishes S and
// writes C = alpha*S + beta*C + gamma*D with separate roundings.
template <int TBM, int TBN, int NT>
__device__ __forceinline__ void slice_sum_update(const int32_t* Ul, const int32_t* ea, const int32_t* fb, int t,
                                                 int s, int bits, int tid, int64_t m0, int64_t n0, int64_t m,
                                                 int64_t n, int64_t npad, double* __restrict__ Sws, double alpha,
                                                 double beta, double* __restrict__ C, int64_t ldc, double gamma,
                                                 const double* __restrict__ D, int64_t ldd) {
  // separate roundings: the products and sums below are not fused (the pragma
  // covers operations written in this function; HIP's __dmul_rn / __dadd_rn
  // inline plain operations from a header compiled with contraction on)
#pragma clang fp contract(off)
  static_assert(NT % TBN == 0, "whole rows per pass");
  const int c = tid % TBN;
  const int64_t col = n0 + c;
  const int32_t ff = fb[c];
#pragma unroll 4
  for (int r = tid / TBN; r < TBM; r += NT / TBN) {
    const int64_t row = m0 + r;
    const int32_t ee = ea[r];
    const bool bad = ee == kBad || ff == kBad;
    double* ps = Sws + row * npad + col;
    const double term = bad ? 0.0 : ldexp((double)Ul[r * TBN + c], ee + ff - bits * t);
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


// Slice products, BF16 or INT8 (EB bytes per digit), on 256-row tiles of C
// of TBN = 128 or 256 columns.  A workgroup of 8 waves (one workgroup per
// CU, two waves per SIMD) computes the tile, each wave a block of 2 x 2
// (TBN = 128: 4 x 2 waves of 64 x 64) or 4 x 2 (TBN = 256: 2 x 4 waves of
// 128 x 64) tiles of V_MFMA_F32_32X32X16_BF16 or V_MFMA_I32_32X32X32_I8.  For
// each weight t (from s+1 down to 2) the steps walk the exactness windows,
// inside a window the pairs (p, t-p), inside a pair the window's chunks of
// 128 bytes per row (64 BF16 or 128 INT8 k).  The A and B plane rows of a
// step (256 + TBN rows of 128 bytes) are loaded straight into one of NST LDS
// stages, NST - 1 steps ahead of the products (three stages of 48 KiB for
// TBN = 128, two of 64 KiB for TBN = 256); the direct loads are written in
// asm so the compiler does not wait for all of them before each LDS read,
// and the barrier between steps is a bare s_barrier after an explicit wait
// for the next step's loads only (__syncthreads would also wait for the
// loads of the step after).  At each window's end the FP32 accumulators are
// folded into the int32 sums U_t; the INT8 products accumulate exactly in
// INT32 over the whole K panel, so they have no windows and their
// accumulators are the sums (which is what leaves the registers for TBN =
// 256).  At each weight's end the sums go through LDS (the stages are idle
// by then; for TBN = 256 one half of the tile at a time) into S = S + U_t
// 2^(e_i + f_j - bits t), accumulated in the workspace tile, and the last
// weight writes C.  A row's 16-byte slots are permuted (slot = chunk ^ ((row
// + row / 8) & 7)) so that 16-byte LDS reads of 8 or of 16 consecutive rows
// fall in distinct banks.
// Operand layouts: lane l supplies A[l%32][8*(l/32) .. +8] and
// B[8*(l/32) .. +8][l%32] (BF16, k16 per instruction) or A[l%32][16*(l/32) .. +16]
// and B[16*(l/32) .. +16][l%32] (INT8, k32): 16 bytes per lane in both, slot
// 2 kk + l/32 of the row for the kk-th instruction of a chunk.  Accumulator
// element v of lane l is D[8*(v/4) + 4*(l/32) + v%4][l%32].
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

template <int EB>
struct SliceMfma;
template <>
struct SliceMfma<2> {
  typedef bf16x8 frag;
  typedef f32x16 acc;
  __device__ static acc mfma(frag a, frag b, acc c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
  static constexpr int kChunk = 64;  // k per 128-byte chunk
  static constexpr bool kWindows = true;
  __device__ static int window_chunks(int t, int) { return window_k(t) / kChunk; }
};
template <>
struct SliceMfma<1> {
  typedef i32x4 frag;
  typedef i32x16 acc;
  __device__ static acc mfma(frag a, frag b, acc c) { return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0); }
  static constexpr int kChunk = 128;
  // |U_t| < 8 * 8192 * 2^14 = 2^30 over a K panel of at most 8192: no windows
  static constexpr bool kWindows = false;
  __device__ static int window_chunks(int, int nchunks) { return nchunks; }
};

constexpr int GBM = 256;  // tile rows
constexpr int GNT = 512;  // threads per workgroup (8 waves)
constexpr int GROW = 128;  // bytes per tile row and step
constexpr int GKK = 4;     // instructions per chunk along k (32 bytes of each row apiece)

// Tile geometry for TBN columns.
template <int TBN>
struct SliceTile {
  static constexpr int WM = TBN == 256 ? 2 : 4, WN = 8 / WM;                    // waves along M and N
  static constexpr int FI = GBM / WM / 32, FJ = TBN / WN / 32;                  // 32 x 32 tiles per wave
  static constexpr int A = GBM * GROW, STAGE = A + TBN * GROW;                  // bytes per LDS stage
  static constexpr int NST = TBN == 256 ? 2 : 3;                                // LDS stages
  static constexpr int ALD = GBM / 8 / 8, BLD = TBN / 8 / 8, LD = ALD + BLD;    // 1-KB loads per wave and step
  static constexpr int HALVES = GBM * TBN * 4 > NST * STAGE ? 2 : 1;           // passes of the sums through LDS
  static_assert(ALD * 64 == GBM && BLD * 64 == TBN, "load split");
  static_assert(GBM / HALVES * TBN * 4 <= NST * STAGE && WM % HALVES == 0, "sum buffer");
  static_assert(NST * STAGE + 4 * (GBM + TBN) <= 160 * 1024, "LDS");
};

__device__ __forceinline__ int gswz(int r) { return (r + (r >> 3)) & 7; }

// One 16-byte-per-lane load into LDS at lds_addr + 16 * lane (M0 = the
// wave-uniform LDS byte address; one wait state after M0 is written).
__device__ __forceinline__ void load_lds16(const void* g, uint32_t lds_addr) {
  asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "{m0}"(lds_addr) : "memory");
}

// Wait until at most N vector-memory operations of this wave are in flight and
// its LDS operations are done, then the workgroup barrier.
template <int N>
__device__ __forceinline__ void wait_vm_barrier() {
  constexpr int imm = (N & 15) | (7 << 4) | ((N >> 4) << 14);  // vmcnt(N) expcnt(7) lgkmcnt(0)
  __builtin_amdgcn_s_waitcnt(imm);
  asm volatile("s_barrier" ::: "memory");
}

template <int EB, int TBN>
__device__ __forceinline__ void split_gemm_body(int64_t m, int64_t n, int64_t kpad, int s,
                                                const uint8_t* __restrict__ Ap, const uint8_t* __restrict__ Bp,
                                                int64_t mpad, int64_t npad, const int32_t* __restrict__ ea,
                                                const int32_t* __restrict__ fb, double* __restrict__ Sws,
                                                double alpha, double beta, double* __restrict__ C, int64_t ldc,
                                                double gamma, const double* __restrict__ D, int64_t ldd,
                                                unsigned char* lds, int32_t* eas, int32_t* fbs) {
  typedef SliceMfma<EB> M;
  typedef SliceTile<TBN> T;
  typedef typename M::frag frag;
  constexpr int FI = T::FI, FJ = T::FJ, NST = T::NST;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / T::WN, wn = w % T::WN;
  int tm, tn;
  xcd_band_tile((int)blockIdx.x, (int)(mpad / GBM), (int)(npad / TBN), kBandRows, &tm, &tn);
  const int64_t m0 = (int64_t)tm * GBM, n0 = (int64_t)tn * TBN;
  for (int r = tid; r < GBM; r += GNT) eas[r] = ea[m0 + r];
  for (int c = tid; c < TBN; c += GNT) fbs[c] = fb[n0 + c];
  const int nchunks = (int)(kpad / M::kChunk);
  const int64_t rowb = kpad * EB;  // bytes per plane row

  // direct loads: wave w fills tile rows [8 ALD w, +8 ALD) of A and
  // [8 BLD w, +8 BLD) of B, 8 rows per 1-KB load; lane l writes slot (l & 7)
  // of row (l >> 3) of the load's 8, which holds the row's 16-byte slot ^ gswz(row)
  const int lrow = lane >> 3, lslot = lane & 7;
  const uint8_t* a_src = Ap + (m0 + 8 * T::ALD * w + lrow) * rowb;
  const uint8_t* b_src = Bp + (n0 + 8 * T::BLD * w + lrow) * rowb;
  const uint32_t lds0 = (uint32_t)(size_t)(__attribute__((address_space(3))) unsigned char*)lds;
  const uint32_t la0 = __builtin_amdgcn_readfirstlane(lds0 + (8 * T::ALD * w) * GROW);
  const uint32_t lb0 = __builtin_amdgcn_readfirstlane(lds0 + T::A + (8 * T::BLD * w) * GROW);
  // with three stages the loads of a step are spread over its GKK
  // instruction groups (part kk issues the A loads j with j % GKK == kk and
  // the B loads j with j * GKK / BLD == kk), so that a wave's requests do not
  // reach the L1 in one burst ahead of its products (8192^3: BF16 862 -> 913
  // TFLOP/s, INT8 1624 -> 1785 TOP/s); with two stages, one step ahead, they
  // go out together at the step's start (spread: 1880 -> 1756 TOP/s)
  constexpr bool kSpread = NST > 2;
  // With three stages each step's last instruction group also runs after the
  // step's barrier, under the next step's first LDS reads (8192^3 BF16: 937 ->
  // 965 TFLOP/s; INT8 unchanged); the 256 x 256 INT8 tile has no registers
  // for fragments held across the barrier (spilled, 1905 -> 1235 TOP/s).
  constexpr bool kCarry = NST > 2;
  auto issue_part = [&](const uint8_t* pa, const uint8_t* pb, uint32_t so, int kk) {
#pragma unroll
    for (int j = 0; j < T::ALD; ++j)
      if (j % GKK == kk)
        load_lds16(pa + 8 * j * rowb + 16 * (lslot ^ gswz(8 * (T::ALD * w + j) + lrow)), la0 + so + 1024 * j);
#pragma unroll
    for (int j = 0; j < T::BLD; ++j)
      if (j * GKK / T::BLD == kk)
        load_lds16(pb + 8 * j * rowb + 16 * (lslot ^ gswz(8 * (T::BLD * w + j) + lrow)), lb0 + so + 1024 * j);
  };
  auto src_a = [&](int p, int cc) { return a_src + (int64_t)(p - 1) * mpad * rowb + (int64_t)cc * GROW; };
  auto src_b = [&](int q, int cc) { return b_src + (int64_t)(q - 1) * npad * rowb + (int64_t)cc * GROW; };
  auto issue = [&](int p, int q, int cc, int stage) {
#pragma unroll
    for (int kk = 0; kk < GKK; ++kk) issue_part(src_a(p, cc), src_b(q, cc), (uint32_t)stage * T::STAGE, kk);
  };
  const int fr = lane & 31, fh = lane >> 5;
  const int a_row0 = wm * (GBM / T::WM) + fr, b_row0 = wn * (TBN / T::WN) + fr;
  auto frags = [&](const unsigned char* As, const unsigned char* Bs, int kk, frag (&a)[FI], frag (&b)[FJ]) {
    const int ch = 2 * kk + fh;
#pragma unroll
    for (int i = 0; i < FI; ++i) {
      const int r = a_row0 + 32 * i;
      a[i] = *reinterpret_cast<const frag*>(As + r * GROW + ((ch ^ gswz(r)) << 4));
    }
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
      const int r = b_row0 + 32 * j;
      b[j] = *reinterpret_cast<const frag*>(Bs + r * GROW + ((ch ^ gswz(r)) << 4));
    }
  };

  for (int t = s + 1; t >= 2; --t) {
    const int plo = t - s > 1 ? t - s : 1, phi = t - 1 < s ? t - 1 : s;
    const int np = phi - plo + 1, wc = M::window_chunks(t, nchunks);
    const int nsteps = np * nchunks;
    // prefetch cursor: window start, window length, pair, chunk in window
    int f_c0 = 0, f_wl = nchunks < wc ? nchunks : wc, f_pi = 0, f_ci = 0;
    auto fadv = [&]() {
      if (++f_ci < f_wl) return;
      f_ci = 0;
      if (++f_pi < np) return;
      f_pi = 0;
      f_c0 += f_wl;
      f_wl = (nchunks - f_c0) < wc ? (nchunks - f_c0) : wc;
    };
    int issued = 0;
#pragma unroll
    for (int x = 0; x < NST - 1; ++x) {
      if (issued < nsteps) {
        issue(plo + f_pi, t - plo - f_pi, f_c0 + f_ci, x);
        fadv();
        ++issued;
      }
    }
    if (issued >= 2)
      wait_vm_barrier<T::LD>();  // step 0 has landed, step 1 may be in flight
    else
      wait_vm_barrier<0>();
    // exact: |U_t| < 8192 * 10 * 2^14 < 2^31 for K panels of at most 8192
    int32_t U[M::kWindows ? FI : 1][M::kWindows ? FJ : 1][16];
    if constexpr (M::kWindows) {
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) U[i][j][v] = 0;
    }
    typename M::acc acc[FI][FJ];
    static_assert(GKK % 2 == 0, "the last instruction group's fragments are in a1, b1");
    auto mfma_group = [&](const frag (&a)[FI], const frag (&b)[FJ]) {
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) acc[i][j] = M::mfma(a[i], b[j], acc[i][j]);
    };
    int stage = 0, st = 0;
    for (int c0 = 0; c0 < nchunks; c0 += wc) {
      const int wl = (nchunks - c0) < wc ? (nchunks - c0) : wc;
      const int wsteps = np * wl;
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[i][j][v] = 0;
      frag a0[FI], b0[FJ], a1[FI], b1[FJ];
      for (int x = 0; x < wsteps; ++x, ++st) {
        // NST - 1 steps ahead, into the stage every wave left at the last
        // barrier (part by part between the products when spread)
        const bool more = issued < nsteps;
        const uint8_t* ipa = src_a(plo + f_pi, f_c0 + f_ci);
        const uint8_t* ipb = src_b(t - plo - f_pi, f_c0 + f_ci);
        const uint32_t iso = (uint32_t)(stage == 0 ? NST - 1 : stage - 1) * T::STAGE;
        if (more) {
          if constexpr (!kSpread) issue(plo + f_pi, t - plo - f_pi, f_c0 + f_ci, stage == 0 ? NST - 1 : stage - 1);
          fadv();
          ++issued;
        }
        const unsigned char* As = lds + stage * T::STAGE;
        const unsigned char* Bs = As + T::A;
        frags(As, Bs, 0, a0, b0);
        // with kCarry the previous step's last instruction group multiplies
        // (its fragments are in registers) while this step's first fragments
        // are read
        if constexpr (kCarry) {
          if (x > 0) mfma_group(a1, b1);
        }
#pragma unroll
        for (int kk = 0; kk < (kCarry ? GKK - 1 : GKK); ++kk) {
          if (kSpread && more) {
            issue_part(ipa, ipb, iso, kk);
            if (kCarry && kk + 2 == GKK) issue_part(ipa, ipb, iso, kk + 1);
          }
          // fragments of the next instruction's k range are read while this
          // one multiplies; with kCarry the last group's stay in a1, b1 past
          // the barrier
          if (kk % 2 == 0) {
            if (kk + 1 < GKK) frags(As, Bs, kk + 1, a1, b1);
            mfma_group(a0, b0);
          } else {
            if (kk + 1 < GKK) frags(As, Bs, kk + 1, a0, b0);
            mfma_group(a1, b1);
          }
        }
        // the next step has landed (with three stages the one after it may
        // still be in flight), and every wave is done with this step's stage
        if (issued - (st + 2) >= 1)
          wait_vm_barrier<T::LD>();
        else
          wait_vm_barrier<0>();
        stage = stage == NST - 1 ? 0 : stage + 1;
      }
      if constexpr (kCarry) mfma_group(a1, b1);  // the window's last group
      if constexpr (M::kWindows) {  // fold the window's FP32 sums into the int32 weight sums (exact)
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FJ; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) U[i][j][v] += (int32_t)acc[i][j][v];
      }
    }
    // the weight's sums through LDS (every stage is idle), a part of the tile
    // at a time, then the FP64 slice-sum update of that part
    int32_t* Ul = reinterpret_cast<int32_t*>(lds);
    constexpr int HR = GBM / T::HALVES;  // tile rows per pass
#pragma unroll 1
    for (int h = 0; h < T::HALVES; ++h) {
      if (wm * (GBM / T::WM) / HR == h) {
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FJ; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int r = wm * (GBM / T::WM) - h * HR + 32 * i + 8 * (v >> 2) + 4 * fh + (v & 3);
              const int c = wn * (TBN / T::WN) + 32 * j + fr;
              if constexpr (M::kWindows)
                Ul[r * TBN + c] = U[i][j][v];
              else
                Ul[r * TBN + c] = acc[i][j][v];
            }
      }
      wait_vm_barrier<0>();
      slice_sum_update<HR, TBN, GNT>(Ul, eas + h * HR, fbs, t, s, SliceFmt<EB>::kBits, tid, m0 + h * HR, n0, m, n,
                                     npad, Sws, alpha, beta, C, ldc, gamma, D, ldd);
      wait_vm_barrier<0>();  // LDS is staging space again
    }
  }
}

// BF16 slices, 256 x 128 tiles.
__global__ __launch_bounds__(GNT, 1) void split_gemm(int64_t m, int64_t n, int64_t kpad, int s,
                                                     const uint8_t* __restrict__ Ap, const uint8_t* __restrict__ Bp,
                                                     int64_t mpad, int64_t npad, const int32_t* __restrict__ ea,
                                                     const int32_t* __restrict__ fb, double* __restrict__ Sws,
                                                     double alpha, double beta, double* __restrict__ C, int64_t ldc,
                                                     double gamma, const double* __restrict__ D, int64_t ldd) {
  __shared__ __attribute__((aligned(1024))) unsigned char lds[SliceTile<128>::NST * SliceTile<128>::STAGE];
  __shared__ int32_t eas[GBM], fbs[128];
  split_gemm_body<2, 128>(m, n, kpad, s, Ap, Bp, mpad, npad, ea, fb, Sws, alpha, beta, C, ldc, gamma, D, ldd, lds,
                          eas, fbs);
}

// INT8 slices, 256 x 128 tiles.
__global__ __launch_bounds__(GNT, 1) void split_gemm_i8(int64_t m, int64_t n, int64_t kpad, int s,
                                                        const uint8_t* __restrict__ Ap, const uint8_t* __restrict__ Bp,
                                                        int64_t mpad, int64_t npad, const int32_t* __restrict__ ea,
                                                        const int32_t* __restrict__ fb, double* __restrict__ Sws,
                                                        double alpha, double beta, double* __restrict__ C, int64_t ldc,
                                                        double gamma, const double* __restrict__ D, int64_t ldd) {
  __shared__ __attribute__((aligned(1024))) unsigned char lds[SliceTile<128>::NST * SliceTile<128>::STAGE];
  __shared__ int32_t eas[GBM], fbs[128];
  split_gemm_body<1, 128>(m, n, kpad, s, Ap, Bp, mpad, npad, ea, fb, Sws, alpha, beta, C, ldc, gamma, D, ldd, lds,
                          eas, fbs);
}

// INT8 slices, 256 x 256 tiles.
__global__ __launch_bounds__(GNT, 1) void split_gemm_i8w(int64_t m, int64_t n, int64_t kpad, int s,
                                                         const uint8_t* __restrict__ Ap, const uint8_t* __restrict__ Bp,
                                                         int64_t mpad, int64_t npad, const int32_t* __restrict__ ea,
                                                         const int32_t* __restrict__ fb, double* __restrict__ Sws,
                                                         double alpha, double beta, double* __restrict__ C, int64_t ldc,
                                                         double gamma, const double* __restrict__ D, int64_t ldd) {
  __shared__ __attribute__((aligned(1024))) unsigned char lds[SliceTile<256>::NST * SliceTile<256>::STAGE];
  __shared__ int32_t eas[GBM], fbs[256];
  split_gemm_body<1, 256>(m, n, kpad, s, Ap, Bp, mpad, npad, ea, fb, Sws, alpha, beta, C, ldc, gamma, D, ldd, lds,
                          eas, fbs);
}

inline int64_t pad64(int64_t x) { return (x + 63) / 64 * 64; }
inline int64_t pad128(int64_t x) { return (x + 127) / 128 * 128; }
inline int64_t pad256(int64_t x) { return (x + 255) / 256 * 256; }

}  // namespace

// Workspace: A planes [s][mp][kp], B planes [s][np][kp] (BF16 or INT8),
// row and column exponents (int32), column maxima (uint64), slice-sum tile
// [mp][np] (FP64), with mp = m rounded up to the slice-product kernel's 256
// tile rows, np = n rounded up to its tile columns (128 BF16; 128 or 256
// INT8, room for 256) and kp = k rounded up to a whole number of 128-byte
// chunks (64 BF16 or 128 INT8 elements).
static int64_t pad_k(int64_t k, SliceFormat f) { return f == kSliceInt8 ? pad128(k) : pad64(k); }
static int64_t pad_m(int64_t m) { return pad256(m); }

// A 256 x 256 INT8 tile moves half the plane bytes per product of a 256 x 128
// one and runs at 1.05 times its rate (8192^3 launches: 1880 against 1785
// TOP/s), so it takes about 1.90 times as long; the wide tiles are used when
// their waves over the CUs (one tile per CU at a time) end sooner.
constexpr double kWideTileTime = 1.90;

bool split_i8_wide(int64_t m, int64_t n, int cus) {
  const double rows = (double)(pad256(m) / 256);
  const double narrow = std::ceil(rows * (double)(pad128(n) / 128) / cus);
  const double wide = std::ceil(rows * (double)(pad256(n) / 256) / cus) * kWideTileTime;
  return wide < narrow;
}

size_t split_workspace_bytes(int64_t m, int64_t n, int64_t k, int s, SliceFormat f) {
  const int64_t mp = pad_m(m), np = f == kSliceInt8 ? pad256(n) : pad128(n);
  const int64_t kp = pad_k(k < kSplitMaxK ? k : kSplitMaxK, f);
  return (size_t)((int64_t)f * s * (mp + np) * kp + 4 * (mp + np) + 8 * np + 8 * mp * np);
}

static hipError_t split_panel(SliceFormat f, int64_t m, int64_t n, int64_t k, int s, double alpha, const double* A,
                              int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                              double gamma, const double* D, int64_t ldd, void* workspace, size_t ws_bytes,
                              hipStream_t stream, KernelTimer* timer, bool transb, bool reuse_a, bool reuse_b);

hipError_t launch_split_gemm(SliceFormat f, int64_t m, int64_t n, int64_t k, int s, double alpha, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                             double gamma, const double* D, int64_t ldd, void* workspace, size_t ws_bytes,
                             hipStream_t stream, KernelTimer* timer, bool transb, bool reuse_a, bool reuse_b) {
  // K panels of at most kSplitMaxK: C = alpha*S_0 + beta*C + gamma*D, then C = alpha*S_p + C.
  // reuse_a / reuse_b: the workspace still holds the slices of this A / B
  // panel (one K panel only), from the previous product on it
  if (m <= 0 || n <= 0) return hipSuccess;
  if (f != kSliceBF16 && f != kSliceInt8) return hipErrorInvalidValue;
  if (k <= kSplitMaxK)
    return split_panel(f, m, n, k, s, alpha, A, lda, B, ldb, beta, C, ldc, gamma, D, ldd, workspace, ws_bytes, stream,
                       timer, transb, reuse_a, reuse_b);
  if (reuse_a || reuse_b) return hipErrorInvalidValue;
  for (int64_t k0 = 0; k0 < k; k0 += kSplitMaxK) {
    const int64_t kk = (k - k0) < kSplitMaxK ? (k - k0) : kSplitMaxK;
    const bool first = k0 == 0;
    hipError_t e = split_panel(f, m, n, kk, s, alpha, A + k0, lda, transb ? B + k0 : B + k0 * ldb, ldb,
                               first ? beta : 1.0, C, ldc, first ? gamma : 0.0, D, ldd, workspace, ws_bytes, stream,
                               timer, transb, false, false);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t split_panel(SliceFormat f, int64_t m, int64_t n, int64_t k, int s, double alpha, const double* A,
                              int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                              double gamma, const double* D, int64_t ldd, void* workspace, size_t ws_bytes,
                              hipStream_t stream, KernelTimer* timer, bool transb, bool reuse_a, bool reuse_b) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (s < 1 || s > 8) return hipErrorInvalidValue;
  if (k <= 0) return launch_dgemm_f64(m, n, 0, alpha, nullptr, 1, nullptr, 1, beta, C, ldc, gamma, D, ldd, stream);
  int dev = 0, cus = 0;
  hipError_t qe = hipGetDevice(&dev);
  if (qe == hipSuccess) qe = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (qe != hipSuccess) return qe;
  const bool wide = f == kSliceInt8 && split_i8_wide(m, n, cus);
  const int64_t mp = pad_m(m), np = wide ? pad256(n) : pad128(n), kp = pad_k(k, f);
  if (split_workspace_bytes(m, n, k, s, f) > ws_bytes) return hipErrorInvalidValue;
  const int eb = (int)f;
  uint8_t* Ap = static_cast<uint8_t*>(workspace);
  uint8_t* Bp = Ap + (size_t)eb * s * mp * kp;
  int32_t* ea = reinterpret_cast<int32_t*>(Bp + (size_t)eb * s * np * kp);
  int32_t* fb = ea + mp;
  unsigned long long* bmax = reinterpret_cast<unsigned long long*>(fb + np);  // 8-byte aligned: mp, np even
  double* Sws = reinterpret_cast<double*>(bmax + np);
  if (gamma == 0.0) D = nullptr;
  if (kp > kSplitMaxK) return hipErrorInvalidValue;  // one K panel per call (split_rows holds a row)
  const dim3 rows_grid((unsigned)mp), cols_grid((unsigned)(kp / 64), (unsigned)(np / 64));
  auto slice_a = [&](auto S) {
    constexpr int sv = decltype(S)::value;
    if (f == kSliceInt8)
      hipLaunchKernelGGL((split_rows<sv, 1>), rows_grid, dim3(kRowThreads), 0, stream, m, k, A, lda, mp, kp, Ap, ea);
    else
      hipLaunchKernelGGL((split_rows<sv, 2>), rows_grid, dim3(kRowThreads), 0, stream, m, k, A, lda, mp, kp, Ap, ea);
  };
  // with transb the stored B^T (n x k) is sliced by rows, straight into the
  // transposed planes the slice-product kernels read
  const dim3 brows_grid((unsigned)np);
  auto slice_bt = [&](auto S) {
    constexpr int sv = decltype(S)::value;
    if (f == kSliceInt8)
      hipLaunchKernelGGL((split_rows<sv, 1>), brows_grid, dim3(kRowThreads), 0, stream, n, k, B, ldb, np, kp, Bp, fb);
    else
      hipLaunchKernelGGL((split_rows<sv, 2>), brows_grid, dim3(kRowThreads), 0, stream, n, k, B, ldb, np, kp, Bp, fb);
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
  if (!reuse_a) with_s(slice_a);
  if (reuse_b) {
  } else if (transb) {
    with_s(slice_bt);
  } else {
    hipLaunchKernelGGL(zero_u64, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, stream,
                       reinterpret_cast<uint64_t*>(bmax), np);
    hipLaunchKernelGGL(col_absmax, dim3((unsigned)((n + 255) / 256), (unsigned)((k + 255) / 256)), dim3(256), 0,
                       stream, k, n, B, ldb, bmax);
    hipLaunchKernelGGL(col_exponents, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, stream, np, bmax, fb);
    with_s(slice_b);
  }
  // one-dimensional grids: the kernels map workgroups to tiles in XCD bands
  const dim3 grid((unsigned)((np / (wide ? 256 : 128)) * (mp / GBM)));
  const bool timed = timer && timer->used < timer->count;
  if (timed) {
    const hipError_t e = hipEventRecord(timer->events[2 * timer->used], stream);
    if (e != hipSuccess) return e;
  }
  if (wide)
    hipLaunchKernelGGL(split_gemm_i8w, grid, dim3(GNT), 0, stream, m, n, kp, s, Ap, Bp, mp, np, ea, fb, Sws, alpha,
                       beta, C, ldc, gamma, D, ldd);
  else if (f == kSliceInt8)
    hipLaunchKernelGGL(split_gemm_i8, grid, dim3(GNT), 0, stream, m, n, kp, s, Ap, Bp, mp, np, ea, fb, Sws, alpha,
                       beta, C, ldc, gamma, D, ldd);
  else
    hipLaunchKernelGGL(split_gemm, grid, dim3(GNT), 0, stream, m, n, kp, s, Ap, Bp, mp, np, ea, fb, Sws, alpha, beta,
                       C, ldc, gamma, D, ldd);
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
