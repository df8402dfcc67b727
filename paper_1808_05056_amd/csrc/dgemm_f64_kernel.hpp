// FP64 tile product on CDNA4 matrix cores: C = alpha*A*B + beta*C + gamma*D, row-major.
//
// This is the DGEMM stage of the paper's pipeline (Section V, stage "DGEMM"
// of Fig. 4), which the paper delegates to a vendor library.  Here it is a
// hand-written gfx950 kernel, templated on its tile shape:
//   * a workgroup of 64*WM*WN threads computes a BM x BN tile of C; wave
//     (wm, wn) computes a (BM/WM) x (BN/WN) sub-tile as FM x FN blocks of
//     V_MFMA_F64_16X16X4_F64 (FM = BM/WM/16, FN = BN/WN/16);
//   * K advances in steps of BK: the next step's A and B tiles are fetched
//     from global memory into registers (16-byte loads along the contiguous
//     dimension) while the current step is multiplied out of LDS; LDS holds
//     two steps, so one barrier per step suffices;
//   * A is stored transposed in LDS (k-major) so that the 16 lanes feeding one
//     MFMA row read 16 consecutive doubles, like the B reads;
//   * optionally (PRIO) a wave raises its priority while it issues the step's
//     matrix instructions and lowers it before its global-load and LDS-store
//     phase, so the wave sharing its SIMD that has MFMAs ready is favoured;
//   * workgroups are numbered so that each of the 8 XCDs (workgroups are dealt
//     to them round robin) receives a contiguous band of tiles, ordered in
//     groups of GROUP_M tile rows so that concurrently running tiles share A
//     rows and B columns in that XCD's L2.
// Operand layout of V_MFMA_F64_16X16X4_F64 (one wave): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator element v of lane l is
// D[l/16 + 4v][l%16].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ooc {
namespace dgemm {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int GROUP_M = 8;
constexpr int PAD = 4;  // LDS row padding (doubles)

template <int BM, int BN, int BK, int WM, int WN>
struct Cfg {
  static constexpr int NT = 64 * WM * WN;       // threads
  static constexpr int FM = BM / WM / 16;       // MFMA blocks per wave along M
  static constexpr int FN = BN / WN / 16;       // along N
  static constexpr int VA = BM * BK / NT;       // A elements per thread per step
  static constexpr int VB = BK * BN / NT;       // B elements per thread per step
  static constexpr int A_TPR = BK / VA;         // threads per A row
  static constexpr int B_TPR = BN / VB;         // threads per B row
  static_assert(FM >= 1 && FN >= 1, "wave tile too small");
  static_assert(BM % (WM * 16) == 0 && BN % (WN * 16) == 0, "tile / wave mismatch");
  static_assert(VA >= 2 && VA % 2 == 0 && BK % VA == 0, "A load split");
  static_assert(VB >= 2 && VB % 2 == 0 && BN % VB == 0, "B load split");
  static_assert(BK % 4 == 0, "BK must be a multiple of the MFMA k (4)");
  static constexpr size_t LDS_BYTES = 2 * (size_t)BK * ((BM + PAD) + (BN + PAD)) * 8;
};

// Tuning knobs: GM = tile rows per L2 group, PRIO = raise the wave priority
// while it issues its MFMA block, PIPE = load the next k sub-step's operands
// from LDS before issuing the current sub-step's MFMAs.
template <int BM, int BN, int BK, int WM, int WN, bool VEC, int MINBLOCKS, int GM = GROUP_M, bool PRIO = false,
          bool PIPE = false, bool TB = false>
__global__ __launch_bounds__(64 * WM * WN, MINBLOCKS) void kernel(
    int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A, int64_t lda,
    const double* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
    double gamma, const double* __restrict__ D, int64_t ldd, int tiles_m, int tiles_n, int64_t tri) {
  using CF = Cfg<BM, BN, BK, WM, WN>;
  constexpr int FM = CF::FM, FN = CF::FN, VA = CF::VA, VB = CF::VB;
  __shared__ __attribute__((aligned(16))) double As[2][BK][BM + PAD];
  __shared__ __attribute__((aligned(16))) double Bs[2][BK][BN + PAD];

  // ---- tile selection: XCD bands, then groups of tile rows -----------------------
  const int ntiles = tiles_m * tiles_n;
  const int b = blockIdx.x;
  const int xcd = b & 7, local = b >> 3;
  const int q = ntiles >> 3, r = ntiles & 7;
  const int lin = xcd * q + (xcd < r ? xcd : r) + local;
  const int group = lin / (GM * tiles_n);
  const int first_m = group * GM;
  const int gm = (tiles_m - first_m) < GM ? (tiles_m - first_m) : GM;
  const int in_group = lin - group * GM * tiles_n;
  const int tm = first_m + in_group % gm;
  const int tn = in_group / gm;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WN, wn = wid % WN;

  // global-load assignment: A row ar, k offset ak (VA doubles); B k-row bk, column offset bn (VB doubles),
  // or with TB B column (row of the transposed B) btn, k offset btk (VB doubles)
  const int ar = tid / CF::A_TPR, ak = (tid % CF::A_TPR) * VA;
  const int bk = tid / CF::B_TPR, bn = (tid % CF::B_TPR) * VB;
  const int btn = tid / (BK / VB), btk = (tid % (BK / VB)) * VB;

  const bool full_mn = (m0 + BM <= M) && (n0 + BN <= N);
  double ra[VA], rb[VB];

  auto gload = [&](int64_t k0) {
    const bool fast = full_mn && (k0 + BK <= K);
    const int64_t arow = m0 + ar;
    const int64_t brow = k0 + bk;
    if (fast) {
      const double* pa = A + arow * lda + k0 + ak;
      const double* pb = TB ? B + (n0 + btn) * ldb + k0 + btk : B + brow * ldb + n0 + bn;
      if (VEC) {
#pragma unroll
        for (int e = 0; e < VA; e += 2) {
          double2 v = *reinterpret_cast<const double2*>(pa + e);
          ra[e] = v.x; ra[e + 1] = v.y;
        }
#pragma unroll
        for (int e = 0; e < VB; e += 2) {
          double2 v = *reinterpret_cast<const double2*>(pb + e);
          rb[e] = v.x; rb[e + 1] = v.y;
        }
      } else {
#pragma unroll
        for (int e = 0; e < VA; ++e) ra[e] = pa[e];
#pragma unroll
        for (int e = 0; e < VB; ++e) rb[e] = pb[e];
      }
    } else {
      // edge tiles: every load reads an address inside the operand (row and
      // k clamped) and the value is then selected, so that no load waits for
      // the one before it
      const int64_t arc = arow < M ? arow : M - 1;
#pragma unroll
      for (int e = 0; e < VA; ++e) {
        const int64_t kk = k0 + ak + e;
        const double v = A[arc * lda + (kk < K ? kk : K - 1)];
        ra[e] = (arow < M && kk < K) ? v : 0.0;
      }
      if (TB) {
        const int64_t nn = n0 + btn;
        const int64_t nnc = nn < N ? nn : N - 1;
#pragma unroll
        for (int e = 0; e < VB; ++e) {
          const int64_t kk = k0 + btk + e;
          const double v = B[nnc * ldb + (kk < K ? kk : K - 1)];
          rb[e] = (nn < N && kk < K) ? v : 0.0;
        }
      } else {
        const int64_t brc = brow < K ? brow : K - 1;
#pragma unroll
        for (int e = 0; e < VB; ++e) {
          const int64_t nn = n0 + bn + e;
          const double v = B[brc * ldb + (nn < N ? nn : N - 1)];
          rb[e] = (brow < K && nn < N) ? v : 0.0;
        }
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < VA; ++e) As[buf][ak + e][ar] = ra[e];
    if (TB) {
#pragma unroll
      for (int e = 0; e < VB; ++e) Bs[buf][btk + e][btn] = rb[e];
    } else {
#pragma unroll
      for (int e = 0; e < VB; e += 2) *reinterpret_cast<double2*>(&Bs[buf][bk][bn + e]) = make_double2(rb[e], rb[e + 1]);
    }
  };

  dbl4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (K + BK - 1) / BK;
  if (nk > 0) {
    gload(0);
    lstore(0);
    __syncthreads();
  }
  const int lrow = lane & 15, lk = lane >> 4;
  const int am0 = wm * (BM / WM), bn0 = wn * (BN / WN);
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) gload((kt + 1) * BK);
    if (PRIO) __builtin_amdgcn_s_setprio(1);
    if (PIPE) {
      double a[2][FM], bb[2][FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[0][i] = As[buf][lk][am0 + i * 16 + lrow];
#pragma unroll
      for (int j = 0; j < FN; ++j) bb[0][j] = Bs[buf][lk][bn0 + j * 16 + lrow];
#pragma unroll
      for (int s = 0; s < BK / 4; ++s) {
        const int cur = s & 1;
        if (s + 1 < BK / 4) {
          const int kn = (s + 1) * 4 + lk;
#pragma unroll
          for (int i = 0; i < FM; ++i) a[cur ^ 1][i] = As[buf][kn][am0 + i * 16 + lrow];
#pragma unroll
          for (int j = 0; j < FN; ++j) bb[cur ^ 1][j] = Bs[buf][kn][bn0 + j * 16 + lrow];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][i], bb[cur][j], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < BK / 4; ++s) {
        const int kk = s * 4 + lk;
        double a[FM], bb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = As[buf][kk][am0 + i * 16 + lrow];
#pragma unroll
        for (int j = 0; j < FN; ++j) bb[j] = Bs[buf][kk][bn0 + j * 16 + lrow];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
      }
    }
    if (PRIO) __builtin_amdgcn_s_setprio(0);
    if (kt + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: C = alpha*acc + beta*C + gamma*D (C, D not read when their weight is 0)
  // One row of MFMA blocks at a time: its C (and D) values are loaded first,
  // from addresses clamped into the matrices, so that the loads are in flight
  // together; then the results are formed, then stored, limited to the
  // tile's part of C (and, with a triangle mask, to row - col >= tri).  No
  // load or result follows a store within a row of blocks, so the stores
  // wait for nothing.
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    double cv[FN][4], dv[FN][4];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t col = n0 + bn0 + j * 16 + lrow;
      const int64_t cc = col < N ? col : N - 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + am0 + i * 16 + lk + 4 * v;
        const int64_t rc = row < M ? row : M - 1;
        if (beta != 0.0) cv[j][v] = C[rc * ldc + cc];
        if (gamma != 0.0) dv[j][v] = D[rc * ldd + cc];
      }
    }
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double val = alpha * acc[i][j][v];
        if (beta != 0.0) val += beta * cv[j][v];
        if (gamma != 0.0) val += gamma * dv[j][v];
        // formed here, before any store (the compiler would otherwise sink
        // it into the conditional store, behind a wait for the last store)
        asm volatile("" : "+v"(val));
        acc[i][j][v] = val;
      }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t col = n0 + bn0 + j * 16 + lrow;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + am0 + i * 16 + lk + 4 * v;
        if (row < M && col < N && row - col >= tri) C[row * ldc + col] = acc[i][j][v];
      }
    }
  }
}

// Launch one configuration; checks the grid size and picks 16-byte loads when
// the operands allow them.
template <int BM, int BN, int BK, int WM, int WN, int MINBLOCKS, int GM = GROUP_M, bool PRIO = false,
          bool PIPE = false, bool TB = false>
hipError_t launch(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda, const double* B,
                  int64_t ldb, double beta, double* C, int64_t ldc, double gamma, const double* D, int64_t ldd,
                  int64_t tri, hipStream_t stream) {
  static_assert(!TB || ((BK / (BN * BK / (64 * WM * WN))) * BN == 64 * WM * WN), "TB load split");
  using CF = Cfg<BM, BN, BK, WM, WN>;
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t tm = (m + BM - 1) / BM, tn = (n + BN - 1) / BN;
  if (tm * tn > 0x7fffffff) return hipErrorInvalidValue;
  const bool vec = ((lda & 1) == 0) && ((ldb & 1) == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
  if (k <= 0) { A = nullptr; B = nullptr; }
  if (gamma == 0.0) D = nullptr;
  dim3 grid((unsigned)(tm * tn)), block(CF::NT);
  if (vec)
    hipLaunchKernelGGL((kernel<BM, BN, BK, WM, WN, true, MINBLOCKS, GM, PRIO, PIPE, TB>), grid, block, 0, stream, m, n,
                       k, alpha, A, lda, B, ldb, beta, C, ldc, gamma, D, ldd, (int)tm, (int)tn, tri);
  else
    hipLaunchKernelGGL((kernel<BM, BN, BK, WM, WN, false, MINBLOCKS, GM, PRIO, PIPE, TB>), grid, block, 0, stream, m,
                       n, k, alpha, A, lda, B, ldb, beta, C, ldc, gamma, D, ldd, (int)tm, (int)tn, tri);
  return hipGetLastError();
}

}  // namespace dgemm
}  // namespace ooc
