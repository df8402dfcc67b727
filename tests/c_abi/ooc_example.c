/* A plain C caller of the library: a tiled out-of-core product through a
 * small budget, checked exactly (integer-valued data, every sum exact) against
 * a naive triple loop; then the same product from the split-BF16 and the
 * split-INT8 forms, whose slices are exact for these small integers; then an
 * out-of-core Cholesky factorisation of A = L L^T with an integer L and the
 * Cholesky solve of X A = B with an integer X, both exact.  Prints "ok" on
 * success. */
#include <stdio.h>
#include <stdlib.h>

#include "ooc.h"

static int check(const double* C, const double* R, int64_t n) {
  for (int64_t x = 0; x < n; ++x)
    if (C[x] != R[x]) {
      fprintf(stderr, "mismatch at %lld: %.17g vs %.17g\n", (long long)x, C[x], R[x]);
      return 1;
    }
  return 0;
}

/* Factor A = L L^T (n = 300, panels of 128 columns through a 1 MiB budget)
 * and solve X A = B for 50 right-hand sides; every pivot is a perfect square
 * and every quotient exact, so L and X come back exactly. */
static int cholesky(void) {
  const int64_t n = 300, m = 50;
  double *A = NULL, *Bm = NULL;
  if (ooc_host_alloc((void**)&A, n * n * 8) || ooc_host_alloc((void**)&Bm, m * n * 8)) return 1;
  double* L = calloc(n * n, 8);
  double* X = malloc(m * n * 8);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < i; ++j) L[i * n + j] = (double)((i * 5 + j * 3) % 7 - 3);
    L[i * n + i] = (double)(1 + i % 4);
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t k = 0; k <= (i < j ? i : j); ++k) s += L[i * n + k] * L[j * n + k];
      A[i * n + j] = s;
    }
  for (int64_t x = 0; x < m * n; ++x) X[x] = (double)(x % 11 - 5);
  for (int64_t r = 0; r < m; ++r)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t k = 0; k < n; ++k) s += X[r * n + k] * A[k * n + j];
      Bm[r * n + j] = s;
    }
  int64_t info = -1;
  ooc_stats st;
  ooc_status s = ooc_potrf(n, A, n, (size_t)1 << 20, NULL, &info, &st);
  if (s != OOC_OK || info != 0 || st.blocks_done < 3) {
    fprintf(stderr, "ooc_potrf: %d info %lld panels %lld %s\n", (int)s, (long long)info, (long long)st.blocks_done,
            ooc_last_error());
    return 1;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j)
      if (A[i * n + j] != L[i * n + j]) {
        fprintf(stderr, "factor mismatch at (%lld, %lld)\n", (long long)i, (long long)j);
        return 1;
      }
  s = ooc_potrs(m, n, A, n, Bm, n, (size_t)1 << 20, NULL, &st);
  if (s != OOC_OK) {
    fprintf(stderr, "ooc_potrs: %d %s\n", (int)s, ooc_last_error());
    return 1;
  }
  if (check(Bm, X, m * n)) return 1;
  ooc_host_free(A);
  ooc_host_free(Bm);
  free(L);
  free(X);
  return 0;
}

int main(void) {
  const int64_t M = 300, N = 200, K = 250;
  double *A = NULL, *B = NULL, *C = NULL;
  if (ooc_host_alloc((void**)&A, M * K * 8) || ooc_host_alloc((void**)&B, K * N * 8) ||
      ooc_host_alloc((void**)&C, M * N * 8)) {
    fprintf(stderr, "host alloc: %s\n", ooc_last_error());
    return 2;
  }
  double* C0 = malloc(M * N * 8);
  double* R = malloc(M * N * 8);
  for (int64_t i = 0; i < M; ++i)
    for (int64_t k = 0; k < K; ++k) A[i * K + k] = (double)((i * 7 + k * 3) % 9 - 4);
  for (int64_t k = 0; k < K; ++k)
    for (int64_t j = 0; j < N; ++j) B[k * N + j] = (double)((k * 5 + j * 11) % 7 - 3);
  for (int64_t x = 0; x < M * N; ++x) C0[x] = (double)(x % 13 - 6);
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) {
      double s = 0.0;
      for (int64_t k = 0; k < K; ++k) s += A[i * K + k] * B[k * N + j];
      R[i * N + j] = 2.0 * s + 0.5 * C0[i * N + j];
    }
  const size_t budget = (size_t)1 << 20; /* below the 1.48 MB of the three operands */
  for (int form = 0; form < 3; ++form) {
    for (int64_t x = 0; x < M * N; ++x) C[x] = C0[x];
    ooc_opts o = {0};
    if (form > 0) {
      o.precision = form == 1 ? OOC_SPLIT_BF16 : OOC_SPLIT_INT8;
      o.slices = 2;
    }
    ooc_stats st;
    ooc_status s = ooc_gemm(M, N, K, 2.0, A, K, B, N, 0.5, C, N, form ? (size_t)2 << 20 : budget, &o, &st);
    if (s != OOC_OK) {
      fprintf(stderr, "ooc_gemm: %d %s\n", (int)s, ooc_last_error());
      return 3;
    }
    if (st.arena_bytes > (form ? (size_t)2 << 20 : budget) || st.tasks < 2) {
      fprintf(stderr, "not tiled within the budget\n");
      return 4;
    }
    if (check(C, R, M * N)) return 5;
  }
  ooc_host_free(A);
  ooc_host_free(B);
  ooc_host_free(C);
  free(C0);
  free(R);
  if (cholesky()) return 6;
  ooc_release(-1);
  printf("ok\n");
  return 0;
}
