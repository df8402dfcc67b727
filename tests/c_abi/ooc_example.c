/* A plain C caller of the library: a tiled out-of-core product through a
 * small budget, checked exactly (integer-valued data, every sum exact) against
 * a naive triple loop; then the same product from the split-BF16 and the
 * split-INT8 forms, whose slices are exact for these small integers.  Prints
 * "ok" on success. */
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
  ooc_release(-1);
  printf("ok\n");
  return 0;
}
