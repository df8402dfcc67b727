/*
 * CPU reference for the out-of-core product -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the bench's CPU-baseline leg load this
 * file's library.  It shares no code, header or constant with the HIP path.
 *
 * What it computes is the plain definition of the operation the paper's MMOOC
 * kernel performs (Section V, the text after Fig. 2):
 *     C_out[i][j] = alpha * S[i][j] + beta * C_in[i][j],
 *     S[i][j]     = sum over k = 0..K-1 of A[i][k] * B[k][j]
 * with A (M x K), B (K x N), C (M x N) row-major with leading dimensions
 * lda, ldb, ldc.  Tiling in the paper's method changes only the order of the
 * additions, so the reference is the untiled definition.
 *
 * Conventions taken where the paper is silent (reference-BLAS semantics):
 *   beta == 0          C_in is not read (NaN in C_in does not propagate);
 *   alpha == 0 or K==0  C_out = beta * C_in, A and B are not read.
 *
 * Arithmetic: each S[i][j] is accumulated in ascending k with a separate
 * multiply and add (this file is compiled with -ffp-contract=off, so no fused
 * multiply-add).  Alongside, D[i][j] = sum_k |A[i][k]| * |B[k][j]| is
 * accumulated; it is the denominator of the normalised error
 * max |C - C_ref| / (|A||B|)_ij used as the acceptance gate.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * Rows of the reference result.  Output row r corresponds to matrix row
 * rows[r] (rows == NULL: row r).  Cin holds the initial C values of those same
 * rows, row r at Cin + r*ldcin (it may be NULL when beta == 0).  Cref and Dabs
 * receive nrows x N values with leading dimension ldo; Dabs may be NULL.
 * Parallel over the requested rows (OpenMP).
 */
void oracle_gemm_rows(int64_t M, int64_t N, int64_t K, double alpha,
                      const double* A, int64_t lda, const double* B, int64_t ldb,
                      double beta, const double* Cin, int64_t ldcin,
                      const int64_t* rows, int64_t nrows,
                      double* Cref, double* Dabs, int64_t ldo) {
  (void)M;
  int use_ab = !(alpha == 0.0 || K == 0);
#pragma omp parallel
  {
    double* s = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double* d = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
      int64_t i = rows ? rows[r] : r;
      for (int64_t j = 0; j < N; ++j) { s[j] = 0.0; d[j] = 0.0; }
      if (use_ab) {
        for (int64_t k = 0; k < K; ++k) {
          double a = A[i * lda + k];
          double aa = fabs(a);
          const double* b = B + k * ldb;
          for (int64_t j = 0; j < N; ++j) {
            double p = a * b[j];
            s[j] = s[j] + p;
            d[j] = d[j] + aa * fabs(b[j]);
          }
        }
      }
      double* out = Cref + r * ldo;
      const double* cin = Cin ? Cin + r * ldcin : NULL;
      for (int64_t j = 0; j < N; ++j) {
        double v;
        if (!use_ab) {
          v = (beta == 0.0) ? 0.0 : beta * cin[j];
        } else if (beta == 0.0) {
          v = alpha * s[j];
        } else {
          double t1 = alpha * s[j];
          double t2 = beta * cin[j];
          v = t1 + t2;
        }
        out[j] = v;
      }
      if (Dabs) memcpy(Dabs + r * ldo, d, sizeof(double) * (size_t)N);
    }
    free(s);
    free(d);
  }
}

/* Number of threads the parallel region above uses (for reporting). */
int oracle_threads(void) {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    {
#ifdef _OPENMP
      extern int omp_get_num_threads(void);
      n = omp_get_num_threads();
#endif
    }
  }
  return n;
}
