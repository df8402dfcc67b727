/*
 * Seeded, counter-based generator of synthetic matrix entries.
 *
 * This module only produces inputs. It holds none of the matrix-product
 * arithmetic; both the HIP path (through its tests and bench) and the CPU
 * reference take their operands from here, so that any entry of A, B or the
 * initial C can be regenerated on its own from (seed, matrix id, row, col).
 *
 * Counter-based construction: the 64-bit key
 *     key = (seed XOR (mat << 56)) + (row << 32) + col      (mod 2^64)
 * is passed through the SplitMix64 output function (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014), and the top
 * 53 bits of the result give u in [0, 1).  Distributions:
 *   SYN_UNIFORM  2u - 1                      in [-1, 1)
 *   SYN_NORMAL   Box-Muller: sqrt(-2 ln(1-u1)) cos(2 pi u2), u2 from key ^ 2^63
 *   SYN_ONES     1
 *   SYN_INT      an integer in [-4, 4] (exact-arithmetic test inputs)
 *   SYN_ZERO     0
 * Optional scaling multiplies entry (r, c) by 2^(x_r) * 2^(y_c), with x_r
 * uniform in [row_lo, row_hi] drawn from key(seed, SYN_ROWSCALE_MAT, r, 0) and
 * y_c uniform in [col_lo, col_hi] from key(seed, SYN_COLSCALE_MAT, 0, c).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define SYN_UNIFORM 0
#define SYN_NORMAL 1
#define SYN_ONES 2
#define SYN_INT 3
#define SYN_ZERO 4

#define SYN_ROWSCALE_MAT 3u
#define SYN_COLSCALE_MAT 4u

typedef struct {
  uint64_t seed;
  uint32_t mat;     /* matrix id: A=0, B=1, C=2 by convention */
  int32_t dist;     /* SYN_* */
  double row_lo, row_hi; /* base-2 exponent range per row; equal bounds 0,0 = none */
  double col_lo, col_hi; /* base-2 exponent range per column */
} syn_spec;

static inline uint64_t syn_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t syn_key(uint64_t seed, uint64_t mat, uint64_t r, uint64_t c) {
  return (seed ^ (mat << 56)) + (r << 32) + c;
}

static inline double syn_u(uint64_t z) { return (double)(z >> 11) * 0x1.0p-53; }

static inline double syn_base(const syn_spec* s, uint64_t r, uint64_t c) {
  uint64_t k = syn_key(s->seed, s->mat, r, c);
  switch (s->dist) {
    case SYN_UNIFORM: return 2.0 * syn_u(syn_mix(k)) - 1.0;
    case SYN_NORMAL: {
      double u1 = syn_u(syn_mix(k));
      double u2 = syn_u(syn_mix(k ^ 0x8000000000000000ull));
      return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
    }
    case SYN_ONES: return 1.0;
    case SYN_INT: return (double)((int64_t)(syn_mix(k) % 9u) - 4);
    default: return 0.0;
  }
}

static inline double syn_rowscale(const syn_spec* s, uint64_t r) {
  if (s->row_lo == 0.0 && s->row_hi == 0.0) return 1.0;
  double u = syn_u(syn_mix(syn_key(s->seed, SYN_ROWSCALE_MAT, r, 0)));
  return exp2(s->row_lo + (s->row_hi - s->row_lo) * u);
}

static inline double syn_colscale(const syn_spec* s, uint64_t c) {
  if (s->col_lo == 0.0 && s->col_hi == 0.0) return 1.0;
  double u = syn_u(syn_mix(syn_key(s->seed, SYN_COLSCALE_MAT, 0, c)));
  return exp2(s->col_lo + (s->col_hi - s->col_lo) * u);
}

/* One entry. */
double syn_entry(const syn_spec* s, int64_t r, int64_t c) {
  double v = syn_base(s, (uint64_t)r, (uint64_t)c);
  if (!(s->row_lo == 0.0 && s->row_hi == 0.0)) v *= syn_rowscale(s, (uint64_t)r);
  if (!(s->col_lo == 0.0 && s->col_hi == 0.0)) v *= syn_colscale(s, (uint64_t)c);
  return v;
}

/*
 * Fill X (row-major, leading dimension ld) with nrows x ncols entries.
 * Row r of X holds matrix row rows[r] (or row0 + r when rows is NULL);
 * column c holds matrix column col0 + c.  Parallel over rows.
 */
void syn_fill(double* X, int64_t ld, const int64_t* rows, int64_t row0, int64_t nrows,
              int64_t col0, int64_t ncols, const syn_spec* s) {
  int scaled_cols = !(s->col_lo == 0.0 && s->col_hi == 0.0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nrows; ++r) {
    uint64_t gr = (uint64_t)(rows ? rows[r] : row0 + r);
    double rs = syn_rowscale(s, gr);
    double* x = X + r * ld;
    for (int64_t c = 0; c < ncols; ++c) {
      uint64_t gc = (uint64_t)(col0 + c);
      double v = syn_base(s, gr, gc) * rs;
      if (scaled_cols) v *= syn_colscale(s, gc);
      x[c] = v;
    }
  }
}

/* Fill with a NaN (used to check that an operand is not read). */
void syn_fill_nan(double* X, int64_t ld, int64_t nrows, int64_t ncols) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r)
    for (int64_t c = 0; c < ncols; ++c) X[r * ld + c] = NAN;
}
