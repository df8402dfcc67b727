"""Reference for the split-BF16 product -- TEST INFRASTRUCTURE ONLY.

The paper computes its tile products in FP64 only.  The split form computes
the same FP64 product from error-free slices (Ozaki, Ogita, Oishi and Rump,
"Error-free transformations of matrix multiplication by using fast routines
of matrix multiplication and its applications", Numer. Algorithms 59, 2012),
with slices small enough that every slice product is exact on BF16 matrix
units with FP32 accumulation.  Steps, for one K panel of A (m x k) and B (k x n):

 1. e_i is the smallest integer with max_k |A_ik| < 2^e_i (row i of A);
    f_j likewise for column j of B.  A zero row or column gets exponent 0
    (its slices are all zero).
 2. With r = A_ik, for p = 1..s:  m_p = rint(r * 2^(8p - e_i)),
    r = r - m_p * 2^(e_i - 8p).  Every step is exact (power-of-two scaling);
    |m_1| <= 256 and |m_p| <= 128 for p >= 2, integers that BF16 (8
    significant bits) holds exactly.  B is sliced the same way with f_j.
 3. For p + q <= s + 1: T_pq = sum_k mA_p[i,k] * mB_q[k,j].  Every product is an
    integer below 2^16 in magnitude, so a sum over at most 256 terms stays
    below 2^24 and FP32 accumulates it exactly; the chunk sums are then added
    exactly in FP64.  (Here the integer sums are formed directly in FP64,
    exact as long as k * 2^16 < 2^53.)
 4. The pairs with the same weight t = p + q are added first (exact integer
    sums U_t), then S = sum over t = s+1 down to 2 of U_t * 2^(e_i + f_j - 8t)
    is accumulated in FP64 from the smallest weight to the largest.
 5. C = alpha * S + beta * C (beta == 0: C is not read).  When K is processed
    in panels of kb, steps 1-4 run per panel and C accumulates:
    C = alpha*S_0 + beta*C, then C = alpha*S_p + C.

The grouping of equal weights in step 4 is a reading of the method, which
only requires the slice sum in FP64, and grouping keeps the result
independent of how the equal-weight pairs are ordered.

Format "i8" is the same scheme with slices that INT8 matrix units multiply
exactly into INT32 sums: in step 2, m_p = trunc(r * 2^(7p - e_i)) (rounded
toward zero), r = r - m_p * 2^(e_i - 7p), so |m_p| <= 127 (|r| < 2^(e_i - 7(p-1))
before step p); in steps 3-4 the weights are 2^(e_i + f_j - 7t).  A product
of two slices is below 2^14 in magnitude, so an INT32 sum over every pair of
one weight is exact for s * k * 2^14 < 2^31.  Seven bits per slice instead of
eight: for the same truncation error the i8 form needs about 8/7 as many
slices.
"""
import numpy as np

# slice format: (bits per slice, rounding of each slice)
FORMATS = {"bf16": (8, np.rint), "i8": (7, np.trunc)}


def exponents(X, axis):
    """Smallest integer e with max |x| < 2^e along `axis` (axis=1: rows, 0: columns)."""
    mx = np.max(np.abs(X), axis=axis) if X.shape[axis] else np.zeros(X.shape[1 - axis])
    _, e = np.frexp(mx)
    e = e.astype(np.int64)
    e[mx == 0] = 0
    return e


def slices(X, e, s, axis, fmt="bf16"):
    """s integer-valued slices of X and the final remainder (float64 arrays).

    axis=1: e holds one exponent per row; axis=0: one per column."""
    bits, rnd = FORMATS[fmt]
    eb = e[:, None] if axis == 1 else e[None, :]
    r = np.array(X, dtype=np.float64, copy=True)
    out = []
    for p in range(1, s + 1):
        m = rnd(np.ldexp(r, (bits * p - eb).astype(np.int64)))
        r = r - np.ldexp(m, (eb - bits * p).astype(np.int64))
        out.append(m)
    return out, r


def slice_sum(A, B, s, fmt="bf16"):
    """Steps 1-4 for one panel: the FP64 slice-sum S of A @ B."""
    m, k = A.shape
    n = B.shape[1]
    if k == 0 or m == 0 or n == 0:
        return np.zeros((m, n))
    e = exponents(A, 1)
    f = exponents(B, 0)
    bits = FORMATS[fmt][0]
    sa, _ = slices(A, e, s, 1, fmt)
    sb, _ = slices(B, f, s, 0, fmt)
    S = np.zeros((m, n))
    for t in range(s + 1, 1, -1):
        U = np.zeros((m, n))
        for p in range(1, t):
            q = t - p
            U = U + sa[p - 1] @ sb[q - 1]
        S = S + np.ldexp(U, (e[:, None] + f[None, :] - bits * t).astype(np.int64))
    return S


def split_gemm(alpha, A, B, beta, C, s, kb=None, fmt="bf16"):
    """alpha*A@B + beta*C by the split scheme with s slices (K panels of kb)."""
    M, K = A.shape
    N = B.shape[1]
    kb = K if not kb else kb
    Cout = np.array(C, dtype=np.float64, copy=True) if beta != 0.0 else np.zeros((M, N))
    if alpha == 0.0 or K == 0:
        return beta * Cout if beta != 0.0 else np.zeros((M, N))
    first = True
    for k0 in range(0, K, kb):
        S = slice_sum(A[:, k0:k0 + kb], B[k0:k0 + kb, :], s, fmt)
        if first:
            Cout = alpha * S + beta * Cout if beta != 0.0 else alpha * S
            first = False
        else:
            Cout = alpha * S + Cout
    return Cout


def truncation_bound(A, B, s, fmt="bf16"):
    """A bound on |S - A@B| per entry from the slice remainders:
    |A@B - sum_{p+q<=s+1} ...| <= sum over dropped pairs + remainder terms,
    bounded here by (s+1) * 2^(-8s) * 2^(e_i+f_j) * k for BF16 slices and
    (s+2) * 2^(-7s) * 2^(e_i+f_j) * k for INT8 slices (crude, entrywise: a
    truncated INT8 slice keeps a remainder up to one unit of its last digit,
    twice the rounded BF16 slice's half unit)."""
    e = exponents(A, 1)
    f = exponents(B, 0)
    k = A.shape[1]
    lead = (s + 1) * 2.0 ** (-8 * s) if fmt == "bf16" else (s + 2) * 2.0 ** (-7 * s)
    return lead * np.ldexp(np.ones((A.shape[0], B.shape[1])), (e[:, None] + f[None, :])) * k
