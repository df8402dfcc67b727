"""CPU reference ("oracle") for the out-of-core FP64 product -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the bench's CPU-baseline leg may import
this package.  It shares no code with the HIP path and never imports it.

Contents
  gemm_ref.c     the plain definition C = alpha*A*B + beta*C (untiled, k ascending,
                 no FMA) plus the |A||B| denominators of the error gate
  plan_ref.py    the paper's partitioner (Section V): h, w and the footprint rule
  sched_ref.py   the pipeline's dependency rules (Fig. 2 events) and a CPU
                 executor/hazard checker for an operation list
  split_ref.py   the split-BF16 product (error-free slicing, Ozaki et al. 2012)
  mlp_ref.py     the MLP planner network: forward, backward, MSE, Adam in FP64
  chol_ref.py    Cholesky factorisation, symmetric rank-k update, forward and back
                 substitution for the two right-hand triangular solves, the Cholesky
                 solve, and their backward-error bounds (plain definitions)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")


def build():
    """Compile gemm_ref.c (gcc -O2 -ffp-contract=off, OpenMP) into liboracle.so."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", _SO, os.path.join(_HERE, "gemm_ref.c"), "-lm"]
    subprocess.check_call(cmd)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.oracle_gemm_rows.argtypes = [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp, i64, vp, vp, i64]
        L.oracle_gemm_rows.restype = None
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(X):
    return None if X is None else X.ctypes.data


def _ld(X):
    if X is None:
        return 0
    assert X.dtype == np.float64 and X.strides[-1] == 8
    return X.strides[0] // 8 if X.ndim == 2 else X.shape[-1]


def gemm_rows(alpha, A, B, beta, Cin_rows, rows=None, want_denominator=True):
    """Reference rows of alpha*A@B + beta*C.

    A (M x K) and B (K x N) are float64 row-major views (any row pitch).
    rows: matrix rows to compute (None = all M rows).  Cin_rows holds the
    initial C values of exactly those rows (row r of Cin_rows = matrix row
    rows[r]); it may be None when beta == 0.
    Returns (Cref, D) with D = |A||B| for the same entries (or None).
    """
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    if rows is None:
        nrows = M
        rows_arr = None
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = rows_arr.shape[0]
        assert nrows == 0 or (rows_arr.min() >= 0 and rows_arr.max() < M)
    if beta != 0.0:
        assert Cin_rows is not None and Cin_rows.shape == (nrows, N)
    Cref = np.empty((nrows, N), dtype=np.float64)
    D = np.empty((nrows, N), dtype=np.float64) if want_denominator else None
    if nrows == 0 or N == 0:
        return Cref, D
    Cin_use = Cin_rows if beta != 0.0 else None
    lib().oracle_gemm_rows(M, N, K, float(alpha), _ptr(A) if K else None, _ld(A) if K else 0,
                           _ptr(B) if K else None, _ld(B) if K else 0, float(beta),
                           _ptr(Cin_use), _ld(Cin_use), _ptr(rows_arr), nrows,
                           Cref.ctypes.data, _ptr(D), N)
    return Cref, D


def threads():
    return int(lib().oracle_threads())


def gate_denominator(alpha, D_ab, beta, Cin):
    """Denominator of the acceptance gate: |alpha| (|A||B|)_ij + |beta| |C_in|_ij.

    For alpha = 1 and beta = 0 this is exactly (|A||B|)_ij.  The beta term is
    the scale of the final addition alpha*S + beta*C: where |beta C_in| exceeds
    (|A||B|)_ij by more than ~2^52 * 1e-12, a single rounding of that addition
    already exceeds 1e-12 of (|A||B|)_ij, whatever the product's accuracy."""
    den = abs(alpha) * np.asarray(D_ab, dtype=np.float64)
    if beta != 0.0 and Cin is not None:
        den = den + abs(beta) * np.abs(np.asarray(Cin, dtype=np.float64))
    return den


def normalized_error(C, Cref, D):
    """max over entries of |C - Cref| / (|A||B|)_ij; where the denominator is 0
    the entries must agree exactly (else the error is reported as inf)."""
    C = np.asarray(C, dtype=np.float64)
    Cref = np.asarray(Cref, dtype=np.float64)
    diff = np.abs(C - Cref)
    same = (C == Cref) | (np.isnan(C) & np.isnan(Cref))
    zero = D == 0
    if np.any(zero & ~same):
        return float("inf")
    if np.any(~zero & (np.isnan(diff))):
        return float("inf")
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(zero | same, 0.0, diff / np.where(zero, 1.0, D))
    return float(r.max()) if r.size else 0.0


def errors(C, Cref, alpha, D_ab, beta, Cin):
    """Both error figures of a result: (literal, generalised).

    literal     max |C - Cref| / (|A||B|)_ij, the metric as the acceptance
                criterion states it;
    generalised max |C - Cref| / (|alpha| (|A||B|)_ij + |beta| |C_in|_ij)
                (gate_denominator), which also accounts for the rounding of the
                final addition alpha*S + beta*C."""
    return (normalized_error(C, Cref, D_ab),
            normalized_error(C, Cref, gate_denominator(alpha, D_ab, beta, Cin)))


GATE = 1e-12  # normalised error bound every result must meet (denominator: gate_denominator)
