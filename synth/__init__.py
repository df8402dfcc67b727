"""Seeded synthetic inputs shared by the tests, the bench and the CPU reference.

Only input generation lives here (see ``gen.c`` for the counter-based
definition); none of the matrix-product arithmetic does.  Any entry of A, B or
the initial C can be regenerated from (seed, matrix id, row, column), which is
how the reference recomputes sampled rows of a product whose C was overwritten
in place.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")

UNIFORM, NORMAL, ONES, INT, ZERO = 0, 1, 2, 3, 4
MAT_A, MAT_B, MAT_C = 0, 1, 2


class SynSpec(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("mat", ctypes.c_uint32), ("dist", ctypes.c_int32),
                ("row_lo", ctypes.c_double), ("row_hi", ctypes.c_double),
                ("col_lo", ctypes.c_double), ("col_hi", ctypes.c_double)]


def build():
    """Compile gen.c into libsynth.so (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO, os.path.join(_HERE, "gen.c"), "-lm"]
    subprocess.check_call(cmd)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.syn_fill.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(SynSpec)]
        L.syn_fill.restype = None
        L.syn_fill_nan.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.syn_fill_nan.restype = None
        L.syn_entry.argtypes = [ctypes.POINTER(SynSpec), ctypes.c_int64, ctypes.c_int64]
        L.syn_entry.restype = ctypes.c_double
        _lib = L
    return _lib


def spec(seed, mat, dist=UNIFORM, row_exp=(0.0, 0.0), col_exp=(0.0, 0.0)):
    return SynSpec(seed, mat, dist, float(row_exp[0]), float(row_exp[1]),
                   float(col_exp[0]), float(col_exp[1]))


def _check_view(X):
    if X.dtype != np.float64 or X.ndim != 2 or X.strides[1] != 8 or X.strides[0] % 8:
        raise ValueError("need a 2-D float64 row-major view")


def fill(X, sp, row0=0, col0=0):
    """Fill the 2-D float64 view X with rows row0.. and columns col0.. of the matrix."""
    _check_view(X)
    nrows, ncols = X.shape
    lib().syn_fill(X.ctypes.data, X.strides[0] // 8, None, row0, nrows, col0, ncols, ctypes.byref(sp))
    return X


def fill_rows(X, rows, sp, col0=0):
    """Fill X[r, :] with matrix row rows[r] (columns col0..)."""
    _check_view(X)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    assert rows.shape[0] == X.shape[0]
    lib().syn_fill(X.ctypes.data, X.strides[0] // 8, rows.ctypes.data, 0, X.shape[0], col0, X.shape[1],
                   ctypes.byref(sp))
    return X


def fill_nan(X):
    _check_view(X)
    lib().syn_fill_nan(X.ctypes.data, X.strides[0] // 8, X.shape[0], X.shape[1])
    return X


def matrix(rows, cols, sp, ld=None):
    """A fresh (non-pinned) numpy matrix; ld > cols gives a padded row pitch."""
    ld = cols if ld is None else ld
    buf = np.empty((rows, ld), dtype=np.float64)
    X = buf[:, :cols]
    fill(X, sp)
    return X
