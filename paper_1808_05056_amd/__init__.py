"""Python binding of libooc.so, the MI355X out-of-core FP64 matrix product.

Argument marshalling only: every step of the product (planning, scheduling,
copies, tile kernels) runs in the native library.  Importing this package
loads the built library and raises if it is missing; build it with
``python paper_1808_05056_amd/build.py``.

Names follow the C ABI in include/ooc.h:
    ooc_gemm, ooc_gemm_planned, ooc_plan, ooc_plan_footprint, ooc_partition,
    ooc_plan_candidates, ooc_plan_predict, ooc_schedule, ooc_host_alloc,
    ooc_host_free, ooc_release, ooc_dgemm_device, ooc_last_error
plus numpy helpers for page-locked host matrices and device buffers.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libooc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_1808_05056_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

# ---- ABI types (mirror include/ooc.h) ------------------------------------------------

OOC_OK, OOC_ERR_ARG, OOC_ERR_BUDGET, OOC_ERR_DEVICE_MEM, OOC_ERR_NOT_PINNED, OOC_ERR_HIP, \
    OOC_ERR_NO_DEVICE, OOC_ERR_INJECTED, OOC_ERR_CAPACITY, OOC_ERR_NOT_SPD = range(10)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_BUDGET", 3: "ERR_DEVICE_MEM", 4: "ERR_NOT_PINNED", 5: "ERR_HIP",
                6: "ERR_NO_DEVICE", 7: "ERR_INJECTED", 8: "ERR_CAPACITY", 9: "ERR_NOT_SPD"}
FP64, SPLIT_BF16, SPLIT_INT8 = 0, 1, 2
PLAN_AUTO, PLAN_PAPER, PLAN_MODEL, PLAN_MLP, PLAN_SWEEP = 0, 1, 2, 3, 4
ORDER_COLS, ORDER_ROWS, ORDER_COLS_P, ORDER_ROWS_P, ORDER_COLS_PS, ORDER_ROWS_PS = 0, 1, 2, 3, 4, 5
OP_H2D, OP_D2H, OP_GEMM, OP_SPLIT_GEMM, OP_POTRF, OP_TRSM = range(6)
OP_NAMES = {0: "h2d", 1: "d2h", 2: "gemm", 3: "split_gemm", 4: "potrf", 5: "trsm"}
OP_KINDS = {v: k for k, v in OP_NAMES.items()}
MAX_WAITS = 6
OPF_TRANSB, OPF_LOWER, OPF_BACK, OPF_REUSE_A, OPF_REUSE_B = 1, 2, 4, 8, 16

i32, i64, u64, dbl, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class ooc_plan_t(ctypes.Structure):
    _fields_ = [("mb", i64), ("nb", i64), ("kb", i64), ("order", i32), ("nbuf_a", i32), ("nbuf_b", i32),
                ("nbuf_c", i32), ("nstreams", i32), ("precision", i32), ("slices", i32), ("nbuf_d", i32),
                ("group", i32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    def __repr__(self):
        return "ooc_plan_t(" + ", ".join(f"{k}={v}" for k, v in self.as_dict().items()) + ")"


P_dbl = ctypes.POINTER(ctypes.c_double)


class ooc_opts(ctypes.Structure):
    _fields_ = [("device", i32), ("planner", i32), ("precision", i32), ("slices", i32), ("nstreams", i32),
                ("profile", i32), ("arena", vp), ("arena_bytes", sz), ("timeline", P_dbl), ("timeline_cap", i64),
                ("streams", vp * 3), ("release_arena", i32)]


class ooc_host_matrix(ctypes.Structure):
    _fields_ = [("ptr", vp), ("rows", i64), ("cols", i64), ("ld", i64)]


class ooc_stats(ctypes.Structure):
    _fields_ = [("plan", ooc_plan_t), ("t_total_s", dbl), ("t_pipeline_s", dbl), ("t_h2d_busy_s", dbl),
                ("t_d2h_busy_s", dbl), ("t_kernel_busy_s", dbl), ("t_predicted_s", dbl), ("flops", dbl),
                ("bytes_h2d", u64), ("bytes_d2h", u64), ("arena_bytes", u64), ("ops", i64), ("tasks", i64),
                ("kernels", i64), ("blocks_done", i64), ("t_plan_s", dbl), ("overlap", dbl),
                ("t_mma_busy_s", dbl), ("mma_launches", i64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "plan"}
        d["plan"] = self.plan.as_dict()
        return d


class ooc_op(ctypes.Structure):
    _fields_ = [("kind", i32), ("stream", i32), ("task", i32), ("nwait", i32), ("wait", i32 * MAX_WAITS),
                ("mat", i32), ("slot", i32), ("flags", i32), ("reserved", i32), ("row0", i64), ("col0", i64),
                ("rows", i64), ("cols", i64),
                ("k0", i64), ("k", i64), ("off_a", i64), ("ld_a", i64), ("off_b", i64), ("ld_b", i64),
                ("off_c", i64), ("ld_c", i64), ("off_d", i64), ("ld_d", i64), ("off_w", i64), ("len_w", i64),
                ("alpha", dbl), ("beta", dbl), ("gamma", dbl)]


P = ctypes.POINTER


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("ooc_gemm", i32, [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, sz, P(ooc_opts), P(ooc_stats)])
_sig("ooc_gemm_planned", i32, [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, sz, P(ooc_plan_t), P(ooc_opts),
                               P(ooc_stats)])
_sig("ooc_plan", i32, [i64, i64, i64, dbl, sz, P(ooc_opts), P(ooc_plan_t)])
_sig("ooc_plan_footprint", i32, [i64, i64, i64, dbl, P(ooc_plan_t), P(u64)])
_sig("ooc_partition", i32, [i64, i64, i64, sz, P(i64), P(i64)])
_sig("ooc_plan_candidates", i32, [i64, i64, i64, dbl, sz, P(ooc_opts), P(ooc_plan_t), P(dbl), i64, P(i64)])
_sig("ooc_plan_predict", i32, [i64, i64, i64, dbl, P(ooc_plan_t), P(dbl)])
_sig("ooc_plan_simulate", i32, [i64, i64, i64, dbl, P(ooc_plan_t), P(dbl), i64, P(i64)])
_sig("ooc_schedule", i32, [i64, i64, i64, dbl, dbl, P(ooc_plan_t), P(ooc_op), i64, P(i64), P(u64)])
_sig("ooc_schedule_ex", i32, [i32, i32, i64, i64, i64, dbl, dbl, P(ooc_plan_t), P(ooc_op), i64, P(i64), P(u64)])
_sig("ooc_syrk", i32, [i64, i64, dbl, vp, i64, dbl, vp, i64, sz, P(ooc_opts), P(ooc_stats)])
_sig("ooc_potrf", i32, [i64, vp, i64, sz, P(ooc_opts), P(i64), P(ooc_stats)])
_sig("ooc_trsm", i32, [i64, i64, vp, i64, vp, i64, sz, P(ooc_opts), P(ooc_stats)])
_sig("ooc_trsm_ex", i32, [i32, i64, i64, vp, i64, vp, i64, sz, P(ooc_opts), P(ooc_stats)])
_sig("ooc_potrs", i32, [i64, i64, vp, i64, vp, i64, sz, P(ooc_opts), P(ooc_stats)])
_sig("ooc_run_ops", i32, [P(ooc_op), i64, P(ooc_host_matrix), i32, u64, P(ooc_opts), P(ooc_stats)])
_sig("ooc_check_ops", i32, [P(ooc_op), i64, P(i64), P(i64)])
_sig("ooc_gemm_ex", i32, [i32, i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, sz, P(ooc_opts),
                          P(ooc_stats)])
_sig("ooc_accum_begin", i32, [i64, i64, dbl, vp, i64, sz, P(ooc_opts), P(vp)])
_sig("ooc_accum_step", i32, [vp, i64, dbl, vp, i64, vp, i64, P(ooc_stats)])
_sig("ooc_accum_end", i32, [vp, P(ooc_stats)])
_sig("ooc_accum_resident_rows", i32, [i64, i64, sz, P(i64)])
_sig("ooc_accum_schedule", i32, [i64, i64, i64, dbl, dbl, sz, P(ooc_opts), i32, P(ooc_op), i64, P(i64), P(u64)])
_sig("ooc_host_alloc", i32, [P(vp), sz])
_sig("ooc_host_free", i32, [vp])
_sig("ooc_device_alloc", i32, [i32, P(vp), sz])
_sig("ooc_device_free", i32, [i32, vp])
_sig("ooc_copy_to_device", i32, [i32, vp, vp, sz])
_sig("ooc_copy_to_host", i32, [i32, vp, vp, sz])
_sig("ooc_release", i32, [i32])
_sig("ooc_device_copy", i32, [i32, vp, vp, sz])
_sig("ooc_dgemm_device", i32, [i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, i32, P(dbl)])
_sig("ooc_split_gemm_device", i32, [i32, i64, i64, i64, i32, dbl, vp, i64, vp, i64, dbl, vp, i64, i32, P(dbl)])
_sig("ooc_split_int8_gemm_device", i32, [i32, i64, i64, i64, i32, dbl, vp, i64, vp, i64, dbl, vp, i64, i32, P(dbl)])
_sig("ooc_split_gemm_device_noalloc", i32, [i32, i64, i64, i64, i32, dbl, vp, i64, vp, i64, dbl, vp, i64, vp])
P_flt = ctypes.POINTER(ctypes.c_float)
_sig("ooc_mlp_features", i32, [i64, i64, i64, dbl, sz, P(ooc_plan_t), i64, P_flt])
_sig("ooc_mlp_forward", i32, [i32, i32, i32, P_flt, P_flt, i64, P_flt])
_sig("ooc_mlp_grad", i32, [i32, i32, i32, P_flt, P_flt, P_flt, i64, ctypes.c_float, P_flt, P_flt])
_sig("ooc_mlp_adam", i32, [i32, i64, P_flt, P_flt, P_flt, P_flt, i32, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, ctypes.c_float])
_sig("ooc_mlp_train", i32, [i32, i32, i32, P_flt, P_flt, P_flt, i64, i32, ctypes.c_float, ctypes.c_float, P_flt])
_sig("ooc_mlp_fit", i32, [i32, P_flt, P_flt, i64, i32, i32, ctypes.c_float, ctypes.c_float, u64, P_flt])
_sig("ooc_mlp_save", i32, [ctypes.c_char_p])
_sig("ooc_mlp_load", i32, [ctypes.c_char_p])
_sig("ooc_mlp_loaded", i32, [])
_sig("ooc_split_int8_wide_tiles", i32, [i64, i64, i32])
_sig("ooc_mlp_predict", i32, [i64, i64, i64, dbl, sz, P(ooc_plan_t), i64, P(dbl)])
_sig("ooc_last_error", ctypes.c_char_p, [])
_sig("ooc_version", ctypes.c_char_p, [])

EXPORTS = ["ooc_gemm", "ooc_gemm_ex", "ooc_schedule_ex", "ooc_syrk", "ooc_potrf", "ooc_trsm", "ooc_trsm_ex", "ooc_potrs", "ooc_run_ops", "ooc_check_ops", "ooc_gemm_planned", "ooc_plan", "ooc_plan_footprint", "ooc_partition", "ooc_plan_candidates",
           "ooc_plan_predict", "ooc_plan_simulate", "ooc_schedule", "ooc_host_alloc", "ooc_host_free", "ooc_device_alloc",
           "ooc_device_free", "ooc_copy_to_device", "ooc_copy_to_host", "ooc_release", "ooc_device_copy", "ooc_dgemm_device",
           "ooc_split_gemm_device", "ooc_split_int8_gemm_device", "ooc_split_int8_wide_tiles", "ooc_split_gemm_device_noalloc", "ooc_mlp_features", "ooc_mlp_forward",
           "ooc_mlp_grad", "ooc_mlp_adam",
           "ooc_mlp_train", "ooc_mlp_fit", "ooc_mlp_save", "ooc_mlp_load", "ooc_mlp_loaded", "ooc_mlp_predict",
           "ooc_accum_begin", "ooc_accum_step", "ooc_accum_end", "ooc_accum_resident_rows", "ooc_accum_schedule",
           "ooc_last_error", "ooc_version"]
MLP_FEATURES = 19


class OOCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def ooc_last_error():
    return _lib.ooc_last_error().decode()


def ooc_version():
    return _lib.ooc_version().decode()


def _check(st):
    if st != OOC_OK:
        raise OOCError(st, ooc_last_error())
    return st


def _mat_arg(X, name):
    """(pointer, leading dimension) of a 2-D row-major float64 view, or (None, 0)."""
    if X is None:
        return None, 0
    if not isinstance(X, np.ndarray) or X.dtype != np.float64 or X.ndim != 2 or X.strides[1] != 8 or X.strides[0] % 8:
        raise TypeError(f"{name} must be a 2-D row-major float64 numpy view")
    return X.ctypes.data, max(X.strides[0] // 8, X.shape[1])


def make_opts(device=0, planner=PLAN_AUTO, precision=FP64, slices=0, nstreams=0, profile=False, arena=None,
              arena_bytes=0, timeline=None, streams=None, release_arena=False):
    """timeline: a float64 numpy array of 2*nops entries to receive per-op start/end (profile mode).
    streams: up to three raw hipStream_t handles (ints) the pipeline borrows (None entries: the library's)."""
    o = ooc_opts(device, planner, precision, slices, nstreams, 1 if profile else 0, arena, arena_bytes, None, 0)
    if streams is not None:
        for x, h in enumerate(streams):
            o.streams[x] = h
    o.release_arena = 1 if release_arena else 0
    if timeline is not None:
        assert timeline.dtype == np.float64 and timeline.flags.c_contiguous
        o.timeline = timeline.ctypes.data_as(P_dbl)
        o.timeline_cap = timeline.size // 2
        o._keep = timeline
    return o


def make_plan(mb, nb, kb, order=ORDER_COLS, nbuf_a=2, nbuf_b=1, nbuf_c=2, nstreams=3, precision=FP64, slices=0,
              nbuf_d=0, group=0):
    return ooc_plan_t(mb, nb, kb, order, nbuf_a, nbuf_b, nbuf_c, nstreams, precision, slices, nbuf_d, group)


# ---- entry points ---------------------------------------------------------------------

def ooc_gemm(alpha, A, B, beta, C, budget_bytes, opts=None, raise_on_error=True):
    """C = alpha*A@B + beta*C in place (A, B, C page-locked float64 views).
    Returns (status, ooc_stats)."""
    M, N = C.shape
    K = A.shape[1] if A is not None else 0
    pa, lda = _mat_arg(A, "A")
    pb, ldb = _mat_arg(B, "B")
    pc, ldc = _mat_arg(C, "C")
    st = ooc_stats()
    s = _lib.ooc_gemm(M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc, budget_bytes,
                      ctypes.byref(opts) if opts is not None else None, ctypes.byref(st))
    if raise_on_error:
        _check(s)
    return s, st


def ooc_gemm_ex(alpha, A, B, beta, C, budget_bytes, transb=False, lower=False, opts=None, raise_on_error=True):
    """C = alpha*A@op(B) + beta*C in place with op(B) = B.T when transb (B is N x K);
    with lower only C's elements on and below the diagonal.  Returns (status, ooc_stats)."""
    M, N = C.shape
    K = A.shape[1] if A is not None else 0
    pa, lda = _mat_arg(A, "A")
    pb, ldb = _mat_arg(B, "B")
    pc, ldc = _mat_arg(C, "C")
    st = ooc_stats()
    s = _lib.ooc_gemm_ex(1 if transb else 0, 1 if lower else 0, M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc,
                         budget_bytes, ctypes.byref(opts) if opts is not None else None, ctypes.byref(st))
    if raise_on_error:
        _check(s)
    return s, st


def ooc_syrk(alpha, A, beta, C, budget_bytes, opts=None, raise_on_error=True):
    """C = alpha*A@A.T + beta*C on the lower triangle of C (N x N); A is N x K.  Returns (status, ooc_stats)."""
    N = C.shape[0]
    K = A.shape[1]
    pa, lda = _mat_arg(A, "A")
    pc, ldc = _mat_arg(C, "C")
    st = ooc_stats()
    s = _lib.ooc_syrk(N, K, alpha, pa, lda, beta, pc, ldc, budget_bytes,
                      ctypes.byref(opts) if opts is not None else None, ctypes.byref(st))
    if raise_on_error:
        _check(s)
    return s, st


def ooc_potrf(A, budget_bytes, opts=None, raise_on_error=True):
    """Cholesky factor of A (N x N, page-locked) in place on its lower triangle.  Returns (status, info, ooc_stats)."""
    N = A.shape[0]
    pa, lda = _mat_arg(A, "A")
    st = ooc_stats()
    info = i64()
    s = _lib.ooc_potrf(N, pa, lda, budget_bytes, ctypes.byref(opts) if opts is not None else None,
                       ctypes.byref(info), ctypes.byref(st))
    if raise_on_error:
        _check(s)
    return s, info.value, st


def ooc_trsm(L, X, budget_bytes, opts=None, raise_on_error=True):
    """X <- X L^{-T} (Y L^T = X) for lower-triangular L (N x N) and X (M x N), both page-locked;
    only L's lower triangle is read.  Returns (status, ooc_stats)."""
    N = L.shape[0]
    M = X.shape[0]
    if L.shape[1] != N or X.shape[1] != N:
        raise ValueError("L must be N x N and X M x N")
    pl, ldl = _mat_arg(L, "L")
    px, ldx = _mat_arg(X, "X")
    st = ooc_stats()
    s = _lib.ooc_trsm(M, N, pl, ldl, px, ldx, budget_bytes, ctypes.byref(opts) if opts is not None else None,
                      ctypes.byref(st))
    if raise_on_error:
        _check(s)
    return s, st


def _solve_args(L, X):
    N = L.shape[0]
    M = X.shape[0]
    if L.shape[1] != N or X.shape[1] != N:
        raise ValueError("L must be N x N and X M x N")
    pl, ldl = _mat_arg(L, "L")
    px, ldx = _mat_arg(X, "X")
    return M, N, pl, ldl, px, ldx


def ooc_trsm_ex(L, X, budget_bytes, trans=1, opts=None, raise_on_error=True):
    """trans=1: X <- X L^{-T} (as ooc_trsm); trans=0: X <- X L^{-1} (Y L = X, back substitution).
    L (N x N, lower triangle read) and X (M x N) page-locked.  Returns (status, ooc_stats)."""
    M, N, pl, ldl, px, ldx = _solve_args(L, X)
    st = ooc_stats()
    s = _lib.ooc_trsm_ex(trans, M, N, pl, ldl, px, ldx, budget_bytes,
                         ctypes.byref(opts) if opts is not None else None, ctypes.byref(st))
    if raise_on_error:
        _check(s)
    return s, st


def ooc_potrs(L, B, budget_bytes, opts=None, raise_on_error=True):
    """B <- B A^{-1} for A = L L^T (L from ooc_potrf): each row of B (M x N) is a right-hand side of A x = b.
    Both page-locked.  Returns (status, ooc_stats)."""
    M, N, pl, ldl, pb, ldb = _solve_args(L, B)
    st = ooc_stats()
    s = _lib.ooc_potrs(M, N, pl, ldl, pb, ldb, budget_bytes, ctypes.byref(opts) if opts is not None else None,
                       ctypes.byref(st))
    if raise_on_error:
        _check(s)
    return s, st


def make_op(kind, stream=0, waits=(), **fields):
    """An ooc_op: kind by name ('h2d', 'd2h', 'gemm', 'split_gemm', 'potrf', 'trsm'), other fields by name."""
    o = ooc_op()
    o.kind = OP_KINDS[kind]
    o.stream = stream
    waits = list(waits)
    if len(waits) > MAX_WAITS:
        raise ValueError("too many waits")
    o.nwait = len(waits)
    for x, w in enumerate(waits):
        o.wait[x] = w
    for k, v in fields.items():
        setattr(o, k, v)
    return o


def _op_array(ops):
    arr = (ooc_op * max(len(ops), 1))()
    for x, o in enumerate(ops):
        arr[x] = o
    return arr


def ooc_run_ops(ops, mats, arena_bytes, opts=None, raise_on_error=True):
    """Run a list of ooc_op on the device; mats: list of page-locked 2-D float64 arrays (op.mat indexes them).
    Returns (status, ooc_stats)."""
    hm = (ooc_host_matrix * max(len(mats), 1))()
    for x, M in enumerate(mats):
        p, ld = _mat_arg(M, f"mats[{x}]")
        hm[x] = ooc_host_matrix(p, M.shape[0], M.shape[1], ld)
    st = ooc_stats()
    s = _lib.ooc_run_ops(_op_array(ops), len(ops), hm, len(mats), arena_bytes,
                         ctypes.byref(opts) if opts is not None else None, ctypes.byref(st))
    if raise_on_error:
        _check(s)
    return s, st


def ooc_check_ops(ops):
    """(status, x, y): OOC_OK, or OOC_ERR_ARG with the first unordered conflicting pair x > y."""
    x, y = i64(), i64()
    s = _lib.ooc_check_ops(_op_array(ops), len(ops), ctypes.byref(x), ctypes.byref(y))
    return s, x.value, y.value


def ooc_gemm_raw(M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc, budget_bytes, opts=None):
    """The ABI call with raw pointers and sizes (for argument-check tests). Returns (status, stats)."""
    st = ooc_stats()
    s = _lib.ooc_gemm(M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc, budget_bytes,
                      ctypes.byref(opts) if opts is not None else None, ctypes.byref(st))
    return s, st


def ooc_gemm_planned(alpha, A, B, beta, C, budget_bytes, plan, opts=None, raise_on_error=True):
    M, N = C.shape
    K = A.shape[1] if A is not None else 0
    pa, lda = _mat_arg(A, "A")
    pb, ldb = _mat_arg(B, "B")
    pc, ldc = _mat_arg(C, "C")
    st = ooc_stats()
    s = _lib.ooc_gemm_planned(M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc, budget_bytes, ctypes.byref(plan),
                              ctypes.byref(opts) if opts is not None else None, ctypes.byref(st))
    if raise_on_error:
        _check(s)
    return s, st


def ooc_plan(M, N, K, beta, budget_bytes, opts=None):
    p = ooc_plan_t()
    _check(_lib.ooc_plan(M, N, K, beta, budget_bytes, ctypes.byref(opts) if opts is not None else None,
                         ctypes.byref(p)))
    return p


def ooc_plan_footprint(M, N, K, beta, plan):
    b = u64()
    _check(_lib.ooc_plan_footprint(M, N, K, beta, ctypes.byref(plan), ctypes.byref(b)))
    return b.value


def ooc_partition(M, N, K, budget_bytes):
    h, w = i64(), i64()
    st = _lib.ooc_partition(M, N, K, budget_bytes, ctypes.byref(h), ctypes.byref(w))
    if st == OOC_ERR_BUDGET:
        return None
    _check(st)
    return h.value, w.value


def ooc_plan_candidates(M, N, K, beta, budget_bytes, opts=None, cap=4096):
    plans = (ooc_plan_t * cap)()
    times = (dbl * cap)()
    n = i64()
    _check(_lib.ooc_plan_candidates(M, N, K, beta, budget_bytes, ctypes.byref(opts) if opts is not None else None,
                                    plans, times, cap, ctypes.byref(n)))
    return [plans[x] for x in range(n.value)], [times[x] for x in range(n.value)]


def ooc_plan_predict(M, N, K, beta, plan):
    t = dbl()
    _check(_lib.ooc_plan_predict(M, N, K, beta, ctypes.byref(plan), ctypes.byref(t)))
    return t.value


def ooc_plan_simulate(M, N, K, beta, plan):
    """The cost model's per-op (start, end) times, shape (nops, 2)."""
    n = i64()
    st = _lib.ooc_plan_simulate(M, N, K, beta, ctypes.byref(plan), None, 0, ctypes.byref(n))
    if st not in (OOC_OK, OOC_ERR_CAPACITY):
        _check(st)
    t = np.zeros(2 * max(n.value, 1))
    _check(_lib.ooc_plan_simulate(M, N, K, beta, ctypes.byref(plan), t.ctypes.data_as(P_dbl), n.value,
                                  ctypes.byref(n)))
    return t[: 2 * n.value].reshape(-1, 2)


def ooc_schedule(M, N, K, alpha, beta, plan, transb=False, lower=False):
    """The operation list as dicts (keys as in the CPU schedule checker) and the arena size in elements."""
    n = i64()
    ab = u64()
    tb, lo = 1 if transb else 0, 1 if lower else 0
    st = _lib.ooc_schedule_ex(tb, lo, M, N, K, alpha, beta, ctypes.byref(plan), None, 0, ctypes.byref(n),
                              ctypes.byref(ab))
    if st not in (OOC_OK, OOC_ERR_CAPACITY):
        _check(st)
    cap = max(n.value, 1)
    arr = (ooc_op * cap)()
    _check(_lib.ooc_schedule_ex(tb, lo, M, N, K, alpha, beta, ctypes.byref(plan), arr, cap, ctypes.byref(n),
                                ctypes.byref(ab)))
    return _ops_as_dicts(arr, n.value), ab.value // 8


def _ops_as_dicts(arr, count):
    ops = []
    for x in range(count):
        o = arr[x]
        kind = OP_NAMES[o.kind]
        d = dict(kind=kind, stream=o.stream, task=o.task, waits=[o.wait[k] for k in range(o.nwait)], slot=o.slot)
        if kind in ("h2d", "d2h"):
            d.update(mat="ABC"[o.mat], row0=o.row0, col0=o.col0, rows=o.rows, cols=o.cols, dev_off=o.off_c,
                     dev_ld=o.ld_c)
        else:
            if kind in ("potrf", "trsm"):
                d.update(m=o.rows, n=o.cols, k0=o.k0, off_a=o.off_a, lda=o.ld_a, off_c=o.off_c, ldc=o.ld_c,
                         off_w=o.off_w)
                if kind == "trsm":
                    d["back"] = bool(o.flags & OPF_BACK)
                ops.append(d)
                continue
            d.update(m=o.rows, n=o.cols, k=o.k, i0=o.row0, j0=o.col0, k0=o.k0, off_a=o.off_a, lda=o.ld_a,
                     off_b=o.off_b, ldb=o.ld_b, off_c=o.off_c, ldc=o.ld_c, off_d=o.off_d, ldd=o.ld_d,
                     off_w=o.off_w, len_w=o.len_w, alpha=o.alpha, beta=o.beta, gamma=o.gamma,
                     transb=bool(o.flags & OPF_TRANSB), lower=bool(o.flags & OPF_LOWER),
                     reuse_a=bool(o.flags & OPF_REUSE_A), reuse_b=bool(o.flags & OPF_REUSE_B))
        ops.append(d)
    return ops


# ---- accumulation sessions ----------------------------------------------------------

class AccumSession:
    """C = beta*C_in + sum of alpha_s * A_s @ B_s over steps (ooc_accum_begin/step/end).
    C must be a page-locked float64 view that stays alive until end()."""

    def __init__(self, beta, C, budget_bytes, opts=None):
        pc, ldc = _mat_arg(C, "C")
        self.C = C
        h = vp()
        _check(_lib.ooc_accum_begin(C.shape[0], C.shape[1], beta, pc, ldc, budget_bytes,
                                    ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)))
        self.handle = h.value

    def step(self, alpha, A, B, raise_on_error=True):
        pa, lda = _mat_arg(A, "A")
        pb, ldb = _mat_arg(B, "B")
        st = ooc_stats()
        s = _lib.ooc_accum_step(self.handle, A.shape[1], alpha, pa, lda, pb, ldb, ctypes.byref(st))
        if raise_on_error:
            _check(s)
        return s, st

    def end(self):
        st = ooc_stats()
        h, self.handle = self.handle, None
        _check(_lib.ooc_accum_end(h, ctypes.byref(st)))
        return st


def ooc_accum_resident_rows(M, N, budget_bytes):
    r = i64()
    _check(_lib.ooc_accum_resident_rows(M, N, budget_bytes, ctypes.byref(r)))
    return r.value


def ooc_accum_schedule(M, N, K, alpha, beta_eff, budget_bytes, part, opts=None):
    """One session step's operation list for part 0 (resident rows) or 1 (streamed rows),
    as dicts, and the arena size in elements."""
    n, ab = i64(), u64()
    o = ctypes.byref(opts) if opts is not None else None
    st = _lib.ooc_accum_schedule(M, N, K, alpha, beta_eff, budget_bytes, o, part, None, 0, ctypes.byref(n),
                                 ctypes.byref(ab))
    if st not in (OOC_OK, OOC_ERR_CAPACITY):
        _check(st)
    cap = max(n.value, 1)
    arr = (ooc_op * cap)()
    _check(_lib.ooc_accum_schedule(M, N, K, alpha, beta_eff, budget_bytes, o, part, arr, cap, ctypes.byref(n),
                                   ctypes.byref(ab)))
    return _ops_as_dicts(arr, n.value), ab.value // 8


def ooc_device_copy(dst, src, nbytes, device=0):
    _check(_lib.ooc_device_copy(device, dst, src, nbytes))


def ooc_release(device=-1):
    _check(_lib.ooc_release(device))


def ooc_split_gemm_device(m, n, k, s, alpha, dA, lda, dB, ldb, beta, dC, ldc, reps=1, timed=False, device=0):
    ms = dbl()
    _check(_lib.ooc_split_gemm_device(device, m, n, k, s, alpha, dA, lda, dB, ldb, beta, dC, ldc, reps,
                                      ctypes.byref(ms) if timed else None))
    return ms.value if timed else None


NOALLOC_SCRATCH_BYTES = 64 << 20  # OOC_NOALLOC_SCRATCH_BYTES


def ooc_split_gemm_device_noalloc(m, n, k, s, alpha, dA, lda, dB, ldb, beta, dC, ldc, stream=None, device=0):
    """Enqueues the product on `stream` (raw hipStream_t, None: the null stream) and returns without waiting."""
    _check(_lib.ooc_split_gemm_device_noalloc(device, m, n, k, s, alpha, dA, lda, dB, ldb, beta, dC, ldc, stream))


def ooc_split_int8_gemm_device(m, n, k, s, alpha, dA, lda, dB, ldb, beta, dC, ldc, reps=1, timed=False, device=0):
    ms = dbl()
    _check(_lib.ooc_split_int8_gemm_device(device, m, n, k, s, alpha, dA, lda, dB, ldb, beta, dC, ldc, reps,
                                           ctypes.byref(ms) if timed else None))
    return ms.value if timed else None


def ooc_split_int8_wide_tiles(m, n, cus=256):
    """1 if the INT8 slice products of an m x n block run on 256 x 256 tiles, 0 on 256 x 128, -1 for bad sizes."""
    return _lib.ooc_split_int8_wide_tiles(m, n, cus)


def ooc_dgemm_device(m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc, reps=1, timed=False, device=0):
    ms = dbl()
    _check(_lib.ooc_dgemm_device(device, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc, reps,
                                 ctypes.byref(ms) if timed else None))
    return ms.value if timed else None


# ---- memory helpers ---------------------------------------------------------------------

class PinnedMatrix:
    """A page-locked host matrix (rows x cols, row pitch ld) exposed as a numpy view."""

    def __init__(self, rows, cols, ld=None):
        self.ld = cols if ld is None else ld
        nbytes = max(1, rows * self.ld * 8)
        p = vp()
        _check(_lib.ooc_host_alloc(ctypes.byref(p), nbytes))
        self.ptr = p.value
        buf = (ctypes.c_double * max(1, rows * self.ld)).from_address(self.ptr)
        full = np.ctypeslib.as_array(buf)[: rows * self.ld].reshape(rows, self.ld) if rows * self.ld else np.empty((rows, self.ld))
        self.array = full[:, :cols]

    def free(self):
        if self.ptr:
            _lib.ooc_host_free(self.ptr)
            self.ptr = None
            self.array = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class DeviceBuffer:
    """Device memory for the tile-kernel entry points."""

    def __init__(self, nbytes, device=0):
        p = vp()
        _check(_lib.ooc_device_alloc(device, ctypes.byref(p), nbytes))
        self.ptr, self.nbytes, self.device = p.value, nbytes, device

    def upload(self, X):
        X = np.ascontiguousarray(X)
        assert X.nbytes <= self.nbytes
        _check(_lib.ooc_copy_to_device(self.device, self.ptr, X.ctypes.data, X.nbytes))

    def download(self, shape, dtype=np.float64):
        out = np.empty(shape, dtype=dtype)
        assert out.nbytes <= self.nbytes
        _check(_lib.ooc_copy_to_host(self.device, out.ctypes.data, self.ptr, out.nbytes))
        return out

    def free(self):
        if self.ptr:
            _lib.ooc_device_free(self.device, self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---- the learned planner ------------------------------------------------------------------

def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(P_flt)


def mlp_param_count(d, H):
    return d * H + H + H * H + H + H + 1


def ooc_mlp_features(M, N, K, beta, budget_bytes, plans):
    arr = (ooc_plan_t * len(plans))(*plans)
    X = np.zeros((len(plans), MLP_FEATURES), dtype=np.float32)
    _check(_lib.ooc_mlp_features(M, N, K, beta, budget_bytes, arr, len(plans), X.ctypes.data_as(P_flt)))
    return X


def ooc_mlp_forward(d, H, params, X, device=0):
    p, pp = _f32(params)
    x, px = _f32(X)
    y = np.zeros(x.shape[0], dtype=np.float32)
    _check(_lib.ooc_mlp_forward(device, d, H, pp, px, x.shape[0], y.ctypes.data_as(P_flt)))
    return y


def ooc_mlp_grad(d, H, params, X, t, weight_decay=0.0, device=0):
    p, pp = _f32(params)
    x, px = _f32(X)
    tt, pt = _f32(t)
    g = np.zeros(p.size, dtype=np.float32)
    loss = ctypes.c_float()
    _check(_lib.ooc_mlp_grad(device, d, H, pp, px, pt, x.shape[0], weight_decay, g.ctypes.data_as(P_flt),
                             ctypes.byref(loss)))
    return g, loss.value


def ooc_mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, device=0):
    """One Adam step; returns new (params, m, v) as float32 arrays."""
    p = np.array(params, dtype=np.float32)
    mm = np.array(m, dtype=np.float32)
    vv = np.array(v, dtype=np.float32)
    g, pg = _f32(grad)
    _check(_lib.ooc_mlp_adam(device, p.size, p.ctypes.data_as(P_flt), pg, mm.ctypes.data_as(P_flt),
                             vv.ctypes.data_as(P_flt), step, lr, beta1, beta2, eps))
    return p, mm, vv


def ooc_mlp_train(d, H, params, X, t, epochs, lr=1e-3, weight_decay=0.0, device=0):
    """Full-batch Adam on the GPU; returns (params, loss history)."""
    p = np.array(params, dtype=np.float32)
    x, px = _f32(X)
    tt, pt = _f32(t)
    hist = np.zeros(max(epochs, 1), dtype=np.float32)
    _check(_lib.ooc_mlp_train(device, d, H, p.ctypes.data_as(P_flt), px, pt, x.shape[0], epochs, lr, weight_decay,
                              hist.ctypes.data_as(P_flt)))
    return p, hist[:epochs]


def ooc_mlp_fit(X, seconds, hidden=64, epochs=1000, lr=3e-3, weight_decay=1e-3, seed=0, device=0):
    """Fit the planner network to measured seconds of candidate plans (features X)."""
    x, px = _f32(X)
    y, py = _f32(seconds)
    hist = np.zeros(max(epochs, 1), dtype=np.float32)
    _check(_lib.ooc_mlp_fit(device, px, py, x.shape[0], hidden, epochs, lr, weight_decay, seed,
                            hist.ctypes.data_as(P_flt)))
    return hist[:epochs]


def ooc_mlp_save(path):
    _check(_lib.ooc_mlp_save(path.encode()))


def ooc_mlp_load(path):
    _check(_lib.ooc_mlp_load(path.encode()))


def ooc_mlp_loaded():
    return bool(_lib.ooc_mlp_loaded())


def ooc_mlp_predict(M, N, K, beta, budget_bytes, plans):
    arr = (ooc_plan_t * len(plans))(*plans)
    out = np.zeros(len(plans))
    _check(_lib.ooc_mlp_predict(M, N, K, beta, budget_bytes, arr, len(plans), out.ctypes.data_as(P(dbl))))
    return out
