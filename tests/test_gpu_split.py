"""GPU parity of the split-BF16 tile product (Ozaki-style slices on BF16
matrix cores) against the split reference (bit-exact: the slice products are
exact and the final FP64 combination follows the same order) and against the
FP64 reference (normalised error gate for s >= 6)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import split_ref
from synth import workloads as W
import paper_1808_05056_amd as ooc
from gpu_helpers import PinnedProblem, gate_errors

pytestmark = pytest.mark.gpu
MiB = 1 << 20


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _device_split(A, B, C0, alpha, beta, s):
    m, k = A.shape
    n = B.shape[1]
    dA = ooc.DeviceBuffer(max(8, A.nbytes)); dB = ooc.DeviceBuffer(max(8, B.nbytes)); dC = ooc.DeviceBuffer(C0.nbytes)
    if k:
        dA.upload(A); dB.upload(B)
    dC.upload(C0)
    ooc.ooc_split_gemm_device(m, n, k, s, alpha, dA.ptr, max(k, 1), dB.ptr, n, beta, dC.ptr, n)
    return dC.download((m, n))


CASES = [
    # m, n, k, s, alpha, beta, dist, row/col exponent spread
    (64, 64, 64, 1, 1.0, 0.0, synth.INT, 0),
    (100, 70, 130, 3, 1.5, 0.5, synth.NORMAL, 0),
    (256, 192, 1000, 6, 1.0, 0.0, synth.NORMAL, 20),
    (129, 257, 77, 8, -0.75, 2.0, synth.UNIFORM, 5),
    (512, 512, 4096, 6, 1.0, 0.0, synth.NORMAL, 20),
    (33, 17, 5, 7, 1.0, 1.0, synth.UNIFORM, 0),
    (200, 150, 9000, 6, 1.0, 0.5, synth.NORMAL, 10),   # more than one 8192-k panel
    (300, 260, 2048, 2, 1.0, 0.0, synth.UNIFORM, 0),   # long exactness windows (t <= 3)
    (131, 67, 257, 5, 0.75, -1.25, synth.NORMAL, 8),   # beta*C inexact: the final sums must not be fused
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_split_kernel_bit_exact_vs_split_reference(case):
    m, n, k, s, alpha, beta, dist, spread = CASES[case]
    _say(f"split kernel case {CASES[case]}")
    A = np.ascontiguousarray(synth.matrix(m, k, synth.spec(200 + case, 0, dist, row_exp=(-spread, spread))))
    B = np.ascontiguousarray(synth.matrix(k, n, synth.spec(200 + case, 1, dist, col_exp=(-spread, spread))))
    C0 = np.ascontiguousarray(synth.matrix(m, n, synth.spec(200 + case, 2, synth.UNIFORM)))
    got = _device_split(A, B, C0, alpha, beta, s)
    want = split_ref.split_gemm(alpha, A, B, beta, C0, s, kb=8192 if k > 8192 else None)
    assert np.array_equal(got, want), np.max(np.abs(got - want))
    if s >= 6:
        ref, D = oracle.gemm_rows(alpha, A, B, beta, C0)
        gate_errors(got, ref, alpha, D, beta, C0)


def test_split_chunk_sums_exact_at_largest_slices():
    # every first slice at its largest magnitude (256) and long K: the FP32 chunk
    # sums reach their bound; the result must still equal the reference exactly
    m, n, k, s = 64, 64, 4096, 2
    A = np.full((m, k), 1.0 - 2.0 ** -9)   # rounds to first slice 256 with exponent 0
    B = np.full((k, n), -(1.0 - 2.0 ** -9))
    A[::2, ::3] *= -1
    got = _device_split(A, B, np.zeros((m, n)), 1.0, 0.0, s)
    want = split_ref.split_gemm(1.0, A, B, 0.0, None, s)
    assert np.array_equal(got, want)
    exact = A @ B  # products of equal magnitudes: exact in FP64 here
    # two slices drop only the (2,2) pair: 4096 * 128^2 * 2^-32 in magnitude at most
    assert np.max(np.abs(got - exact)) <= 4096 * 128 ** 2 * 2.0 ** -32


def test_split_nonfinite_rows_and_columns_give_nan():
    m, n, k = 70, 50, 40
    A = np.ascontiguousarray(synth.matrix(m, k, synth.spec(5, 0)))
    B = np.ascontiguousarray(synth.matrix(k, n, synth.spec(5, 1)))
    A[3, 7] = np.nan
    B[11, 9] = np.inf
    got = _device_split(A, B, np.zeros((m, n)), 1.0, 0.0, 6)
    assert np.all(np.isnan(got[3])) and np.all(np.isnan(got[:, 9]))
    mask = np.ones((m, n), bool); mask[3] = False; mask[:, 9] = False
    ref, D = oracle.gemm_rows(1.0, A, B, 0.0, None)
    gate_errors(got[mask], ref[mask], 1.0, D[mask], 0.0, None)


@pytest.mark.parametrize("planner", ["paper", "ksplit"])
def test_split_pipeline_bit_exact(planner):
    w = W.Workload("split-small", 1000, 900, 1100, 1.5, 0.5, 8 * MiB, seed=21, dist_a=synth.NORMAL,
                   dist_b=synth.NORMAL, a_row_exp=(-20, 20), b_col_exp=(-20, 20))
    pp = PinnedProblem(w)
    try:
        C0 = pp.C.copy()
        if planner == "paper":
            st, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget,
                                     ooc.make_opts(planner=ooc.PLAN_PAPER, precision=ooc.SPLIT_BF16, slices=6))
            kb = None
        else:
            plan = ooc.make_plan(256, 320, 320, ooc.ORDER_COLS, 2, 2, 2, 3, precision=ooc.SPLIT_BF16, slices=6)
            st, stats = ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, plan)
            kb = 320
        assert stats.arena_bytes <= w.budget and stats.plan.precision == ooc.SPLIT_BF16
        want = split_ref.split_gemm(w.alpha, pp.A, pp.B, w.beta, C0, 6, kb=kb)
        assert np.array_equal(pp.C, want)
        ref, D = oracle.gemm_rows(w.alpha, pp.A, pp.B, w.beta, C0)
        gate_errors(pp.C, ref, w.alpha, D, w.beta, C0)
    finally:
        pp.free()


def test_split_pipeline_model_planner_staged():
    w = W.Workload("split-model", 1500, 1300, 1700, 1.0, 1.0, 8 * MiB, seed=22)
    pp = PinnedProblem(w)
    try:
        C0 = pp.C.copy()
        st, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget,
                                 ooc.make_opts(planner=ooc.PLAN_MODEL, precision=ooc.SPLIT_BF16, slices=7))
        assert stats.arena_bytes <= w.budget
        ref, D = oracle.gemm_rows(w.alpha, pp.A, pp.B, w.beta, C0)
        gate_errors(pp.C, ref, w.alpha, D, w.beta, C0)
    finally:
        pp.free()


@pytest.mark.parametrize("case", ["ld-padded", "alpha-zero", "k-zero", "beta-zero-nan-c"])
def test_split_pipeline_edge_cases(case):
    """The split path through the pipeline: host leading dimensions wider than
    the rows, alpha = 0 and K = 0 (C = beta*C, A and B unread), and beta = 0
    with C full of NaN (C unread)."""
    alpha = 0.0 if case == "alpha-zero" else 1.25
    beta = 0.0 if case == "beta-zero-nan-c" else 0.5
    w = W.Workload("split-edge", 600, 500, 700, alpha, beta, 6 * MiB, seed=23, dist_a=synth.NORMAL,
                   dist_b=synth.NORMAL, a_row_exp=(-10, 10), b_col_exp=(-10, 10))
    pp = PinnedProblem(w, ld_pad=(5, 3, 7) if case == "ld-padded" else (0, 0, 0),
                       nan_c=case == "beta-zero-nan-c")
    try:
        C0 = pp.C.copy()
        if case == "alpha-zero":
            synth.fill_nan(pp.A)  # A is not read
        A, B = (pp.A[:, :0], pp.B[:0, :]) if case == "k-zero" else (pp.A, pp.B)
        plan = ooc.make_plan(256, 192, 320, ooc.ORDER_ROWS, 2, 2, 2, 3, precision=ooc.SPLIT_BF16, slices=6)
        _, stats = ooc.ooc_gemm_planned(w.alpha, A, B, w.beta, pp.C, w.budget, plan)
        assert stats.arena_bytes <= w.budget
        _say(f"split edge case {case}: plan {stats.plan}")
        if case in ("alpha-zero", "k-zero"):
            assert np.array_equal(pp.C, beta * C0)
            return
        Cin = None if beta == 0.0 else C0
        want = split_ref.split_gemm(alpha, np.array(pp.A), np.array(pp.B), beta,
                                    np.zeros_like(C0) if Cin is None else Cin, 6, kb=320)
        assert np.array_equal(pp.C, want)
        ref, D = oracle.gemm_rows(alpha, np.array(pp.A), np.array(pp.B), beta, Cin)
        gate_errors(pp.C, ref, alpha, D, beta, Cin)
    finally:
        pp.free()


@pytest.mark.parametrize("prec,slices,order", [(ooc.SPLIT_BF16, 6, ooc.ORDER_ROWS), (ooc.SPLIT_BF16, 6, ooc.ORDER_COLS),
                                               (ooc.SPLIT_BF16, 6, ooc.ORDER_ROWS_P),
                                               (ooc.SPLIT_INT8, 7, ooc.ORDER_ROWS_P)])
def test_split_pipeline_reuses_slices_bit_exact(prec, slices, order):
    """Consecutive products on one A panel (ROWS, ROWS_P in groups) or one B
    panel (COLS) take its slices from the workspace instead of slicing it
    again; the result is the split reference's bit for bit."""
    w = W.Workload("split-reuse", 1000, 900, 1100, 1.5, 0.5, 0, seed=24, dist_a=synth.NORMAL,
                   dist_b=synth.NORMAL, a_row_exp=(-20, 20), b_col_exp=(-20, 20))
    if order == ooc.ORDER_ROWS_P:
        plan = ooc.make_plan(256, 320, 320, order, 2, 4, 3, 3, precision=prec, slices=slices, group=2)
    elif order == ooc.ORDER_ROWS:
        plan = ooc.make_plan(256, 320, 1100, order, 1, 2, 2, 3, precision=prec, slices=slices)
    else:
        plan = ooc.make_plan(256, 320, 1100, order, 2, 1, 2, 3, precision=prec, slices=slices)
    ops, _ = ooc.ooc_schedule(w.M, w.N, w.K, w.alpha, w.beta, plan)
    reused = sum(op["reuse_a"] or op["reuse_b"] for op in ops if op["kind"] == "split_gemm")
    assert reused >= 4
    budget = ooc.ooc_plan_footprint(w.M, w.N, w.K, w.beta, plan)
    pp = PinnedProblem(w)
    try:
        C0 = pp.C.copy()
        _, stats = ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, budget, plan)
        _say(f"split reuse {prec} order {order}: {reused} products reuse slices, t {stats.t_total_s * 1e3:.1f} ms")
        fmt = "i8" if prec == ooc.SPLIT_INT8 else "bf16"
        want = split_ref.split_gemm(w.alpha, pp.A, pp.B, w.beta, C0, slices, kb=plan.kb, fmt=fmt)
        assert np.array_equal(pp.C, want)
        ref, D = oracle.gemm_rows(w.alpha, pp.A, pp.B, w.beta, C0)
        gate_errors(pp.C, ref, w.alpha, D, w.beta, C0)
    finally:
        pp.free()
