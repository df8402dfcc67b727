"""GPU parity of the split-INT8 tile product (7-bit slices truncated toward
zero, INT8 matrix cores with exact INT32 sums) against the split reference in
its INT8 format (bit-exact: the integer slice sums are exact and the FP64
combination follows the same order) and against the FP64 reference
(normalised error gate for s >= 7 on normal data, s >= 6 on uniform data)."""
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


def _device_split_i8(A, B, C0, alpha, beta, s):
    m, k = A.shape
    n = B.shape[1]
    dA = ooc.DeviceBuffer(max(8, A.nbytes)); dB = ooc.DeviceBuffer(max(8, B.nbytes)); dC = ooc.DeviceBuffer(C0.nbytes)
    if k:
        dA.upload(A); dB.upload(B)
    dC.upload(C0)
    ooc.ooc_split_int8_gemm_device(m, n, k, s, alpha, dA.ptr, max(k, 1), dB.ptr, n, beta, dC.ptr, n)
    return dC.download((m, n))


CASES = [
    # m, n, k, s, alpha, beta, dist, row/col exponent spread
    (64, 64, 64, 2, 1.0, 0.0, synth.INT, 0),
    (100, 70, 130, 3, 1.5, 0.5, synth.NORMAL, 0),
    (256, 192, 1000, 7, 1.0, 0.0, synth.NORMAL, 20),
    (129, 257, 77, 8, -0.75, 2.0, synth.UNIFORM, 5),
    (512, 512, 4096, 6, 1.0, 0.0, synth.UNIFORM, 20),
    (33, 17, 5, 1, 1.0, 1.0, synth.UNIFORM, 0),
    (200, 150, 9000, 7, 1.0, 0.5, synth.NORMAL, 10),   # more than one 8192-k panel
    (300, 260, 2048, 5, 1.0, 0.0, synth.UNIFORM, 0),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_int8_kernel_bit_exact_vs_split_reference(case):
    m, n, k, s, alpha, beta, dist, spread = CASES[case]
    _say(f"split-int8 kernel case {CASES[case]}")
    A = np.ascontiguousarray(synth.matrix(m, k, synth.spec(300 + case, 0, dist, row_exp=(-spread, spread))))
    B = np.ascontiguousarray(synth.matrix(k, n, synth.spec(300 + case, 1, dist, col_exp=(-spread, spread))))
    C0 = np.ascontiguousarray(synth.matrix(m, n, synth.spec(300 + case, 2, synth.UNIFORM)))
    got = _device_split_i8(A, B, C0, alpha, beta, s)
    want = split_ref.split_gemm(alpha, A, B, beta, C0, s, kb=8192 if k > 8192 else None, fmt="i8")
    assert np.array_equal(got, want), np.max(np.abs(got - want))
    if s >= (6 if dist == synth.UNIFORM else 7):
        ref, D = oracle.gemm_rows(alpha, A, B, beta, C0)
        gate_errors(got, ref, alpha, D, beta, C0)


@pytest.mark.parametrize("shape", [(3900, 4000, 700, 6), (4096, 4096, 9000, 7)])
def test_int8_wide_tiles_bit_exact_on_sampled_rows(shape):
    # 3900 x 4000 and 4096^2 make 512 tiles of 256 x 128 (two waves on the
    # 256 CUs of an MI355X) against 256 of 256 x 256 (one wave), so the
    # kernel takes the wide tiles; ragged edges in M and N, and a second K
    # panel in the second shape.  The split reference's row exponents are per
    # row, so its result on the sampled rows is those rows of the whole one.
    m, n, k, s = shape
    _say(f"split-int8 wide tiles {shape}")
    A = np.ascontiguousarray(synth.matrix(m, k, synth.spec(330, 0, synth.NORMAL, row_exp=(-10, 10))))
    B = np.ascontiguousarray(synth.matrix(k, n, synth.spec(330, 1, synth.NORMAL, col_exp=(-10, 10))))
    C0 = np.ascontiguousarray(synth.matrix(m, n, synth.spec(330, 2, synth.UNIFORM)))
    got = _device_split_i8(A, B, C0, 1.25, 0.5, s)
    rows = np.unique(np.concatenate([[0, 255, 256, m - 1], np.random.default_rng(7).integers(0, m, 60)]))
    want = split_ref.split_gemm(1.25, A[rows], B, 0.5, C0[rows], s, kb=8192 if k > 8192 else None, fmt="i8")
    assert np.array_equal(got[rows], want), np.max(np.abs(got[rows] - want))


def test_int8_largest_digits_and_weight_sums():
    # x = 1 - 2^-53: the first seven digits are 127 (the INT8 maximum) and the
    # eighth 120; with s = 8 and 8192 k every weight's INT32 sum over all its
    # pairs is at its largest (below 2^30) and must stay exact
    m, n, k, s = 128, 128, 8192, 8
    x = 1.0 - 2.0 ** -53
    A = np.full((m, k), x)
    B = np.full((k, n), -x)
    A[::2, ::3] *= -1
    _say("split-int8 largest digits")
    got = _device_split_i8(A, B, np.zeros((m, n)), 1.0, 0.0, s)
    want = split_ref.split_gemm(1.0, A, B, 0.0, None, s, fmt="i8")
    assert np.array_equal(got, want)


def test_int8_nonfinite_rows_and_columns_give_nan():
    m, n, k = 70, 50, 40
    A = np.ascontiguousarray(synth.matrix(m, k, synth.spec(6, 0)))
    B = np.ascontiguousarray(synth.matrix(k, n, synth.spec(6, 1)))
    A[3, 7] = np.nan
    B[11, 9] = np.inf
    got = _device_split_i8(A, B, np.zeros((m, n)), 1.0, 0.0, 7)
    assert np.all(np.isnan(got[3])) and np.all(np.isnan(got[:, 9]))
    mask = np.ones((m, n), bool); mask[3] = False; mask[:, 9] = False
    ref, D = oracle.gemm_rows(1.0, A, B, 0.0, None)
    gate_errors(got[mask], ref[mask], 1.0, D[mask], 0.0, None)


def test_int8_k_zero_and_alpha_zero():
    m, n = 40, 30
    C0 = np.ascontiguousarray(synth.matrix(m, n, synth.spec(7, 2, synth.UNIFORM)))
    got = _device_split_i8(np.zeros((m, 0)), np.zeros((0, n)), C0, 1.0, 0.5, 6)
    assert np.array_equal(got, 0.5 * C0)
    A = np.ascontiguousarray(synth.matrix(m, 20, synth.spec(7, 0)))
    B = np.ascontiguousarray(synth.matrix(20, n, synth.spec(7, 1)))
    got = _device_split_i8(A, B, C0, 0.0, 2.0, 6)
    assert np.array_equal(got, split_ref.split_gemm(0.0, A, B, 2.0, C0, 6, fmt="i8"))


@pytest.mark.parametrize("planner", ["paper", "ksplit"])
def test_int8_pipeline_bit_exact(planner):
    w = W.Workload("split-int8-small", 1000, 900, 1100, 1.5, 0.5, 8 * MiB, seed=23, dist_a=synth.NORMAL,
                   dist_b=synth.NORMAL, a_row_exp=(-20, 20), b_col_exp=(-20, 20))
    pp = PinnedProblem(w)
    try:
        C0 = pp.C.copy()
        _say(f"split-int8 pipeline {planner}")
        if planner == "paper":
            st, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget,
                                     ooc.make_opts(planner=ooc.PLAN_PAPER, precision=ooc.SPLIT_INT8, slices=7))
            kb = None
        else:
            plan = ooc.make_plan(256, 320, 384, ooc.ORDER_COLS, 2, 2, 2, 3, precision=ooc.SPLIT_INT8, slices=7)
            st, stats = ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, plan)
            kb = 384
        assert stats.arena_bytes <= w.budget and stats.plan.precision == ooc.SPLIT_INT8
        want = split_ref.split_gemm(w.alpha, pp.A, pp.B, w.beta, C0, 7, kb=kb, fmt="i8")
        assert np.array_equal(pp.C, want)
        ref, D = oracle.gemm_rows(w.alpha, pp.A, pp.B, w.beta, C0)
        gate_errors(pp.C, ref, w.alpha, D, w.beta, C0)
    finally:
        pp.free()


def test_int8_pipeline_model_planner():
    w = W.Workload("split-int8-model", 1500, 1300, 1700, 1.0, 1.0, 8 * MiB, seed=24)
    pp = PinnedProblem(w)
    try:
        C0 = pp.C.copy()
        _say("split-int8 pipeline model planner")
        st, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget,
                                 ooc.make_opts(planner=ooc.PLAN_MODEL, precision=ooc.SPLIT_INT8, slices=7))
        assert stats.arena_bytes <= w.budget and stats.plan.precision == ooc.SPLIT_INT8
        ref, D = oracle.gemm_rows(w.alpha, pp.A, pp.B, w.beta, C0)
        gate_errors(pp.C, ref, w.alpha, D, w.beta, C0)
    finally:
        pp.free()


@pytest.mark.parametrize("s", range(1, 9))
def test_int8_every_slice_count_ragged(s):
    # every slice count on a shape ragged in m, n and k (one partial tile and chunk each)
    m, n, k = 131, 67, 257
    A = np.ascontiguousarray(synth.matrix(m, k, synth.spec(400 + s, 0, synth.NORMAL, row_exp=(-8, 8))))
    B = np.ascontiguousarray(synth.matrix(k, n, synth.spec(400 + s, 1, synth.NORMAL, col_exp=(-8, 8))))
    C0 = np.ascontiguousarray(synth.matrix(m, n, synth.spec(400 + s, 2, synth.UNIFORM)))
    _say(f"split-int8 s={s} ragged")
    got = _device_split_i8(A, B, C0, 0.75, -1.25, s)
    assert np.array_equal(got, split_ref.split_gemm(0.75, A, B, -1.25, C0, s, fmt="i8"))


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 300, 2), (300, 1, 3), (2, 2, 8192), (129, 1, 8193)])
def test_int8_tiny_and_long_shapes(shape):
    m, n, k = shape
    A = np.ascontiguousarray(synth.matrix(m, k, synth.spec(500 + k, 0, synth.UNIFORM)))
    B = np.ascontiguousarray(synth.matrix(k, n, synth.spec(500 + k, 1, synth.UNIFORM)))
    C0 = np.zeros((m, n))
    _say(f"split-int8 shape {shape}")
    got = _device_split_i8(A, B, C0, 1.0, 0.0, 7)
    want = split_ref.split_gemm(1.0, A, B, 0.0, None, 7, kb=8192 if k > 8192 else None, fmt="i8")
    assert np.array_equal(got, want)
