"""GPU parity of the HIP path against the CPU reference, through the C ABI.

Gate: max |C - C_ref| / (|A||B|)_ij <= 1e-12 (integer inputs: bit-exact)."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import workloads as W
import paper_1808_05056_amd as ooc
from gpu_helpers import PinnedProblem, sample_rows, check_rows, reference_rows, gate_errors

pytestmark = pytest.mark.gpu
MiB, GiB = 1 << 20, 1 << 30


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# ---- the tile kernel on device memory ------------------------------------------------

KERNEL_CASES = [
    # m, n, k, lda_pad, ldb_pad, ldc_pad, alpha, beta, dist
    (1, 1, 1, 0, 0, 0, 1.0, 0.0, synth.UNIFORM),
    (128, 128, 16, 0, 0, 0, 1.0, 0.0, synth.INT),
    (256, 384, 512, 0, 0, 0, 1.5, 0.5, synth.UNIFORM),
    (130, 257, 33, 0, 0, 0, -2.0, 0.25, synth.INT),      # ragged m, n, k
    (77, 45, 63, 0, 0, 0, 1.0, 1.0, synth.UNIFORM),       # odd leading dims: scalar loads
    (300, 200, 1000, 6, 2, 4, 0.75, -1.0, synth.NORMAL),  # padded leading dims
    (1024, 1024, 2048, 0, 0, 0, 1.0, 0.0, synth.NORMAL),
    (64, 64, 0, 0, 0, 0, 1.0, 0.5, synth.UNIFORM),        # k = 0: C = beta*C
    # tile counts that leave remainders in the XCD bands and the row groups
    (1100, 1500, 96, 0, 0, 0, 1.0, 0.0, synth.INT),       # 9 x 12 = 108 tiles
    (2900, 2100, 300, 2, 0, 6, 0.5, 2.0, synth.INT),      # 23 x 17 = 391 tiles, more than two per CU
]


@pytest.mark.parametrize("case", range(len(KERNEL_CASES)))
def test_dgemm_kernel_parity(case):
    m, n, k, pa, pb, pc, alpha, beta, dist = KERNEL_CASES[case]
    _say(f"kernel case {KERNEL_CASES[case]}")
    lda, ldb, ldc = k + pa, n + pb, n + pc
    A = synth.matrix(m, k, synth.spec(100 + case, 0, dist), ld=lda) if k else np.zeros((m, 0))
    B = synth.matrix(k, n, synth.spec(100 + case, 1, dist), ld=ldb) if k else np.zeros((0, n))
    C0 = synth.matrix(m, n, synth.spec(100 + case, 2, dist), ld=ldc)
    dA = ooc.DeviceBuffer(max(8, A.base.nbytes if A.base is not None else A.nbytes))
    dB = ooc.DeviceBuffer(max(8, B.base.nbytes if B.base is not None else B.nbytes))
    dC = ooc.DeviceBuffer(C0.base.nbytes)
    if k:
        dA.upload(A.base if A.base is not None else A)
        dB.upload(B.base if B.base is not None else B)
    dC.upload(C0.base)
    ooc.ooc_dgemm_device(m, n, k, alpha, dA.ptr, max(lda, 1), dB.ptr, max(ldb, 1), beta, dC.ptr, ldc)
    got = dC.download((m, ldc))[:, :n]
    ref, D = oracle.gemm_rows(alpha, A, B, beta, C0)
    if dist == synth.INT:
        assert np.array_equal(got, ref)
    gate_errors(got, ref, alpha, D, beta, C0)


def test_dgemm_kernel_beta_zero_ignores_nan():
    m, n, k = 200, 136, 40
    A = synth.matrix(m, k, synth.spec(7, 0))
    B = synth.matrix(k, n, synth.spec(7, 1))
    dA, dB, dC = ooc.DeviceBuffer(A.nbytes), ooc.DeviceBuffer(B.nbytes), ooc.DeviceBuffer(m * n * 8)
    dA.upload(A); dB.upload(B); dC.upload(np.full((m, n), np.nan))
    ooc.ooc_dgemm_device(m, n, k, 1.0, dA.ptr, k, dB.ptr, n, 0.0, dC.ptr, n)
    got = dC.download((m, n))
    ref, D = oracle.gemm_rows(1.0, A, B, 0.0, None)
    assert np.all(np.isfinite(got))
    gate_errors(got, ref, 1.0, D, 0.0, None)


# ---- the out-of-core product on the small workload, every planner and plan shape --------

SMALL_PLANS = [
    ("paper", None, ooc.PLAN_PAPER),
    ("model", None, ooc.PLAN_MODEL),
    ("cols-3s", ooc.make_plan(128, 256, 1024, ooc.ORDER_COLS, 2, 1, 2, 3), None),
    ("rows-3s", ooc.make_plan(256, 128, 1024, ooc.ORDER_ROWS, 1, 2, 2, 3), None),
    ("cols-ksplit", ooc.make_plan(384, 256, 320, ooc.ORDER_COLS, 2, 2, 2, 3), None),
    ("colsp", ooc.make_plan(256, 256, 256, ooc.ORDER_COLS_P, 2, 2, 5, 3), None),
    ("rowsp-2s", ooc.make_plan(200, 300, 192, ooc.ORDER_ROWS_P, 2, 2, 5, 2), None),
    ("one-stream", ooc.make_plan(128, 512, 1024, ooc.ORDER_COLS, 2, 1, 2, 1), None),
    ("colsp-staged", ooc.make_plan(256, 256, 256, ooc.ORDER_COLS_P, 2, 2, 4, 3, nbuf_d=1), None),
    ("rows-ksplit-staged", ooc.make_plan(384, 256, 320, ooc.ORDER_ROWS, 2, 2, 2, 3, nbuf_d=1), None),
    ("rowsp-group2", ooc.make_plan(256, 256, 256, ooc.ORDER_ROWS_P, 4, 2, 3, 3, group=2), None),
    ("colsp-group3-staged", ooc.make_plan(256, 256, 256, ooc.ORDER_COLS_P, 2, 4, 3, 3, nbuf_d=1, group=3), None),
    ("rowsps-group3", ooc.make_plan(256, 256, 256, ooc.ORDER_ROWS_PS, 4, 3, 4, 3, group=3), None),
    ("colsps-staged", ooc.make_plan(256, 256, 256, ooc.ORDER_COLS_PS, 2, 2, 4, 3, nbuf_d=1), None),
]


@pytest.mark.parametrize("beta", [0.0, 0.5])
@pytest.mark.parametrize("case", range(len(SMALL_PLANS)))
def test_small_workload_all_plans(case, beta):
    name, plan, planner = SMALL_PLANS[case]
    w = W.Workload("small", 1024, 1024, 1024, 1.5, beta, 8 * MiB, seed=1)
    _say(f"small workload plan {name} beta {beta}")
    pp = PinnedProblem(w, nan_c=(beta == 0.0))
    try:
        if plan is None:
            st, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, ooc.make_opts(planner=planner))
        else:
            st, stats = ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, plan)
        assert stats.arena_bytes <= w.budget
        check_rows(w, pp, np.arange(w.M))
        assert stats.blocks_done == -(-w.M // stats.plan.mb) * -(-w.N // stats.plan.nb)
    finally:
        pp.free()


def test_small_workload_integer_inputs_bit_exact():
    w = W.Workload("small-int", 1000, 700, 900, 2.0, -0.5, 4 * MiB, seed=9, dist_a=synth.INT, dist_b=synth.INT,
                   dist_c=synth.INT)
    pp = PinnedProblem(w, ld_pad=(3, 5, 1))
    try:
        ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget)
        ref, _, _ = reference_rows(w, pp.A, pp.B, np.arange(w.M))
        assert np.array_equal(pp.C, ref)
    finally:
        pp.free()


def test_configured_small_workload():
    w = W.SMALL
    pp = PinnedProblem(w, nan_c=True)
    try:
        st, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget)
        assert stats.arena_bytes <= w.budget
        check_rows(w, pp, np.arange(w.M))
    finally:
        pp.free()


def test_alpha_zero_and_k_zero():
    w = W.Workload("a0", 300, 260, 100, 0.0, 0.5, 1 * MiB, seed=3)
    pp = PinnedProblem(w)
    try:
        synth.fill_nan(pp.A)
        C0 = pp.C.copy()
        ooc.ooc_gemm(0.0, pp.A, pp.B, 0.5, pp.C, w.budget)
        assert np.array_equal(pp.C, 0.5 * C0)
        ooc.ooc_gemm(1.0, pp.A[:, :0], pp.B[:0, :], 0.0, pp.C, w.budget)
        assert np.all(pp.C == 0.0)
    finally:
        pp.free()


def test_pageable_memory_rejected():
    A = np.ones((64, 64)); B = np.ones((64, 64)); C = np.ones((64, 64))
    st, _ = ooc.ooc_gemm(1.0, A, B, 0.0, C, 1 * MiB, raise_on_error=False)
    assert st == ooc.OOC_ERR_NOT_PINNED


def test_budget_above_device_memory():
    w = W.Workload("big-arena", 1024, 1024, 64, 1.0, 0.0, 400 * GiB, seed=4)
    pp = PinnedProblem(w)
    try:
        # 80000 C buffers of 512 x 1024 doubles: 312.5 GiB, more than the device has
        plan = ooc.make_plan(512, 1024, 64, ooc.ORDER_COLS, 2, 1, 80000, 3)
        st, _ = ooc.ooc_gemm_planned(1.0, pp.A, pp.B, 0.0, pp.C, w.budget, plan, raise_on_error=False)
        assert st == ooc.OOC_ERR_DEVICE_MEM
    finally:
        pp.free()


def test_injected_failure_then_recovery(monkeypatch):
    w = W.Workload("inject", 1024, 1024, 512, 1.0, 0.5, 4 * MiB, seed=5)
    pp = PinnedProblem(w)
    try:
        plan = ooc.make_plan(256, 256, 512, ooc.ORDER_COLS, 2, 1, 2, 3)
        ops, _ = ooc.ooc_schedule(w.M, w.N, w.K, w.alpha, w.beta, plan)
        cut = len(ops) // 2
        monkeypatch.setenv("OOC_FAIL_AT", str(cut))
        st, stats = ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, plan, raise_on_error=False)
        assert st == ooc.OOC_ERR_INJECTED
        assert stats.blocks_done == sum(1 for o in ops[:cut] if o["kind"] == "d2h")
        monkeypatch.delenv("OOC_FAIL_AT")
        synth.fill(pp.C, w.spec_c())
        ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, plan)
        check_rows(w, pp, np.arange(w.M))
    finally:
        pp.free()


# ---- full-size workloads, sampled rows ------------------------------------------------

@pytest.mark.parametrize("wname", [W.SQUARE.name, W.TALL.name, W.SCALED.name])
def test_full_size_sampled(wname):
    """Every full-size workload in all three tile precisions (FP64, split-BF16
    with 5 slices, split-INT8 with 6), each checked on 256 random rows plus rows
    0, M-1 and both sides of every block-row boundary.  C is refilled with its
    initial values before each product, so beta != 0 workloads are checked in
    every form."""
    w = W.BY_NAME[wname]
    _say(f"full-size workload {w.name}: allocating {w.host_bytes() / GiB:.1f} GiB pinned")
    pp = PinnedProblem(w)
    try:
        forms = [("fp64", ooc.make_opts()),
                 ("split-BF16 x5", ooc.make_opts(precision=ooc.SPLIT_BF16, slices=5)),
                 ("split-INT8 x6", ooc.make_opts(precision=ooc.SPLIT_INT8, slices=6))]
        for x, (label, opts) in enumerate(forms):
            if x > 0 and w.beta != 0.0:
                synth.fill(pp.C, w.spec_c())
            st, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, opts)
            _say(f"  {label}: plan {stats.plan} t={stats.t_total_s:.3f}s "
                 f"{stats.flops / stats.t_total_s / 1e12:.1f} TFLOP/s")
            assert stats.arena_bytes <= w.budget and stats.plan.precision == opts.precision
            rows = sample_rows(w.M, stats.plan.mb, count=256, seed=1 + x)
            check_rows(w, pp, rows, label=f"{label}: ")
    finally:
        pp.free()


# ---- degenerate shapes through tiny budgets (vectors, rank-one updates, skinny C) -----

DEGENERATE = [
    # M, N, K, alpha, beta, budget bytes, precision
    (1, 1, 1, 1.5, 0.5, 64 << 10, ooc.FP64),
    (1, 5000, 300, 1.0, 0.5, 256 << 10, ooc.FP64),
    (5000, 1, 300, -2.0, 1.0, 256 << 10, ooc.FP64),
    (3000, 3000, 1, 1.0, 0.5, 1 << 20, ooc.FP64),
    (2000, 17, 2000, 0.5, 0.0, 512 << 10, ooc.FP64),
    (1500, 1300, 1700, 1.0, 0.5, 3 << 20, ooc.SPLIT_BF16),
    (257, 3001, 129, 1.0, 0.5, 2 << 20, ooc.SPLIT_BF16),
    (1500, 1300, 1700, 1.0, 0.5, 3 << 20, ooc.SPLIT_INT8),
    (3001, 257, 130, -1.0, 0.0, 2 << 20, ooc.SPLIT_INT8),
]


@pytest.mark.parametrize("case", range(len(DEGENERATE)))
def test_degenerate_shapes_small_budgets(case):
    M, N, K, alpha, beta, budget, prec = DEGENERATE[case]
    _say(f"degenerate case {case}: M={M} N={N} K={K} budget={budget} precision={prec}")
    w = W.Workload(f"degenerate{case}", M, N, K, alpha, beta, budget, seed=50 + case)
    pp = PinnedProblem(w, nan_c=(beta == 0.0))
    try:
        # INT8 digits carry 7 bits: 7 slices for the margin 5 BF16 slices give
        slices = 7 if prec == ooc.SPLIT_INT8 else 5
        st, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget,
                                 ooc.make_opts(precision=prec, slices=slices))
        assert stats.arena_bytes <= budget and stats.plan.precision == prec
        rows = np.arange(M) if M * N * K < 2e8 else sample_rows(M, stats.plan.mb)
        check_rows(w, pp, rows)
    finally:
        pp.free()


# ---- boundary options: borrowed caller streams, arena release, planning time, overlap ---

def test_borrowed_streams_arena_release_and_stats():
    """The pipeline runs on three caller-owned streams (created at the default
    priority through the HIP runtime the library links), the result meets the
    gate, the stats carry the planning time and the copy/compute overlap, and
    release_arena frees the arena before the call returns (device free memory
    is back)."""
    from gpu_helpers import HipRuntime
    hip = HipRuntime()
    w = W.Workload("borrowed", 2048, 2048, 2048, 1.0, 0.5, 256 * MiB, seed=31)
    pp = PinnedProblem(w)
    streams = []
    try:
        ooc.ooc_release(-1)
        hip.set_device(0)
        streams = [hip.stream_create() for _ in range(3)]
        plan = ooc.make_plan(512, 1024, 2048, ooc.ORDER_COLS, 2, 2, 2, 3)
        opts = ooc.make_opts(streams=streams, profile=True)
        hip.device_synchronize()
        free0 = hip.mem_free()
        _, stats = ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, plan, opts)
        hip.device_synchronize()
        free_cached = hip.mem_free()
        _say(f"borrowed streams: overlap {stats.overlap:.3f} t_plan {stats.t_plan_s * 1e3:.3f} ms "
             f"t_total {stats.t_total_s * 1e3:.2f} ms arena {stats.arena_bytes}")
        check_rows(w, pp, np.arange(w.M))
        assert 0.0 < stats.overlap <= 1.0
        assert 0.0 < stats.t_plan_s < stats.t_total_s
        assert free0 - free_cached >= 0.9 * stats.arena_bytes  # cached for the next call
        synth.fill(pp.C, w.spec_c())
        opts = ooc.make_opts(streams=streams, release_arena=True)
        _, stats = ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, plan, opts)
        hip.device_synchronize()
        free_released = hip.mem_free()
        _say(f"free device memory: before {free0}, arena cached {free_cached}, arena released {free_released}")
        check_rows(w, pp, np.arange(w.M))
        # the arena went back to the runtime: its free-memory reading rises, or
        # the runtime keeps the freed block for reuse, and then a hipMalloc of
        # the same size takes that block without lowering the reading (which it
        # would lower by the arena's size if the library still held its arena)
        if free_released - free_cached < 0.5 * stats.arena_bytes:
            p = hip.malloc(stats.arena_bytes)
            hip.device_synchronize()
            taken = free_released - hip.mem_free()
            hip.free(p)
            _say(f"the reading did not rise at the release; a same-size hipMalloc then took {taken} bytes")
            assert taken < 0.5 * stats.arena_bytes
        assert stats.overlap == 0.0  # not profiled
        for s in streams:
            hip.stream_synchronize(s)
    finally:
        for s in streams:
            hip.stream_destroy(s)
        pp.free()
        ooc.ooc_release(-1)
