"""Host-side checks of the C ABI library (no GPU needed): it loads and exports
every declared entry point, its partitioner agrees with the reference, its
operation lists are race free and compute the reference product when run on
the CPU in random legal orders, and it rejects bad arguments before touching
a device."""
import os
import re

import numpy as np
import pytest

import oracle
import synth
from oracle import plan_ref, sched_ref
import paper_1808_05056_amd as ooc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MiB, GiB = 1 << 20, 1 << 30


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "ooc.h")).read()
    names = sorted(set(re.findall(r"^(?:ooc_status|const char\*|int32_t)\s+(ooc_\w+)\s*\(", hdr, re.M)))
    assert len(names) >= 15
    for n in names:
        assert hasattr(ooc._lib, n), n
    assert set(names) == set(ooc.EXPORTS)


def test_partition_matches_reference():
    rng = np.random.default_rng(0)
    cases = [(4, 4, 8, 44 * 8), (1024, 1024, 1024, 8 * MiB), (32768, 32768, 32768, 4 * GiB),
             (65536, 16384, 32768, 8 * GiB), (262144, 8192, 8192, 2 * GiB)]
    for _ in range(300):
        M, N, K = (int(x) for x in rng.integers(1, 300, 3))
        cases.append((M, N, K, int(rng.integers(8, 8 * (M * K + K * N + M * N) + 64))))
    for M, N, K, b in cases:
        assert ooc.ooc_partition(M, N, K, b) == plan_ref.partition(M, N, K, b // 8), (M, N, K, b)


def test_paper_plan_footprint_is_the_papers():
    for M, N, K, b in [(4, 4, 8, 44 * 8), (1024, 1024, 1024, 8 * MiB), (32768, 32768, 32768, 4 * GiB),
                       (300, 200, 100, 200000)]:
        p = ooc.ooc_plan(M, N, K, 0.5, b, ooc.make_opts(planner=ooc.PLAN_PAPER))
        h, w = plan_ref.partition(M, N, K, b // 8)
        assert (p.mb, p.nb, p.kb) == (-(-M // h), -(-N // w), K)
        assert (p.order, p.nbuf_a, p.nbuf_b, p.nbuf_c, p.nstreams) == (ooc.ORDER_COLS, 2, 1, 2, 2)
        assert ooc.ooc_plan_footprint(M, N, K, 0.5, p) == 8 * plan_ref.footprint(M, N, K, h, w) <= b


def _problem(M, N, K, seed):
    A = synth.matrix(M, K, synth.spec(seed, 0, synth.INT))
    B = synth.matrix(K, N, synth.spec(seed, 1, synth.INT))
    C = synth.matrix(M, N, synth.spec(seed, 2, synth.INT))
    return A, B, C


PLANS = [
    # (M, N, K, plan)
    (40, 36, 24, ooc.make_plan(10, 18, 24, ooc.ORDER_COLS, 2, 1, 2, 2)),   # the paper's configuration
    (40, 36, 24, ooc.make_plan(10, 18, 24, ooc.ORDER_COLS, 2, 1, 2, 3)),
    (40, 36, 24, ooc.make_plan(10, 18, 24, ooc.ORDER_COLS, 2, 2, 2, 3)),
    (40, 36, 24, ooc.make_plan(10, 18, 24, ooc.ORDER_ROWS, 1, 2, 2, 3)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS, 2, 2, 2, 3)),     # ragged everywhere, K split
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS, 2, 2, 2, 2)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS_P, 2, 2, 6, 3)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_P, 3, 2, 5, 3)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS_P, 2, 2, 5, 1)),
    (41, 37, 29, ooc.make_plan(41, 37, 29, ooc.ORDER_COLS, 1, 1, 1, 3)),   # one block (in-core)
    (41, 37, 29, ooc.make_plan(9, 37, 29, ooc.ORDER_COLS, 5, 1, 2, 3)),    # all A slices resident
    # initial C staged and folded at a spread K panel
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS_P, 2, 2, 5, 3, nbuf_d=1)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_P, 2, 2, 4, 3, nbuf_d=2)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS, 2, 2, 2, 3, nbuf_d=1)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS, 2, 2, 2, 2, nbuf_d=1)),
    (41, 37, 29, ooc.make_plan(9, 10, 29, ooc.ORDER_COLS, 2, 1, 2, 3, nbuf_d=1)),  # one panel: fold at once
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS_P, 2, 2, 5, 1, nbuf_d=1)),
    # groups of C blocks walked K panel by K panel (ragged last group)
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_P, 4, 2, 4, 3, group=3)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_P, 5, 2, 3, 2, group=2)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS_P, 2, 4, 3, 3, nbuf_d=1, group=2)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS_P, 2, 3, 2, 3, nbuf_d=2, group=2)),
    # every other row (column) walked backwards
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_PS, 4, 2, 4, 3, group=3)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_PS, 3, 2, 5, 3)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS_PS, 2, 4, 3, 3, nbuf_d=1, group=2)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS_PS, 2, 2, 5, 2, nbuf_d=1)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_PS, 5, 2, 3, 1, group=2)),
]


def test_group_walk_order():
    # w = 4 C blocks per row, P = 4 panels, groups of 3: blocks 0-2 panel by panel, then block 3
    plan = ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_P, 4, 2, 4, 3, group=3)
    ops, _ = ooc.ooc_schedule(41, 37, 29, 1.0, 0.0, plan)
    walk = [(op["i0"] // 9, op["j0"] // 10, op["k0"] // 8) for op in ops if op["kind"] == "gemm"]
    row0 = [(0, j, p) for p in range(4) for j in range(3)] + [(0, 3, p) for p in range(4)]
    assert walk[:16] == row0
    assert len(walk) == 5 * 4 * 4
    # group 0 is the whole row; the group size is clamped to the row
    for g in (0, 4, 9):
        p0 = ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_P, 4, 2, 5, 3, group=g)
        ops, _ = ooc.ooc_schedule(41, 37, 29, 1.0, 0.0, p0)
        walk = [(op["i0"] // 9, op["j0"] // 10, op["k0"] // 8) for op in ops if op["kind"] == "gemm"]
        assert walk[:16] == [(0, j, p) for p in range(4) for j in range(4)]
    with pytest.raises(ooc.OOCError):
        ooc.ooc_schedule(41, 37, 29, 1.0, 0.0, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_P, 4, 2, 4, 3, group=-1))


def test_backwards_alternating_walk_order():
    # ROWS_PS: row 0 as ROWS_P; row 1 backwards (last group first, K panels and
    # blocks in reverse), so it starts with the group, panel and block row 0 ended with
    plan = ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_PS, 4, 2, 4, 3, group=3)
    ops, _ = ooc.ooc_schedule(41, 37, 29, 1.0, 0.0, plan)
    walk = [(op["i0"] // 9, op["j0"] // 10, op["k0"] // 8) for op in ops if op["kind"] == "gemm"]
    row0 = [(0, j, p) for p in range(4) for j in range(3)] + [(0, 3, p) for p in range(4)]
    row1 = [(1, 3, p) for p in (3, 2, 1, 0)] + [(1, j, p) for p in (3, 2, 1, 0) for j in (2, 1, 0)]
    assert walk[:32] == row0 + row1
    assert walk[32:48] == [(2, j, p) for p in range(4) for j in range(3)] + [(2, 3, p) for p in range(4)]
    assert sorted(walk) == sorted((i, j, p) for i in range(5) for j in range(4) for p in range(4))
    # COLS_PS is its transpose
    plan = ooc.make_plan(10, 9, 8, ooc.ORDER_COLS_PS, 2, 4, 4, 3, group=3)
    ops, _ = ooc.ooc_schedule(37, 41, 29, 1.0, 0.0, plan)
    walk = [(op["i0"] // 10, op["j0"] // 9, op["k0"] // 8) for op in ops if op["kind"] == "gemm"]
    assert walk[:32] == [(j, i, p) for (i, j, p) in row0 + row1]
    # a C block that accumulates its K panels backwards reads C once, at its first panel
    ops, _ = ooc.ooc_schedule(41, 37, 29, 1.0, 0.5, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_PS, 4, 2, 4, 3, group=3))
    first = {}
    for op in ops:
        if op["kind"] == "gemm":
            key = (op["i0"], op["j0"])
            assert (op["beta"] == 0.5) == (key not in first)
            first.setdefault(key, op["k0"])
    assert first[(9, 30)] == 24  # row 1 starts block (1, 3) at the last K panel


def test_copies_in_order_of_free_buffers():
    # with a copy stream, each copy waits for at most kernels that precede every
    # later copy's wait: the copy stream never idles behind a copy whose buffer
    # frees later than the next one's
    M, N, K = 41, 37, 29
    plan = ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_P, 4, 2, 4, 3, group=3)
    ops, _ = ooc.ooc_schedule(M, N, K, 1.0, 0.5, plan)
    rank = {x: r for r, x in enumerate(x for x, op in enumerate(ops) if op["kind"] == "gemm")}
    for x, op in enumerate(ops):  # a copy back to the host ranks just after its kernel
        if op["kind"] == "d2h":
            rank[x] = max(rank[y] for y in op["waits"]) + 0.5
    war = [max([rank[y] for y in op["waits"]], default=-1) for op in ops if op["kind"] == "h2d"]
    assert war == sorted(war)
    assert sched_ref.check_hazards(ops) == []


@pytest.mark.parametrize("beta", [0.0, 0.5])
@pytest.mark.parametrize("case", range(len(PLANS)))
def test_schedule_is_race_free_and_correct(case, beta):
    M, N, K, plan = PLANS[case]
    ops, arena = ooc.ooc_schedule(M, N, K, 1.5, beta, plan)
    assert arena * 8 == ooc.ooc_plan_footprint(M, N, K, beta, plan)
    assert sched_ref.check_hazards(ops) == []
    assert sched_ref.check_cover(ops, M, N, K) == []
    assert all(op["stream"] < plan.nstreams for op in ops)
    A, B, C = _problem(M, N, K, 7 + case)
    want, _ = oracle.gemm_rows(1.5, A, B, beta, C)
    for seed in range(8):
        Cw = C.copy() if beta != 0 else np.full_like(C, np.nan)
        sched_ref.execute(ops, A, B, Cw, arena, seed=seed)
        assert np.array_equal(Cw, want), seed


def test_paper_configuration_implies_the_papers_event_order():
    for (M, K, N, budget) in [(4, 8, 4, 44 * 8), (64, 30, 50, 3000 * 8)]:
        h, w = plan_ref.partition(M, N, K, budget // 8)
        p = ooc.ooc_plan(M, N, K, 0.5, budget, ooc.make_opts(planner=ooc.PLAN_PAPER))
        for beta in (0.0, 0.5):
            ops, arena = ooc.ooc_schedule(M, N, K, 1.0, beta, p)
            assert arena <= budget // 8
            reach = sched_ref.happens_before(ops)
            names = sched_ref.logical_names(ops, h)
            # a slice still resident in its buffer is not sent again: its
            # arrival is the earlier copy of the same rows
            for x, op in enumerate(ops):
                if op["kind"] == "gemm" and (sched_ref.H2D_A, op["task"]) not in names:
                    src = max(y for y in range(x) if ops[y]["kind"] == "h2d" and ops[y]["mat"] == "A"
                              and ops[y]["row0"] == op["i0"])
                    names[(sched_ref.H2D_A, op["task"])] = src
                    names[("resident", op["task"])] = True
            checked = 0
            for later, earlier in sched_ref.paper_rules(h, w, beta != 0):
                if later[0] == sched_ref.H2D_A and ("resident", later[1]) in names:
                    continue  # no copy, so nothing to order
                assert (reach[names[later]] >> names[earlier]) & 1, (later, earlier)
                checked += 1
            assert checked > 0


def test_alpha_zero_and_k_zero_schedules_read_no_ab():
    plan = ooc.make_plan(10, 9, 8, ooc.ORDER_COLS, 2, 1, 2, 3)
    for (alpha, K) in [(0.0, 16), (1.0, 0)]:
        ops, arena = ooc.ooc_schedule(30, 27, K, alpha, 0.5, plan)
        assert not any(op["kind"] == "h2d" and op["mat"] in "AB" for op in ops)
        C = synth.matrix(30, 27, synth.spec(3, 2, synth.INT))
        Cw = C.copy()
        sched_ref.execute(ops, np.full((30, max(K, 1)), np.nan), np.full((max(K, 1), 27), np.nan), Cw, arena)
        assert np.array_equal(Cw, 0.5 * C)


def test_candidates_fit_budget_and_are_sorted():
    for (M, N, K, b) in [(32768, 32768, 32768, 4 * GiB), (8000, 9000, 7000, 512 * MiB), (1024, 1024, 1024, 8 * MiB)]:
        plans, times = ooc.ooc_plan_candidates(M, N, K, 0.5, b)
        assert plans and times == sorted(times)
        for p in plans:
            assert ooc.ooc_plan_footprint(M, N, K, 0.5, p) <= b
        best = ooc.ooc_plan(M, N, K, 0.5, b)
        assert ooc.ooc_plan_footprint(M, N, K, 0.5, best) <= b


def test_argument_errors_before_device_access():
    s, _ = ooc.ooc_gemm_raw(-1, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 1 << 20)
    assert s == ooc.OOC_ERR_ARG
    A = np.zeros((4, 4)); B = np.zeros((4, 4)); C = np.zeros((4, 4))
    s, _ = ooc.ooc_gemm_raw(4, 4, 4, 1.0, A.ctypes.data, 3, B.ctypes.data, 4, 0.0, C.ctypes.data, 4, 1 << 20)
    assert s == ooc.OOC_ERR_ARG and "lda" in ooc.ooc_last_error()
    s, _ = ooc.ooc_gemm_raw(4, 4, 4, 1.0, A.ctypes.data, 4, B.ctypes.data, 4, 0.0, None, 4, 1 << 20)
    assert s == ooc.OOC_ERR_ARG
    s, _ = ooc.ooc_gemm_raw(4, 4, 4, 1.0, None, 4, B.ctypes.data, 4, 0.0, C.ctypes.data, 4, 1 << 20)
    assert s == ooc.OOC_ERR_ARG
    # nothing fits in 100 bytes
    s, _ = ooc.ooc_gemm_raw(4, 4, 8, 1.0, A.ctypes.data, 8, B.ctypes.data, 4, 0.0, C.ctypes.data, 4, 100)
    assert s == ooc.OOC_ERR_BUDGET
    # empty problems return at once
    s, _ = ooc.ooc_gemm_raw(0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 0)
    assert s == ooc.OOC_OK
    # a plan larger than the budget is refused
    plan = ooc.make_plan(4, 4, 8, ooc.ORDER_COLS, 1, 1, 1, 3)
    st = ooc._lib.ooc_gemm_planned(4, 4, 8, 1.0, A.ctypes.data, 8, B.ctypes.data, 4, 0.0, C.ctypes.data, 4, 64,
                                   ooc.ctypes.byref(plan), None, None)
    assert st == ooc.OOC_ERR_BUDGET
    bad = ooc.make_plan(0, 4, 8)
    with pytest.raises(ooc.OOCError):
        ooc.ooc_plan_footprint(4, 4, 8, 0.0, bad)
    # the split tile products check their arguments before touching a device
    for fn in (ooc._lib.ooc_split_gemm_device, ooc._lib.ooc_split_int8_gemm_device):
        for s_bad in (0, 9):
            st = fn(0, 4, 4, 4, s_bad, 1.0, A.ctypes.data, 4, B.ctypes.data, 4, 0.0, C.ctypes.data, 4, 1, None)
            assert st == ooc.OOC_ERR_ARG and "slices" in ooc.ooc_last_error()
        st = fn(0, 4, 4, 4, 6, 1.0, A.ctypes.data, 3, B.ctypes.data, 4, 0.0, C.ctypes.data, 4, 1, None)
        assert st == ooc.OOC_ERR_ARG
        assert fn(0, 0, 4, 4, 6, 1.0, None, 4, None, 4, 0.0, None, 4, 1, None) == ooc.OOC_OK
    # a split plan with a slice count outside 1..8 or an unknown precision is refused
    for prec, sl in ((ooc.SPLIT_INT8, 0), (ooc.SPLIT_INT8, 9), (3, 6)):
        with pytest.raises(ooc.OOCError):
            ooc.ooc_plan_footprint(64, 64, 64, 0.0, ooc.make_plan(32, 32, 32, precision=prec, slices=sl))


SPLIT_PLANS = [
    (41, 37, 29, ooc.make_plan(9, 10, 29, ooc.ORDER_COLS, 2, 1, 2, 2, precision=ooc.SPLIT_BF16, slices=3)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS_P, 2, 2, 5, 2, precision=ooc.SPLIT_BF16, slices=2, nbuf_d=1)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS, 2, 2, 2, 3, precision=ooc.SPLIT_BF16, slices=1)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_PS, 4, 2, 4, 2, precision=ooc.SPLIT_BF16, slices=2, group=3)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_COLS, 2, 2, 2, 2, precision=ooc.SPLIT_INT8, slices=2)),
    (41, 37, 29, ooc.make_plan(9, 10, 8, ooc.ORDER_ROWS_P, 2, 2, 5, 3, precision=ooc.SPLIT_INT8, slices=1, nbuf_d=1)),
]


@pytest.mark.parametrize("case", range(len(SPLIT_PLANS)))
def test_split_schedule_race_free(case):
    from oracle import split_ref
    M, N, K, plan = SPLIT_PLANS[case]
    ops, arena = ooc.ooc_schedule(M, N, K, 1.0, 0.5, plan)
    assert any(op["kind"] == "split_gemm" and op["len_w"] > 0 for op in ops)
    assert sched_ref.check_hazards(ops) == []
    assert sched_ref.check_cover(ops, M, N, K) == []
    A, B, C = _problem(M, N, K, 30 + case)
    want, _ = oracle.gemm_rows(1.0, A, B, 0.5, C)

    # the workspace: the panels whose slices the last split product left there;
    # a product flagged to reuse them takes them from here, not from the arena,
    # so a wrong flag gives a wrong result
    ws = {}

    def split_model(op, ar):
        def view(off, r, c, ld):
            return np.lib.stride_tricks.as_strided(ar[off:], shape=(r, c), strides=(ld * 8, 8))
        a = np.array(view(op["off_a"], op["m"], op["k"], op["lda"]))
        b = np.array(view(op["off_b"], op["k"], op["n"], op["ldb"]))
        c = view(op["off_c"], op["m"], op["n"], op["ldc"])
        if op["reuse_a"]:
            assert ws["a"].shape == a.shape
            a = ws["a"]
        if op["reuse_b"]:
            assert ws["b"].shape == b.shape
            b = ws["b"]
        ws["a"], ws["b"] = a, b
        fmt = "i8" if plan.precision == ooc.SPLIT_INT8 else "bf16"
        res = op["alpha"] * split_ref.slice_sum(a, b, plan.slices, fmt)
        if op["beta"] != 0.0:
            res = res + op["beta"] * c
        if op["gamma"] != 0.0:
            res = res + op["gamma"] * view(op["off_d"], op["m"], op["n"], op["ldd"])
        c[...] = res
        ar[op["off_w"]:op["off_w"] + op["len_w"]] = np.nan  # scribble over the workspace

    for seed in range(4):
        Cw = C.copy()
        ws.clear()
        sched_ref.execute(ops, A, B, Cw, arena, seed=seed, kernels={"split_gemm": split_model})
        assert np.array_equal(Cw, want)


def test_split_schedules_reuse_the_slices_of_shared_panels():
    # consecutive products on one A panel (rows in groups) or one B panel
    # (a column without a K split) slice it once; edge blocks of other extents,
    # and K panels walked inside a block, do not reuse
    counts = []
    for M, N, K, plan in SPLIT_PLANS:
        ops, _ = ooc.ooc_schedule(M, N, K, 1.0, 0.5, plan)
        sp = [op for op in ops if op["kind"] == "split_gemm"]
        counts.append((sum(op["reuse_a"] for op in sp), sum(op["reuse_b"] for op in sp)))
        prev = None
        for op in sp:
            if op["reuse_a"] or op["reuse_b"]:
                assert prev is not None and (prev["m"], prev["n"], prev["k"]) == (op["m"], op["n"], op["k"])
            if op["reuse_a"]:
                assert (prev["off_a"], prev["lda"]) == (op["off_a"], op["lda"])
            if op["reuse_b"]:
                assert (prev["off_b"], prev["ldb"]) == (op["off_b"], op["ldb"])
            prev = op
    assert counts[0] == (0, 12) and counts[3][0] == 40 and counts[5] == (40, 0)
    assert counts[2] == (0, 0) and counts[4] == (0, 0)


def test_split_footprint_counts_workspace():
    p64 = ooc.make_plan(512, 512, 1024, ooc.ORDER_COLS, 2, 1, 2, 3)
    ps = ooc.make_plan(512, 512, 1024, ooc.ORDER_COLS, 2, 1, 2, 3, precision=ooc.SPLIT_BF16, slices=6)
    extra = ooc.ooc_plan_footprint(2048, 2048, 1024, 0.0, ps) - ooc.ooc_plan_footprint(2048, 2048, 1024, 0.0, p64)
    assert extra >= 2 * 6 * (512 + 512) * 1024
    # INT8 slices take one byte per element and slice instead of two
    pi = ooc.make_plan(512, 512, 1024, ooc.ORDER_COLS, 2, 1, 2, 3, precision=ooc.SPLIT_INT8, slices=6)
    extra8 = ooc.ooc_plan_footprint(2048, 2048, 1024, 0.0, pi) - ooc.ooc_plan_footprint(2048, 2048, 1024, 0.0, p64)
    assert extra8 >= 6 * (512 + 512) * 1024
    assert extra - extra8 == 6 * (512 + 512) * 1024


def test_int8_plans_and_mlp_decline():
    # the cost model prices INT8 slice products at twice the BF16 rate: for the
    # same plan its predicted time is lower; the learned planner, which has not
    # seen INT8 timings, leaves the choice to the cost model
    M = N = K = 8192
    budget = 2 << 30
    pb = ooc.ooc_plan(M, N, K, 0.0, budget, ooc.make_opts(planner=ooc.PLAN_MODEL, precision=ooc.SPLIT_BF16, slices=6))
    pi = ooc.ooc_plan(M, N, K, 0.0, budget, ooc.make_opts(planner=ooc.PLAN_MODEL, precision=ooc.SPLIT_INT8, slices=6))
    assert pi.precision == ooc.SPLIT_INT8 and pi.slices == 6
    same = ooc.make_plan(pb.mb, pb.nb, pb.kb, pb.order, pb.nbuf_a, pb.nbuf_b, pb.nbuf_c, pb.nstreams,
                         precision=ooc.SPLIT_INT8, slices=6, nbuf_d=pb.nbuf_d, group=pb.group)
    assert ooc.ooc_plan_predict(M, N, K, 0.0, same) < ooc.ooc_plan_predict(M, N, K, 0.0, pb)
    pm = ooc.ooc_plan(M, N, K, 0.0, budget, ooc.make_opts(planner=ooc.PLAN_MLP, precision=ooc.SPLIT_INT8, slices=6))
    assert pm.as_dict() == pi.as_dict()


def test_planner_features():
    plans, times = ooc.ooc_plan_candidates(32768, 32768, 32768, 0.5, 4 << 30)
    X = ooc.ooc_mlp_features(32768, 32768, 32768, 0.5, 4 << 30, plans[:10])
    assert X.shape == (10, ooc.MLP_FEATURES)
    assert np.allclose(X[:, 0], 15) and np.allclose(X[:, 3], 32)
    assert np.allclose(X[:, 7:11].sum(axis=1), 1)
    # the cost-model feature is log2 of the candidate's modelled time
    assert np.allclose(X[:, 16], np.log2(times[:10]), atol=1e-5)


def test_gpu_test_plans_fit_their_budgets():
    # the fixed plans of the GPU tests must fit the 8 MiB budget of their workload
    import test_gpu_parity
    for name, plan, _ in test_gpu_parity.SMALL_PLANS:
        if plan is not None:
            for beta in (0.0, 0.5):
                assert ooc.ooc_plan_footprint(1024, 1024, 1024, beta, plan) <= 8 << 20, name
    split_plan = ooc.make_plan(256, 320, 320, ooc.ORDER_COLS, 2, 2, 2, 3, precision=ooc.SPLIT_BF16, slices=6)
    assert ooc.ooc_plan_footprint(1000, 900, 1100, 0.5, split_plan) <= 8 << 20
    # the race-stress plans fit their 6 MiB budget and pass the CPU hazard checker
    import test_gpu_race_stress
    for name, plan, _ in test_gpu_race_stress.PLANS:
        if plan is not None:
            assert ooc.ooc_plan_footprint(1024, 768, 640, 0.5, plan) <= 6 << 20, name
            ops, _ = ooc.ooc_schedule(1024, 768, 640, 1.5, 0.5, plan)
            assert sched_ref.check_hazards(ops) == [], name


DEGENERATE = [
    # M, N, K, beta, budget bytes, precision
    (1, 1, 1, 0.5, 64 << 10, ooc.FP64),
    (1, 5000, 300, 0.5, 256 << 10, ooc.FP64),     # a row vector times a wide matrix
    (5000, 1, 300, 1.0, 256 << 10, ooc.FP64),     # a matrix times a column vector
    (3000, 3000, 1, 0.5, 1 << 20, ooc.FP64),      # rank-one update
    (2000, 17, 2000, 0.0, 512 << 10, ooc.FP64),   # skinny C
    (1500, 1300, 1700, 0.5, 3 << 20, ooc.SPLIT_BF16),
    (257, 3001, 129, 0.5, 2 << 20, ooc.SPLIT_BF16),
]


@pytest.mark.parametrize("case", range(len(DEGENERATE)))
def test_model_planner_covers_small_budgets(case):
    M, N, K, beta, budget, prec = DEGENERATE[case]
    opts = ooc.make_opts(precision=prec, slices=5)
    plan = ooc.ooc_plan(M, N, K, beta, budget, opts)
    assert ooc.ooc_plan_footprint(M, N, K, beta, plan) <= budget
    ops, arena = ooc.ooc_schedule(M, N, K, 1.0, beta, plan)
    assert sched_ref.check_hazards(ops) == []
    assert sched_ref.check_cover(ops, M, N, K) == []


def test_model_planner_finds_a_plan_where_the_papers_rule_does():
    rng = np.random.default_rng(12)
    for _ in range(30):
        M, N, K = (int(x) for x in rng.integers(1, 3000, 3))
        budget = int(rng.integers(8, 4096)) * 1024
        try:
            ooc.ooc_plan(M, N, K, 0.5, budget, ooc.make_opts(planner=ooc.PLAN_PAPER))
        except ooc.OOCError:
            continue
        plan = ooc.ooc_plan(M, N, K, 0.5, budget)
        assert ooc.ooc_plan_footprint(M, N, K, 0.5, plan) <= budget


def test_size_sweep_in_core_limit():
    """The in-core limit of the size sweep is the largest N with 3 * 8 * N^2
    bytes within the budget: 16384 exactly at 6 GiB (the paper's Xeon Phi
    threshold, Section VI), 23170 at 12 GiB (the paper's largest in-core size
    for its 12 GiB GPU is 22528, the last size of its sweep below the limit)."""
    from paper_1808_05056_amd import size_sweep as S
    GiB = 1 << 30
    assert S.in_core_limit(6 * GiB) == 16384
    assert S.in_core_limit(12 * GiB) == 23170
    for b in (6 * GiB, 12 * GiB, 192 << 20, 1 << 20):
        n = S.in_core_limit(b)
        assert 24 * n * n <= b < 24 * (n + 1) ** 2
    # the paper's partitioner is in core exactly up to the limit
    for b in (192 << 20, 6 * GiB):
        n = S.in_core_limit(b)
        assert S.is_in_core(ooc.ooc_plan(n, n, n, 0.0, b, ooc.make_opts(planner=ooc.PLAN_PAPER)), n)
        assert not S.is_in_core(ooc.ooc_plan(n + 1, n + 1, n + 1, 0.0, b, ooc.make_opts(planner=ooc.PLAN_PAPER)), n + 1)


def test_planner_sweep_refeature(tmp_path):
    """Saved timings are re-featured with the current cost model: the features
    equal those the library computes for the same plans now."""
    import json
    from paper_1808_05056_amd import planner_sweep as ps
    plans, _ = ooc.ooc_plan_candidates(9000, 7000, 5000, 0.0, 1 << 30, ooc.make_opts(precision=ooc.SPLIT_BF16, slices=5))
    meta = [{"problem": 0, "M": 9000, "N": 7000, "K": 5000, "beta": 0.0, "budget": 1 << 30, "plan": p.as_dict(),
             "seconds": 0.1 + 0.01 * i} for i, p in enumerate(plans[:5])]
    path = str(tmp_path / "t.npz")
    with open(path + ".json", "w") as f:
        json.dump(meta, f)
    X, y = ps.refeature(path)
    assert np.array_equal(X, ooc.ooc_mlp_features(9000, 7000, 5000, 0.0, 1 << 30, plans[:5]))
    assert np.allclose(y, [r["seconds"] for r in meta])
    assert np.all(X[:, -1] == 5)  # the slice-count feature


def test_binding_structs_match_the_header(tmp_path):
    """Every field of the ABI structs sits at the same offset, and every struct
    has the same size, in the ctypes binding as in include/ooc.h (compiled with
    gcc): the binding marshals the new fields (borrowed streams, arena release,
    planning time, overlap) where the library reads and writes them."""
    import subprocess
    structs = {"ooc_plan_t": ooc.ooc_plan_t, "ooc_opts": ooc.ooc_opts, "ooc_stats": ooc.ooc_stats,
               "ooc_op": ooc.ooc_op}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ooc.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", exe])
    out = subprocess.check_output([exe], text=True).split("\n")
    got = {}
    for ln in out:
        if ln:
            s, f, v = ln.split()
            got[(s, f)] = int(v)
    import ctypes
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
    for f in ("streams", "release_arena"):
        assert f in dict(ooc.ooc_opts._fields_)
    for f in ("t_plan_s", "overlap"):
        assert f in dict(ooc.ooc_stats._fields_)


def test_make_opts_borrowed_streams_and_release():
    o = ooc.make_opts(streams=[0x1234, None, 0x5678], release_arena=True)
    assert o.streams[0] == 0x1234 and not o.streams[1] and o.streams[2] == 0x5678
    assert o.release_arena == 1
    d = ooc.make_opts()
    assert not any(d.streams) and d.release_arena == 0


def test_sweep_planner_in_planning_only_calls_is_the_cost_model():
    # the measured sweep needs the caller's operands: planning-only calls
    # return the cost model's choice for PLAN_SWEEP (the product calls time it)
    for (M, N, K, beta, budget) in ((8192, 6000, 4000, 0.5, 256 << 20), (3000, 40000, 1000, 0.0, 1 << 30)):
        sw = ooc.ooc_plan(M, N, K, beta, budget, ooc.make_opts(planner=ooc.PLAN_SWEEP))
        mo = ooc.ooc_plan(M, N, K, beta, budget, ooc.make_opts(planner=ooc.PLAN_MODEL))
        assert sw.as_dict() == mo.as_dict()


def test_int8_tile_width_rule():
    # 8192^2 blocks on 256 CUs: 1024 wide tiles (4 waves) against 2048 narrow
    # ones (8 waves): wide; a 4096 x 2048 block: 128 wide tiles (1 wave of half
    # the CUs) against 256 narrow (1 wave): narrow; bad sizes are refused
    assert ooc.ooc_split_int8_wide_tiles(8192, 8192, 256) == 1
    assert ooc.ooc_split_int8_wide_tiles(4096, 2048, 256) == 0
    assert ooc.ooc_split_int8_wide_tiles(0, 2048, 256) == -1
    assert ooc.ooc_split_int8_wide_tiles(4096, 2048, 0) == -1
    # any valid block gets a width
    for m, n in [(256, 256), (1024, 4096), (65536, 8192), (300, 9000)]:
        assert ooc.ooc_split_int8_wide_tiles(m, n, 256) in (0, 1)
