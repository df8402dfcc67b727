"""Pins of the schedule checker: a two-stream pipeline in the paper's
configuration (Fig. 2, the worked example of Fig. 3) is race free and gives
the reference product in any legal order; removing one event wait is caught
both by the hazard check and by the randomised CPU execution."""
import numpy as np
import pytest

import oracle
import synth
from oracle import sched_ref


def paper_pipeline(M, N, K, h, w, alpha, beta, drop=None):
    """Operation list of the paper's two-stream MMOOC for an h x w split.

    Device layout (elements): two A slice buffers, one B slice buffer, two C
    block buffers.  `drop` = (op kind, mat, block) whose waits are removed."""
    mb, nb = -(-M // h), -(-N // w)
    offA = [0, mb * K]
    offB = 2 * mb * K
    offC = [offB + K * nb, offB + K * nb + mb * nb]
    arena = offC[1] + mb * nb
    ops = []
    ev = {}

    def add(op, key):
        if drop is not None and key == drop:
            op["waits"] = []
        ops.append(op)
        ev[key] = len(ops) - 1

    def blk(idx):
        return idx % h, idx // h

    def rows_of(i):
        return i * mb, min(mb, M - i * mb)

    def cols_of(j):
        return j * nb, min(nb, N - j * nb)

    def load_a(idx, stream, waits):
        i, _ = blk(idx)
        r0, r = rows_of(i)
        add(dict(kind="h2d", mat="A", stream=stream, task=idx, waits=waits, row0=r0, col0=0, rows=r, cols=K,
                 dev_off=offA[idx % 2], dev_ld=K), ("h2d", "A", idx))

    def load_b(j, stream, waits):
        c0, c = cols_of(j)
        add(dict(kind="h2d", mat="B", stream=stream, task=j * h, waits=waits, row0=0, col0=c0, rows=K, cols=c,
                 dev_off=offB, dev_ld=nb), ("h2d", "B", j))

    def load_c(idx, stream, waits):
        i, j = blk(idx)
        r0, r = rows_of(i)
        c0, c = cols_of(j)
        add(dict(kind="h2d", mat="C", stream=stream, task=idx, waits=waits, row0=r0, col0=c0, rows=r, cols=c,
                 dev_off=offC[idx % 2], dev_ld=nb), ("h2d", "C", idx))

    n = h * w
    for idx in range(n):
        i, j = blk(idx)
        s1, s2 = idx % 2, (idx + 1) % 2
        if idx == 0:
            load_b(0, s1, [])
            load_a(0, s1, [])
            if beta != 0:
                load_c(0, s1, [])
        r0, r = rows_of(i)
        c0, c = cols_of(j)
        waits = [ev[("h2d", "B", j)], ev[("h2d", "A", idx)]] + ([ev[("h2d", "C", idx)]] if beta != 0 else [])
        add(dict(kind="gemm", stream=s1, task=idx, waits=waits, m=r, n=c, k=K, i0=r0, j0=c0, k0=0,
                 off_a=offA[idx % 2], lda=K, off_b=offB, ldb=nb, off_c=offC[idx % 2], ldc=nb,
                 alpha=alpha, beta=beta), ("gemm", None, idx))
        if idx + 1 < n:
            load_a(idx + 1, s2, [ev[("gemm", None, idx - 1)]] if idx > 0 else [])
            if beta != 0:
                load_c(idx + 1, s2, [ev[("d2h", "C", idx - 1)]] if idx > 0 else [])
            if i == h - 1:
                load_b(j + 1, s2, [ev[("gemm", None, idx)]] + ([ev[("gemm", None, idx - 1)]] if idx > 0 else []))
        add(dict(kind="d2h", mat="C", stream=s1, task=idx, waits=[], row0=r0, col0=c0, rows=r, cols=c,
                 dev_off=offC[idx % 2], dev_ld=nb), ("d2h", "C", idx))
    return ops, arena


def _problem(M, N, K, seed):
    A = synth.matrix(M, K, synth.spec(seed, 0, synth.INT))
    B = synth.matrix(K, N, synth.spec(seed, 1, synth.INT))
    C = synth.matrix(M, N, synth.spec(seed, 2, synth.INT))
    return A, B, C


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_paper_pipeline_worked_example(beta):
    M, K, N, h, w = 4, 8, 4, 4, 2
    ops, arena = paper_pipeline(M, N, K, h, w, 1.0, beta)
    assert arena <= 44
    assert sched_ref.check_hazards(ops) == []
    assert sched_ref.check_cover(ops, M, N, K) == []
    reach = sched_ref.happens_before(ops)
    names = sched_ref.logical_names(ops, h)
    for later, earlier in sched_ref.paper_rules(h, w, beta != 0):
        assert (reach[names[later]] >> names[earlier]) & 1, (later, earlier)
    A, B, C = _problem(M, N, K, 3)
    want, _ = oracle.gemm_rows(1.0, A, B, beta, C)
    for seed in range(20):
        Cw = C.copy()
        sched_ref.execute(ops, A, B, Cw, arena, seed=seed)
        assert np.array_equal(Cw, want)


def test_paper_footprint_matches_partitioner():
    # buffers of the two-stream pipeline are exactly the partitioner's footprint
    from oracle import plan_ref
    M, K, N, h, w = 4, 8, 4, 4, 2
    _, arena = paper_pipeline(M, N, K, h, w, 1.0, 0.5)
    assert arena == plan_ref.footprint(M, N, K, h, w) == 36


@pytest.mark.parametrize("drop", [("h2d", "B", 1), ("gemm", None, 5), ("gemm", None, 1)])
def test_missing_wait_is_caught(drop):
    M, K, N, h, w = 8, 6, 6, 4, 2
    ops, arena = paper_pipeline(M, N, K, h, w, 1.0, 0.5, drop=drop)
    assert sched_ref.check_hazards(ops) != []
    A, B, C = _problem(M, N, K, 4)
    want, _ = oracle.gemm_rows(1.0, A, B, 0.5, C)
    wrong = 0
    for seed in range(200):
        Cw = C.copy()
        sched_ref.execute(ops, A, B, Cw, arena, seed=seed)
        wrong += not np.array_equal(Cw, want)
    assert wrong > 0


@pytest.mark.parametrize("drop", [("h2d", "A", 3), ("h2d", "C", 2)])
def test_same_stream_waits_are_implied(drop):
    # the A slice and C block of block idx+1 go on the stream of block idx-1,
    # so the waits on eA[idx-1] / eC[idx-1] are already implied by stream order
    M, K, N, h, w = 8, 6, 6, 4, 2
    ops, arena = paper_pipeline(M, N, K, h, w, 1.0, 0.5, drop=drop)
    assert sched_ref.check_hazards(ops) == []


def test_ragged_split_pipeline():
    M, K, N, h, w = 10, 7, 9, 3, 2
    ops, arena = paper_pipeline(M, N, K, h, w, -2.0, 0.25)
    assert sched_ref.check_hazards(ops) == []
    assert sched_ref.check_cover(ops, M, N, K) == []
    A, B, C = _problem(M, N, K, 5)
    want, _ = oracle.gemm_rows(-2.0, A, B, 0.25, C)
    Cw = C.copy()
    sched_ref.execute(ops, A, B, Cw, arena, seed=1)
    assert np.array_equal(Cw, want)


def test_cycle_or_forward_wait_rejected():
    ops = [dict(kind="d2h", mat="C", stream=0, task=0, waits=[1], row0=0, col0=0, rows=1, cols=1, dev_off=0, dev_ld=1),
           dict(kind="h2d", mat="C", stream=1, task=0, waits=[], row0=0, col0=0, rows=1, cols=1, dev_off=0, dev_ld=1)]
    with pytest.raises(ValueError):
        sched_ref.happens_before(ops)


# ---- check_cover must reject lists that lose, repeat or misorder work ------------------

def _ksplit_pipeline():
    """One stream, a 2 x 2 grid of C blocks, K split into three panels of 4, 3
    and 5: every C block gets three GEMM ops and one d2h."""
    M, N, K = 6, 4, 12
    mb, nb = 3, 2
    panels = [(0, 4), (4, 3), (7, 5)]
    offA, offB, offC = 0, mb * K, mb * K + K * nb
    ops = []
    for i in range(2):
        for j in range(2):
            ops.append(dict(kind="h2d", mat="C", stream=0, task=0, waits=[], row0=i * mb, col0=j * nb, rows=mb,
                            cols=nb, dev_off=offC, dev_ld=nb))
            for k0, k in panels:
                ops.append(dict(kind="h2d", mat="A", stream=0, task=0, waits=[], row0=i * mb, col0=k0, rows=mb,
                                cols=k, dev_off=offA, dev_ld=k))
                ops.append(dict(kind="h2d", mat="B", stream=0, task=0, waits=[], row0=k0, col0=j * nb, rows=k,
                                cols=nb, dev_off=offB, dev_ld=nb))
                ops.append(dict(kind="gemm", stream=0, task=0, waits=[], m=mb, n=nb, k=k, i0=i * mb, j0=j * nb,
                                k0=k0, off_a=offA, lda=k, off_b=offB, ldb=nb, off_c=offC, ldc=nb, alpha=1.0,
                                beta=1.0))
            ops.append(dict(kind="d2h", mat="C", stream=0, task=0, waits=[], row0=i * mb, col0=j * nb, rows=mb,
                            cols=nb, dev_off=offC, dev_ld=nb))
    return ops, M, N, K, offC + mb * nb


def test_cover_accepts_a_k_split_pipeline():
    ops, M, N, K, arena = _ksplit_pipeline()
    assert sched_ref.check_cover(ops, M, N, K) == []
    A, B, C = _problem(M, N, K, 6)
    want, _ = oracle.gemm_rows(1.0, A, B, 1.0, C)
    Cw = C.copy()
    sched_ref.execute(ops, A, B, Cw, arena)
    assert np.array_equal(Cw, want)


def test_cover_catches_a_dropped_d2h():
    ops, M, N, K, _ = _ksplit_pipeline()
    last = max(x for x, o in enumerate(ops) if o["kind"] == "d2h")
    bad = sched_ref.check_cover(ops[:last] + ops[last + 1:], M, N, K)
    assert any("returned 0 times" in p for p in bad), bad


def test_cover_catches_a_duplicated_d2h():
    ops, M, N, K, _ = _ksplit_pipeline()
    first = min(x for x, o in enumerate(ops) if o["kind"] == "d2h")
    bad = sched_ref.check_cover(ops + [dict(ops[first])], M, N, K)
    assert any("returned 2 times" in p for p in bad), bad


def test_cover_catches_a_missing_k_panel():
    ops, M, N, K, _ = _ksplit_pipeline()
    x = [x for x, o in enumerate(ops) if o["kind"] == "gemm"][4]  # block (0, 1), panel [4, 7)
    bad = sched_ref.check_cover(ops[:x] + ops[x + 1:], M, N, K)
    assert any("[4, 7) not computed" in p for p in bad), bad


def test_cover_catches_a_repeated_panel_that_keeps_the_k_total():
    # the middle panel of block (0, 0) is moved from [4, 7) to [0, 3): every C element still
    # sums k = 12, but [0, 3) is added twice and [4, 7) never
    ops, M, N, K, _ = _ksplit_pipeline()
    gx = [x for x, o in enumerate(ops) if o["kind"] == "gemm"][:3]  # block (0, 0)
    ops = [dict(o) for o in ops]
    ops[gx[1]]["k0"] = 0
    total = sum(ops[x]["k"] for x in gx)
    assert total == K  # a check that only sums k per element would pass this list
    bad = sched_ref.check_cover(ops, M, N, K)
    assert any("computed twice" in p for p in bad) and any("[4, 7) not computed" in p for p in bad), bad


def test_cover_catches_a_d2h_before_the_last_panel():
    ops, M, N, K, _ = _ksplit_pipeline()
    # move block (1, 1)'s d2h in front of its last GEMM on the same stream
    d = max(x for x, o in enumerate(ops) if o["kind"] == "d2h")
    g = max(x for x, o in enumerate(ops) if o["kind"] == "gemm")
    moved = ops[:g] + [ops[d]] + ops[g:d] + ops[d + 1:]
    bad = sched_ref.check_cover(moved, M, N, K)
    assert any("not ordered after GEMM" in p for p in bad), bad
