"""Accumulation sessions on the host (no GPU): the operation lists of every
session step (resident rows updated in place, the other rows streamed) are race
free, cover every product term exactly once, and -- run on the CPU in random
legal orders, with the resident rows kept in a device arena that outlives the
steps -- give exactly the oracle's C = beta*C_in + sum_s alpha_s A_s B_s
(applied one step after the other) on integer data.

Section V: the paper's MMOOC as the local step of SUMMA / HSUMMA (the
step/nsteps logic of Fig. 2)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import sched_ref
import paper_1808_05056_amd as ooc

MiB = 1 << 20

# M, N, budget bytes, beta, K per step, alpha per step
CASES = [
    (300, 200, 4 * MiB, 0.5, [50, 70, 40], [1.0, -2.0, 0.5]),      # C fits half the budget: all rows resident
    (700, 300, 2 * MiB, -1.5, [64, 33], [1.0, 1.0]),                # 384 rows resident, 316 streamed
    (260, 900, 1 * MiB, 0.0, [100, 1, 90], [2.0, 1.0, -1.0]),       # beta = 0: C never read; 72 rows resident
    (5000, 40, 1 * MiB, 2.0, [20, 30], [1.0, 0.25]),                # 1536 resident rows of 5000
]


def _mats(M, N, Ks, seed):
    A = [synth.matrix(M, K, synth.spec(seed + s, 0, synth.INT)) for s, K in enumerate(Ks)]
    B = [synth.matrix(K, N, synth.spec(seed + s, 1, synth.INT)) for s, K in enumerate(Ks)]
    C = synth.matrix(M, N, synth.spec(seed, 2, synth.INT))
    return A, B, C


def _oracle(beta, C0, A, B, alphas):
    """The session's result by the oracle, one step after the other."""
    C = C0.copy()
    for s, (a, b) in enumerate(zip(A, B)):
        C, _ = oracle.gemm_rows(alphas[s], a, b, beta if s == 0 else 1.0, C if (beta != 0.0 or s > 0) else None)
    return C


@pytest.mark.parametrize("case", range(len(CASES)))
def test_session_steps_race_free_and_exact(case):
    M, N, budget, beta, Ks, alphas = CASES[case]
    R = ooc.ooc_accum_resident_rows(M, N, budget)
    assert 0 < R <= M
    if R < M:
        assert 8 * R * N <= budget // 2 and (R % 128 == 0 or R < 128)
    A, B, C0 = _mats(M, N, Ks, 10 * case + 1)
    want = _oracle(beta, C0, A, B, alphas)
    for seed in range(3):
        C = C0.copy()
        arena = np.full(budget // 8, np.nan)
        if beta != 0.0:
            arena[:R * N] = C[:R].reshape(-1)  # the resident rows as the session loads them
        for s, K in enumerate(Ks):
            beta_eff = beta if s == 0 else 1.0
            for part in (0, 1):
                ops, elems = ooc.ooc_accum_schedule(M, N, K, alphas[s], beta_eff, budget, part)
                if (part == 0 and R == 0) or (part == 1 and R == M):
                    assert ops == []
                    continue
                assert elems <= budget // 8
                rows = slice(0, R) if part == 0 else slice(R, M)
                mrows = R if part == 0 else M - R
                assert sched_ref.check_hazards(ops) == []
                assert sched_ref.check_cover(ops, mrows, N, K, returns_home=(part == 1)) == []
                if part == 0:
                    # the resident rows are only written inside [0, R*N) of the arena, never copied
                    assert all(o["kind"] != "d2h" and not (o["kind"] == "h2d" and o["mat"] == "C") for o in ops)
                    assert all(o["off_c"] + (o["m"] - 1) * o["ldc"] + o["n"] <= R * N
                               for o in ops if o["kind"] == "gemm")
                    assert all(o["dev_off"] >= R * N for o in ops if o["kind"] == "h2d")
                else:
                    # the streamed rows' buffers lie after the resident rows
                    assert all(min(o[k] for k in ("off_a", "off_b", "off_c")) >= R * N
                               for o in ops if o["kind"] == "gemm")
                    assert all(o["dev_off"] >= R * N for o in ops if o["kind"] in ("h2d", "d2h"))
                sched_ref.execute(ops, A[s][rows], B[s], C[rows], elems, seed=seed + s, arena=arena)
        C[:R] = arena[:R * N].reshape(R, N)  # written back at the end of the session
        assert np.array_equal(C, want), (case, seed)


def test_resident_cover_rejects_a_copy_home():
    # a resident op list that returns a block is flagged
    M, N, budget = 300, 200, 4 * MiB
    ops, _ = ooc.ooc_accum_schedule(M, N, 50, 1.0, 0.5, budget, 0)
    assert sched_ref.check_cover(ops, M, N, 50, returns_home=False) == []
    bad = ops + [dict(kind="d2h", mat="C", stream=0, task=0, waits=[], row0=0, col0=0, rows=M, cols=N, dev_off=0,
                      dev_ld=N)]
    assert any("returned 1 times" in p for p in sched_ref.check_cover(bad, M, N, 50, returns_home=False))


def test_resident_rows_rule():
    assert ooc.ooc_accum_resident_rows(100, 100, 160000) == 100  # 80000 bytes = half the budget
    assert ooc.ooc_accum_resident_rows(101, 100, 160000) == 100  # one row more does not fit
    assert ooc.ooc_accum_resident_rows(1000, 1000, 4 * MiB) == 256  # 262 rows fit, rounded to 128s
    assert ooc.ooc_accum_resident_rows(10, 10 ** 6, MiB) == 0  # not even one row fits half the budget
    assert ooc.ooc_accum_resident_rows(0, 10, MiB) == 0


def test_session_argument_errors_before_device_access():
    import ctypes
    h = ctypes.c_void_p()
    assert ooc._lib.ooc_accum_begin(-1, 4, 0.0, None, 4, MiB, None, ctypes.byref(h)) == ooc.OOC_ERR_ARG
    assert ooc._lib.ooc_accum_begin(4, 4, 0.0, None, 4, MiB, None, ctypes.byref(h)) == ooc.OOC_ERR_ARG
    assert ooc._lib.ooc_accum_begin(4, 4, 0.0, 1, 3, MiB, None, ctypes.byref(h)) == ooc.OOC_ERR_ARG
    assert ooc._lib.ooc_accum_step(None, 4, 1.0, None, 4, None, 4, None) == ooc.OOC_ERR_ARG
    assert ooc._lib.ooc_accum_end(None, None) == ooc.OOC_ERR_ARG
