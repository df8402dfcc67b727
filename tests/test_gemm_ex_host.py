"""Host checks of the transposed-B and lower-triangle forms of the
out-of-core product (ooc_gemm_ex): their operation lists are race free,
cover every owed element of C exactly once, never touch blocks wholly above
the diagonal, and, executed on the CPU in random orders that respect the
waits, give alpha*A@op(B) + beta*C on the lower triangle with the upper
triangle unchanged (exact on integer inputs)."""
import numpy as np
import pytest

import synth
from oracle import sched_ref
import paper_1808_05056_amd as ooc

from test_abi_host import PLANS


def _problem(M, N, K, seed, transb):
    A = synth.matrix(M, K, synth.spec(seed, 0, synth.INT))
    B = synth.matrix(N, K, synth.spec(seed, 1, synth.INT)) if transb else synth.matrix(K, N, synth.spec(seed, 1, synth.INT))
    C = synth.matrix(M, N, synth.spec(seed, 2, synth.INT))
    return A, B, C


def _want(alpha, A, B, beta, C, transb, lower):
    opB = B.T if transb else B
    full = alpha * (A @ opB) + (beta * C if beta != 0.0 else 0.0)
    if not lower:
        return full
    M, N = C.shape
    keep = np.tril(np.ones((M, N), dtype=bool))
    out = C.copy()
    out[keep] = full[keep]
    return out


FORMS = [(True, False), (False, True), (True, True)]


@pytest.mark.parametrize("form", range(len(FORMS)))
@pytest.mark.parametrize("beta", [0.0, 0.5])
@pytest.mark.parametrize("case", [0, 1, 3, 4, 5, 6, 7, 9, 10, 11])
def test_ex_schedule_race_free_and_correct(case, beta, form):
    transb, lower = FORMS[form]
    M, N, K, plan = PLANS[case]
    ops, arena = ooc.ooc_schedule(M, N, K, 1.5, beta, plan, transb=transb, lower=lower)
    assert sched_ref.check_hazards(ops) == []
    assert sched_ref.check_cover(ops, M, N, K, lower=lower) == []
    for op in ops:
        if op["kind"] == "gemm":
            assert op["transb"] == transb and op["lower"] == lower
            if lower:  # no block wholly above the diagonal is computed
                assert op["i0"] + op["m"] - 1 >= op["j0"]
    A, B, C = _problem(M, N, K, 30 + case, transb)
    if lower:
        C[np.triu_indices(M, 1, N)] = np.nan  # never read by the arithmetic, must come back as it was
    want = _want(1.5, A, B, beta, C, transb, lower)
    for seed in range(4):
        Cw = C.copy()
        if beta == 0.0:
            Cw[np.tril(np.ones((M, N), dtype=bool)) if lower else np.ones((M, N), dtype=bool)] = np.nan
        sched_ref.execute(ops, A, B, Cw, arena, seed=seed)
        assert np.array_equal(Cw, want, equal_nan=True), seed


def test_lower_skips_blocks_above_the_diagonal():
    M = N = 64
    K = 16
    plan = ooc.make_plan(16, 16, 16, ooc.ORDER_COLS, 2, 1, 2, 3)
    full, _ = ooc.ooc_schedule(M, N, K, 1.0, 0.0, plan, transb=True)
    low, _ = ooc.ooc_schedule(M, N, K, 1.0, 0.0, plan, transb=True, lower=True)
    ng = lambda ops: sum(op["kind"] == "gemm" for op in ops)
    assert ng(full) == 16 and ng(low) == 10  # 4 x 4 blocks, 10 on or below the diagonal
    # straddling (diagonal) blocks are loaded even with beta == 0 so their upper part survives
    c_loads = [op for op in low if op["kind"] == "h2d" and op["mat"] == "C"]
    assert len(c_loads) == 4 and all(op["row0"] == op["col0"] for op in c_loads)


def test_transb_panels_are_rows_of_the_stored_transpose():
    plan = ooc.make_plan(10, 18, 24, ooc.ORDER_COLS, 2, 1, 2, 3)
    ops, _ = ooc.ooc_schedule(40, 36, 24, 1.0, 0.0, plan, transb=True)
    for op in ops:
        if op["kind"] == "h2d" and op["mat"] == "B":
            assert op["cols"] == 24 and op["rows"] in (18,) and op["dev_ld"] == 24
        if op["kind"] == "gemm":
            assert op["ldb"] == op["k"]


def test_lower_rejects_split_precision():
    A = np.zeros((8, 8)); C = np.zeros((8, 8))
    st, _ = ooc.ooc_gemm_ex(1.0, A, A, 0.0, C, 1 << 20, transb=True, lower=True,
                            opts=ooc.make_opts(precision=ooc.SPLIT_BF16, slices=5), raise_on_error=False)
    assert st == ooc.OOC_ERR_ARG
