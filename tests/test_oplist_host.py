"""Host checks of the general executor's interface (ooc_run_ops,
ooc_check_ops): the C++ ordering check agrees with the CPU schedule checker
on the product's own operation lists and on lists with waits removed, and
malformed lists are refused before any device work (OOC_ERR_ARG), while a
well-formed one gets as far as the device (no GPU here: OOC_ERR_NO_DEVICE)."""
import random

import numpy as np
import pytest

from oracle import sched_ref
import paper_1808_05056_amd as ooc

from test_abi_host import PLANS


def _to_ops(M, N, K, beta, plan, transb=False, lower=False):
    """The product's operation list as ooc_op records (and as dicts)."""
    n = ooc.i64()
    ab = ooc.u64()
    tb, lo = int(transb), int(lower)
    ooc._lib.ooc_schedule_ex(tb, lo, M, N, K, 1.0, beta, plan, None, 0, n, ab)
    arr = (ooc.ooc_op * n.value)()
    assert ooc._lib.ooc_schedule_ex(tb, lo, M, N, K, 1.0, beta, plan, arr, n.value, n, ab) == ooc.OOC_OK
    return list(arr), ooc._ops_as_dicts(arr, n.value), ab.value


@pytest.mark.parametrize("case", [0, 2, 4, 6, 7, 11])
def test_check_ops_agrees_with_the_cpu_checker(case):
    M, N, K, plan = PLANS[case]
    recs, dicts, _ = _to_ops(M, N, K, 0.5, plan, transb=case % 2 == 0, lower=case == 4)
    st, x, y = ooc.ooc_check_ops(recs)
    assert st == ooc.OOC_OK and sched_ref.check_hazards(dicts) == []
    rng = random.Random(case)
    found = 0
    for trial in range(12):
        # remove one wait at random: both checkers must agree on whether that opens a race
        cand = [i for i, o in enumerate(recs) if o.nwait > 0]
        i = rng.choice(cand)
        r2 = [ooc.ooc_op.from_buffer_copy(o) for o in recs]
        k = rng.randrange(r2[i].nwait)
        w = list(r2[i].wait)[:r2[i].nwait]
        del w[k]
        r2[i].nwait = len(w)
        for q, v in enumerate(w):
            r2[i].wait[q] = v
        d2 = [dict(d) for d in dicts]
        d2[i]["waits"] = w
        st, x, y = ooc.ooc_check_ops(r2)
        bad = sched_ref.check_hazards(d2)
        assert (st == ooc.OOC_OK) == (bad == []), (i, bad[:3], x, y)
        if st != ooc.OOC_OK:
            assert (x, y) in bad
            found += 1
    assert found > 0  # the mutations do open races the checker sees


def _gemm_list():
    # A (4 x 3) and B (3 x 5) to the arena, C = A B on stream 1, C home on stream 2
    h_a = ooc.make_op("h2d", 0, mat=0, rows=4, cols=3, off_c=0, ld_c=3)
    h_b = ooc.make_op("h2d", 0, mat=1, rows=3, cols=5, off_c=12, ld_c=5)
    g = ooc.make_op("gemm", 1, waits=[0, 1], rows=4, cols=5, k=3, off_a=0, ld_a=3, off_b=12, ld_b=5, off_c=27,
                    ld_c=5, alpha=1.0, beta=0.0)
    d = ooc.make_op("d2h", 2, waits=[2], mat=2, rows=4, cols=5, off_c=27, ld_c=5)
    return [h_a, h_b, g, d]


def _mats():
    return [np.zeros((4, 3)), np.zeros((3, 5)), np.zeros((4, 5))]


ARENA = (27 + 20) * 8


def test_run_ops_accepts_a_wellformed_list_up_to_the_device():
    st, _ = ooc.ooc_run_ops(_gemm_list(), _mats(), ARENA, raise_on_error=False)
    assert st in (ooc.OOC_ERR_NO_DEVICE, ooc.OOC_ERR_NOT_PINNED)
    assert ooc.ooc_check_ops(_gemm_list())[0] == ooc.OOC_OK


@pytest.mark.parametrize("mutation", ["copy_outside_host", "operand_outside_arena", "wait_on_later_op",
                                      "bad_stream", "unknown_kind", "lda_too_small", "bad_mat_index",
                                      "split_without_precision", "unknown_flag"])
def test_run_ops_refuses_malformed_lists(mutation):
    ops = _gemm_list()
    arena = ARENA
    if mutation == "copy_outside_host":
        ops[0].row0 = 1  # rows 1..4 of a 4-row matrix
    elif mutation == "operand_outside_arena":
        arena = ARENA - 8  # the last element of C falls outside
    elif mutation == "wait_on_later_op":
        ops[2].wait[0] = 3
    elif mutation == "bad_stream":
        ops[3].stream = 3
    elif mutation == "unknown_kind":
        ops[1].kind = 9
    elif mutation == "lda_too_small":
        ops[2].ld_a = 2
    elif mutation == "bad_mat_index":
        ops[3].mat = 3
    elif mutation == "split_without_precision":
        ops[2].kind = ooc.OP_SPLIT_GEMM
    elif mutation == "unknown_flag":
        ops[2].flags = 4
    st, _ = ooc.ooc_run_ops(ops, _mats(), arena, raise_on_error=False)
    assert st == ooc.OOC_ERR_ARG, ooc.ooc_last_error()


def test_check_ops_finds_a_missing_wait():
    ops = _gemm_list()
    ops[3].nwait = 0  # C home before the product wrote it
    st, x, y = ooc.ooc_check_ops(ops)
    assert st == ooc.OOC_ERR_ARG and (x, y) == (3, 2)


def test_potrf_and_syrk_argument_checks_on_the_host():
    A = np.zeros((8, 8))
    # a budget that holds no 64-column panel
    st, info, _ = ooc.ooc_potrf(A, 1024, raise_on_error=False)
    assert st == ooc.OOC_ERR_BUDGET


def test_solve_argument_checks_on_the_host():
    L, X = np.zeros((8, 8)), np.zeros((5, 8))
    assert ooc.ooc_trsm_ex(L, X, 1 << 20, trans=2, raise_on_error=False)[0] == ooc.OOC_ERR_ARG
    for trans in (0, 1):
        assert ooc.ooc_trsm_ex(L, X, 1024, trans=trans, raise_on_error=False)[0] == ooc.OOC_ERR_BUDGET
    assert ooc.ooc_potrs(L, X, 1024, raise_on_error=False)[0] == ooc.OOC_ERR_BUDGET
    with pytest.raises(ValueError):
        ooc.ooc_potrs(L, np.zeros((5, 7)), 1 << 20)


def _trsm_op(flags):
    # a 4 x 3 block solved against the 3 x 3 triangle at arena offset 0
    h_l = ooc.make_op("h2d", 0, mat=0, rows=3, cols=3, off_c=0, ld_c=3)
    h_x = ooc.make_op("h2d", 0, mat=1, rows=4, cols=3, off_c=9, ld_c=3)
    t = ooc.make_op("trsm", 1, waits=[0, 1], rows=4, cols=3, off_c=9, ld_c=3, off_a=0, ld_a=3, flags=flags)
    d = ooc.make_op("d2h", 2, waits=[2], mat=1, rows=4, cols=3, off_c=9, ld_c=3)
    return [h_l, h_x, t, d]


@pytest.mark.parametrize("flags,ok", [(0, True), (ooc.OPF_BACK, True), (ooc.OPF_TRANSB, False),
                                      (ooc.OPF_LOWER, False), (ooc.OPF_BACK | 8, False)])
def test_trsm_op_flags(flags, ok):
    ops = _trsm_op(flags)
    st, _ = ooc.ooc_run_ops(ops, [np.zeros((3, 3)), np.zeros((4, 3))], 21 * 8, raise_on_error=False)
    if ok:
        assert st in (ooc.OOC_ERR_NO_DEVICE, ooc.OOC_ERR_NOT_PINNED)
        assert ooc.ooc_check_ops(ops)[0] == ooc.OOC_OK
    else:
        assert st == ooc.OOC_ERR_ARG, ooc.ooc_last_error()


def _split_pair(first_flags=0, second_flags=ooc.OPF_REUSE_A | ooc.OPF_REUSE_B, second=None):
    # A (4 x 3) at 0, its copy at 12, B (3 x 5) at 24, C (4 x 5) at 39, the
    # slice workspace after it; two split products on the same panels
    W = 45376  # workspace elements for 4 x 5 x 3 at s = 2 (BF16 planes padded to 256 x 128 x 64)
    ops = [ooc.make_op("h2d", 0, mat=0, rows=4, cols=3, off_c=0, ld_c=3),
           ooc.make_op("h2d", 0, mat=0, rows=4, cols=3, off_c=12, ld_c=3),
           ooc.make_op("h2d", 0, mat=1, rows=3, cols=5, off_c=24, ld_c=5)]
    prod = dict(rows=4, cols=5, k=3, off_a=0, ld_a=3, off_b=24, ld_b=5, off_c=39, ld_c=5, alpha=1.0, beta=0.0,
                off_w=59, len_w=W)
    ops.append(ooc.make_op("split_gemm", 1, waits=[0, 1, 2], flags=first_flags, **prod))
    prod2 = dict(prod, beta=1.0, flags=second_flags)
    prod2.update(second or {})
    ops.append(ooc.make_op("split_gemm", 1, **prod2))
    ops.append(ooc.make_op("d2h", 2, waits=[4], mat=2, rows=4, cols=5, off_c=39, ld_c=5))
    return ops, (59 + W) * 8


@pytest.mark.parametrize("case,ok", [("reuse_both", True), ("reuse_a", True), ("first_op", False),
                                     ("other_a_panel", False), ("other_k", False), ("fp64_flag", False)])
def test_split_slice_reuse_flags(case, ok):
    mats = [np.zeros((4, 3)), np.zeros((3, 5)), np.zeros((4, 5))]
    if case == "reuse_both":
        ops, arena = _split_pair()
    elif case == "reuse_a":
        ops, arena = _split_pair(second_flags=ooc.OPF_REUSE_A)
    elif case == "first_op":
        ops, arena = _split_pair(first_flags=ooc.OPF_REUSE_A)
    elif case == "other_a_panel":  # the same values, but another panel of the arena
        ops, arena = _split_pair(second_flags=ooc.OPF_REUSE_A, second=dict(off_a=12))
    elif case == "other_k":
        ops, arena = _split_pair(second=dict(k=2))
    else:
        ops, arena = _split_pair()
        ops[4].kind = ooc.OP_GEMM
    opts = ooc.make_opts(precision=ooc.SPLIT_BF16, slices=2)
    st, _ = ooc.ooc_run_ops(ops, mats, arena, opts=opts, raise_on_error=False)
    if ok:
        assert st in (ooc.OOC_ERR_NO_DEVICE, ooc.OOC_ERR_NOT_PINNED), ooc.ooc_last_error()
    else:
        assert st == ooc.OOC_ERR_ARG, ooc.ooc_last_error()
