"""GPU parity of the out-of-core level-3 routines built on the pipeline
(transposed-B and lower-triangle products, the rank-k update, the Cholesky
factorisation) and of the general executor, against the oracle: bit-exact
where every intermediate value is an integer, within the normalised gate or
the backward-error bound otherwise.  Budgets are small so that every call
runs several blocks, panels and chunks."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import chol_ref
import paper_1808_05056_amd as ooc

pytestmark = pytest.mark.gpu
MiB = 1 << 20


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pinned(X):
    P = ooc.PinnedMatrix(X.shape[0], X.shape[1])
    P.array[...] = X
    return P


def _int_factor(n, seed):
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(-3, 4, (n, n)).astype(np.float64), -1)
    L[np.arange(n), np.arange(n)] = rng.integers(1, 5, n)
    return L


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    return G @ G.T / n + np.eye(n)


# ---- transposed-B and lower-triangle products --------------------------------------

GEMM_EX = [
    # M, N, K, transb, lower, beta, budget, integer inputs
    (700, 650, 900, True, False, 0.5, 2 * MiB, True),
    (700, 650, 900, True, True, 0.5, 2 * MiB, True),
    (640, 640, 300, False, True, 0.0, 1 * MiB, False),
    (513, 777, 1025, True, True, -1.0, 3 * MiB, False),
]


@pytest.mark.parametrize("case", range(len(GEMM_EX)))
def test_gemm_ex_against_the_oracle(case):
    M, N, K, transb, lower, beta, budget, integer = GEMM_EX[case]
    _say(f"gemm_ex case {GEMM_EX[case]}")
    dist = synth.INT if integer else synth.NORMAL
    A = synth.matrix(M, K, synth.spec(900 + case, 0, dist))
    Bs = synth.matrix(N, K, synth.spec(900 + case, 1, dist)) if transb else synth.matrix(K, N, synth.spec(900 + case, 1, dist))
    C0 = synth.matrix(M, N, synth.spec(900 + case, 2, dist))
    up = np.triu(np.ones((M, N), dtype=bool), 1)
    if lower:
        C0[up] = np.nan  # above the diagonal: neither read nor changed
    Pa, Pb, Pc = _pinned(A), _pinned(Bs), _pinned(C0)
    try:
        _, st = ooc.ooc_gemm_ex(1.25, Pa.array, Pb.array, beta, Pc.array, budget, transb=transb, lower=lower)
        got = Pc.array.copy()
        B = np.ascontiguousarray(Bs.T) if transb else Bs
        Cin = np.where(up, 0.0, C0) if lower else C0
        ref, D = oracle.gemm_rows(1.25, A, B, beta, Cin if beta != 0.0 else None)
        keep = ~up if lower else np.ones((M, N), dtype=bool)
        if integer:
            assert np.array_equal(got[keep], ref[keep])
        else:
            lit, gen = oracle.errors(np.where(keep, got, ref), ref, 1.25, D, beta, Cin if beta != 0.0 else None)
            _say(f"  error literal {lit:.3e} generalised {gen:.3e}; plan {st.plan}")
            assert gen <= oracle.GATE
        if lower:
            assert np.all(np.isnan(got[up]))
        assert st.arena_bytes <= budget
    finally:
        for P in (Pa, Pb, Pc):
            P.free()
        ooc.ooc_release(-1)


def test_syrk_against_the_oracle():
    N, K = 900, 700
    A = synth.matrix(N, K, synth.spec(77, 0, synth.INT))
    C0 = synth.matrix(N, N, synth.spec(77, 2, synth.INT))
    C0[np.triu_indices(N, 1)] = np.nan
    Pa, Pc = _pinned(A), _pinned(C0)
    try:
        _, st = ooc.ooc_syrk(-0.5, Pa.array, 2.0, Pc.array, 2 * MiB)
        want = chol_ref.syrk_lower(-0.5, A, 2.0, C0)
        assert np.array_equal(Pc.array, want, equal_nan=True)
        _say(f"syrk: plan {st.plan} ops {st.ops} arena {st.arena_bytes}")
    finally:
        Pa.free(); Pc.free()
        ooc.ooc_release(-1)


# ---- Cholesky factorisation --------------------------------------------------------

@pytest.mark.parametrize("n,budget", [(37, 1 * MiB), (700, 2 * MiB), (1500, 3 * MiB)])
def test_potrf_integer_factor_exact(n, budget):
    L = _int_factor(n, n)
    A = L @ L.T
    A[np.triu_indices(n, 1)] = np.nan  # never read, left as it was
    P = _pinned(A)
    try:
        _, info, st = ooc.ooc_potrf(P.array, budget)
        _say(f"potrf n={n}: panels {st.blocks_done} ops {st.ops} arena {st.arena_bytes} t {st.t_total_s * 1e3:.1f} ms")
        got = P.array
        assert info == 0
        assert np.array_equal(np.tril(got), L)
        assert np.all(np.isnan(got[np.triu_indices(n, 1)]))
        assert st.arena_bytes <= budget
    finally:
        P.free()
        ooc.ooc_release(-1)


def test_potrf_random_spd_against_the_oracle():
    n = 2000
    A = _spd(n, 5)
    P = _pinned(A)
    try:
        _, info, st = ooc.ooc_potrf(P.array, 4 * MiB)
        L = np.tril(P.array)
        Lref = chol_ref.potrf_lower(A)
        fwd = np.max(np.abs(L - Lref)) / np.max(np.abs(Lref))
        back = np.abs(A - L @ L.T)
        bound = 2.0 * chol_ref.backward_bound(L)
        _say(f"potrf n={n}: forward {fwd:.3e}, backward worst ratio {np.max(back / bound):.3e}, panels {st.blocks_done}")
        assert info == 0
        assert fwd <= 1e-12
        assert np.all(back <= bound)
    finally:
        P.free()
        ooc.ooc_release(-1)


@pytest.mark.parametrize("col", [0, 333, 699])
def test_potrf_reports_the_failing_pivot(col):
    n = 700
    L = _int_factor(n, 3)
    A = L @ L.T
    A[col, col] -= L[col, col] ** 2  # pivot col becomes 0
    P = _pinned(A)
    try:
        st, info, _ = ooc.ooc_potrf(P.array, 2 * MiB, raise_on_error=False)
        assert st == ooc.OOC_ERR_NOT_SPD and info == col + 1
        # the block columns before the failing one hold L
        b = 256
        done = (col // b) * b
        assert np.array_equal(np.tril(P.array)[:, :done], L[:, :done])
    finally:
        P.free()
        ooc.ooc_release(-1)


def test_potrf_large_sampled_rows():
    # 12288^2 (1.1 GiB) through a 256 MiB budget: several panels, chunked solves,
    # out-of-core updates; checked on sampled rows by the backward-error bound
    n = 12288
    G = synth.matrix(n, 64, synth.spec(4242, 0, synth.UNIFORM))
    P = ooc.PinnedMatrix(n, n)
    try:
        A = P.array
        A[...] = G @ G.T / 64.0
        A[np.arange(n), np.arange(n)] += 2.0
        diag = A.diagonal().copy()
        rows = np.array([0, 1, 4095, 4096, 8191, 8192, 12287] + list(np.random.default_rng(1).integers(0, n, 9)))
        Arows = A[rows].copy()
        _, info, st = ooc.ooc_potrf(A, 256 * MiB)
        _say(f"potrf n={n}: {st.flops / st.t_total_s / 1e12:.2f} TFLOP/s, {st.t_total_s:.3f} s, panels "
             f"{st.blocks_done}, H2D {st.bytes_h2d / 1e9:.2f} GB, planning {st.t_plan_s * 1e3:.1f} ms")
        assert info == 0
        Lf = np.tril(A)
        aL = np.abs(Lf)
        gamma = (n + 1) * 2.0 ** -53 / (1 - (n + 1) * 2.0 ** -53)
        for r, arow in zip(rows, Arows):
            # (L L^T)[r, :r+1] = L[:r+1, :] @ L[r, :], against the bound of the backward error
            prod = Lf[:r + 1, :r + 1] @ Lf[r, :r + 1]
            bnd = 2.0 * gamma * (aL[:r + 1, :r + 1] @ aL[r, :r + 1])
            assert np.all(np.abs(arow[:r + 1] - prod) <= bnd), r
        assert np.all(np.diagonal(A) > 0)
    finally:
        P.free()
        ooc.ooc_release(-1)


# ---- out-of-core triangular solve Y L^T = X -----------------------------------------

@pytest.mark.parametrize("m,n,budget", [(37, 29, 1 * MiB), (700, 500, 2 * MiB), (3000, 200, 1 * MiB),
                                        (1500, 1300, 3 * MiB)])
def test_trsm_integer_solution_exact(m, n, budget):
    # X = Y L^T with integer Y and L: every quotient of the solve is exact, and
    # L's strict upper triangle (NaN) is never read
    L = _int_factor(n, n + 1)
    Y = np.random.default_rng(m).integers(-9, 10, (m, n)).astype(np.float64)
    X = Y @ L.T
    Lh = L.copy()
    Lh[np.triu_indices(n, 1)] = np.nan
    PL, PX = _pinned(Lh), _pinned(X)
    try:
        _, st = ooc.ooc_trsm(PL.array, PX.array, budget)
        _say(f"trsm m={m} n={n}: panels {st.blocks_done} ops {st.ops} arena {st.arena_bytes} "
             f"t {st.t_total_s * 1e3:.1f} ms")
        assert np.array_equal(PX.array, Y)
        assert st.arena_bytes <= budget
        assert np.array_equal(np.isnan(PL.array), np.isnan(Lh))  # L left as it was
    finally:
        PL.free()
        PX.free()
        ooc.ooc_release(-1)


def test_trsm_random_against_the_oracle():
    m, n = 2000, 1500
    rng = np.random.default_rng(17)
    L = np.tril(rng.standard_normal((n, n))) + n ** 0.5 * np.eye(n)
    X = rng.standard_normal((m, n))
    PL, PX = _pinned(L), _pinned(X)
    try:
        _, st = ooc.ooc_trsm(PL.array, PX.array, 4 * MiB)
        Y = PX.array.copy()
        Yref = chol_ref.trsm_rlt(L, X)
        fwd = np.max(np.abs(Y - Yref)) / np.max(np.abs(Yref))
        back = np.abs(X - Y @ L.T)
        bound = 2.0 * chol_ref.trsm_bound(L, Y)
        _say(f"trsm m={m} n={n}: forward {fwd:.3e}, backward worst ratio {np.max(back / bound):.3e}, "
             f"panels {st.blocks_done}")
        assert fwd <= 1e-12
        assert np.all(back <= bound)
    finally:
        PL.free()
        PX.free()
        ooc.ooc_release(-1)


def test_trsm_large_sampled_rows_and_degenerate_calls():
    # 16384 x 8192 right-hand sides (1 GiB) against an 8192^2 factor through a
    # 256 MiB budget; the rows of the solve are independent, so the oracle
    # solves the sampled rows alone
    m, n = 16384, 8192
    rng = np.random.default_rng(23)
    PL, PX = ooc.PinnedMatrix(n, n), ooc.PinnedMatrix(m, n)
    try:
        L = PL.array
        # off-diagonal entries in [-1/n, 1/n] under a diagonal in [1, 2]: diagonally
        # dominant, so the solve is well conditioned
        L[...] = np.tril(synth.matrix(n, n, synth.spec(4343, 0, synth.UNIFORM))) / n
        L[np.arange(n), np.arange(n)] = 1.0 + n * np.abs(L.diagonal())
        X = PX.array
        X[...] = synth.matrix(m, n, synth.spec(4343, 1, synth.UNIFORM))
        rows = np.unique(np.concatenate([[0, m - 1], rng.integers(0, m, 30)]))
        Xrows = X[rows].copy()
        _, st = ooc.ooc_trsm(L, X, 256 * MiB)
        _say(f"trsm m={m} n={n}: {st.flops / st.t_total_s / 1e12:.2f} TFLOP/s, {st.t_total_s:.3f} s, panels "
             f"{st.blocks_done}, H2D {st.bytes_h2d / 1e9:.2f} GB, planning {st.t_plan_s * 1e3:.1f} ms")
        Yref = chol_ref.trsm_rlt(L, Xrows)
        fwd = np.max(np.abs(X[rows] - Yref)) / np.max(np.abs(Yref))
        assert fwd <= 1e-12, fwd
        # degenerate calls: no rows, no columns, and a budget without a 64-column panel
        empty = ooc.PinnedMatrix(1, n)
        try:
            assert ooc.ooc_trsm(L, empty.array[:0], 256 * MiB)[0] == ooc.OOC_OK
        finally:
            empty.free()
        assert ooc.ooc_trsm(L[:0, :0], X[:, :0], 256 * MiB)[0] == ooc.OOC_OK
        assert ooc.ooc_trsm(L, X, 64 * 1024, raise_on_error=False)[0] == ooc.OOC_ERR_BUDGET
    finally:
        PL.free()
        PX.free()
        ooc.ooc_release(-1)


# ---- back substitution Y L = X and the Cholesky solve --------------------------------

@pytest.mark.parametrize("m,n,budget", [(37, 29, 1 * MiB), (700, 500, 2 * MiB), (3000, 200, 1 * MiB),
                                        (1500, 1300, 3 * MiB)])
def test_trsm_back_integer_solution_exact(m, n, budget):
    # X = Y L with integer Y and L: every quotient of the back substitution is
    # exact; L's strict upper triangle (NaN) is never read
    L = _int_factor(n, n + 2)
    Y = np.random.default_rng(m + 1).integers(-9, 10, (m, n)).astype(np.float64)
    X = Y @ L
    Lh = L.copy()
    Lh[np.triu_indices(n, 1)] = np.nan
    PL, PX = _pinned(Lh), _pinned(X)
    try:
        _, st = ooc.ooc_trsm_ex(PL.array, PX.array, budget, trans=0)
        _say(f"trsm back m={m} n={n}: panels {st.blocks_done} ops {st.ops} arena {st.arena_bytes} "
             f"t {st.t_total_s * 1e3:.1f} ms")
        assert np.array_equal(PX.array, Y)
        assert st.arena_bytes <= budget
        # trans=1 is ooc_trsm: the same L solves Y L^T = X exactly too
        PX.array[...] = Y @ L.T
        ooc.ooc_trsm_ex(PL.array, PX.array, budget, trans=1)
        assert np.array_equal(PX.array, Y)
    finally:
        PL.free()
        PX.free()
        ooc.ooc_release(-1)


@pytest.mark.parametrize("m", [1, 15, 17])
def test_solves_with_few_right_hand_sides_exact(m):
    # fewer rows than one solve-leaf wave holds (16), and one more: both
    # triangular forms and the Cholesky solve stay exact on integer data
    n = 300
    L = _int_factor(n, 77)
    Y = np.random.default_rng(m + 5).integers(-9, 10, (m, n)).astype(np.float64)
    PL = _pinned(L)
    PX = _pinned(Y @ L.T)
    try:
        ooc.ooc_trsm_ex(PL.array, PX.array, 1 * MiB, trans=1)
        assert np.array_equal(PX.array, Y)
        PX.array[...] = Y @ L
        ooc.ooc_trsm_ex(PL.array, PX.array, 1 * MiB, trans=0)
        assert np.array_equal(PX.array, Y)
        PX.array[...] = Y @ (L @ L.T)
        _, st = ooc.ooc_potrs(PL.array, PX.array, 1 * MiB)
        _say(f"solves with {m} right-hand sides of {n}: panels {st.blocks_done}")
        assert np.array_equal(PX.array, Y)
    finally:
        PL.free()
        PX.free()
        ooc.ooc_release(-1)


def test_trsm_back_and_potrs_random_against_the_oracle():
    m, n = 1800, 1400
    rng = np.random.default_rng(29)
    L = np.tril(rng.standard_normal((n, n))) + n ** 0.5 * np.eye(n)
    X = rng.standard_normal((m, n))
    PL, PX = _pinned(L), _pinned(X)
    try:
        _, st = ooc.ooc_trsm_ex(PL.array, PX.array, 4 * MiB, trans=0)
        Y = PX.array.copy()
        Yref = chol_ref.trsm_rln(L, X)
        fwd = np.max(np.abs(Y - Yref)) / np.max(np.abs(Yref))
        back = np.abs(X - Y @ L)
        gamma = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)
        bound = 2.0 * gamma * (np.abs(Y) @ np.abs(L))
        _say(f"trsm back m={m} n={n}: forward {fwd:.3e}, backward worst ratio {np.max(back / bound):.3e}, "
             f"panels {st.blocks_done}")
        assert fwd <= 1e-12
        assert np.all(back <= bound)
        # the Cholesky solve: B A^{-1} with A = L L^T
        PX.array[...] = X
        _, st = ooc.ooc_potrs(PL.array, PX.array, 4 * MiB)
        Z = PX.array.copy()
        Zref = chol_ref.potrs(L, X)
        fwd = np.max(np.abs(Z - Zref)) / np.max(np.abs(Zref))
        res = np.max(np.abs(Z @ L @ L.T - X)) / (np.max(np.abs(L)) ** 2 * n * np.max(np.abs(Z)))
        _say(f"potrs m={m} n={n}: forward {fwd:.3e}, normalised residual {res:.3e}, panels {st.blocks_done}")
        assert fwd <= 1e-12
        assert res <= 1e-15
        assert st.blocks_done >= 2
    finally:
        PL.free()
        PX.free()
        ooc.ooc_release(-1)


def test_factor_then_solve_through_the_device():
    # ooc_potrf then ooc_potrs on one SPD matrix: x solves A x = b for each row b
    n, m = 1500, 700
    A = _spd(n, 41)
    B = np.random.default_rng(43).standard_normal((m, n))
    Pa, Pb = _pinned(A), _pinned(B)
    try:
        _, info, _ = ooc.ooc_potrf(Pa.array, 4 * MiB)
        assert info == 0
        _, st = ooc.ooc_potrs(Pa.array, Pb.array, 4 * MiB)
        Xs = Pb.array.copy()
        Xref = np.linalg.solve(A, B.T).T
        err = np.max(np.abs(Xs - Xref)) / np.max(np.abs(Xref))
        cond = np.linalg.cond(A)
        _say(f"potrf + potrs n={n} m={m}: forward {err:.3e} (cond {cond:.1f})")
        assert err <= 50 * cond * n * 2.0 ** -53
    finally:
        Pa.free()
        Pb.free()
        ooc.ooc_release(-1)


def test_potrs_large_sampled_rows():
    # 16384 right-hand sides of an 8192^2 system through a 256 MiB budget; the
    # rows of the solve are independent, so the oracle solves the sampled rows
    m, n = 16384, 8192
    rng = np.random.default_rng(47)
    PL, PX = ooc.PinnedMatrix(n, n), ooc.PinnedMatrix(m, n)
    try:
        L = PL.array
        L[...] = np.tril(synth.matrix(n, n, synth.spec(4747, 0, synth.UNIFORM))) / n
        L[np.arange(n), np.arange(n)] = 1.0 + n * np.abs(L.diagonal())
        X = PX.array
        X[...] = synth.matrix(m, n, synth.spec(4747, 1, synth.UNIFORM))
        rows = np.unique(np.concatenate([[0, m - 1], rng.integers(0, m, 30)]))
        Xrows = X[rows].copy()
        _, st = ooc.ooc_potrs(L, X, 256 * MiB)
        _say(f"potrs m={m} n={n}: {st.flops / st.t_total_s / 1e12:.2f} TFLOP/s, {st.t_total_s:.3f} s, panels "
             f"{st.blocks_done}, H2D {st.bytes_h2d / 1e9:.2f} GB, planning {st.t_plan_s * 1e3:.1f} ms")
        Zref = chol_ref.potrs(L, Xrows)
        fwd = np.max(np.abs(X[rows] - Zref)) / np.max(np.abs(Zref))
        assert fwd <= 1e-12, fwd
        assert ooc.ooc_potrs(L[:0, :0], X[:, :0], 256 * MiB)[0] == ooc.OOC_OK
    finally:
        PL.free()
        PX.free()
        ooc.ooc_release(-1)


# ---- the general executor: hand-built operation lists -------------------------------

def test_run_ops_product_list():
    A = synth.matrix(300, 200, synth.spec(5, 0, synth.INT))
    B = synth.matrix(200, 250, synth.spec(5, 1, synth.INT))
    Pa, Pb, Pc = _pinned(A), _pinned(B), _pinned(np.full((300, 250), np.nan))
    try:
        offb, offc = 300 * 200, 300 * 200 + 200 * 250
        ops = [ooc.make_op("h2d", 0, mat=0, rows=300, cols=200, off_c=0, ld_c=200),
               ooc.make_op("h2d", 0, mat=1, rows=200, cols=250, off_c=offb, ld_c=250),
               ooc.make_op("gemm", 1, waits=[0, 1], rows=300, cols=250, k=200, off_a=0, ld_a=200, off_b=offb,
                           ld_b=250, off_c=offc, ld_c=250, alpha=1.0, beta=0.0),
               ooc.make_op("d2h", 2, waits=[2], mat=2, rows=300, cols=250, off_c=offc, ld_c=250)]
        assert ooc.ooc_check_ops(ops)[0] == ooc.OOC_OK
        ooc.ooc_run_ops(ops, [Pa.array, Pb.array, Pc.array], (offc + 300 * 250) * 8)
        assert np.array_equal(Pc.array, A @ B)
    finally:
        for P in (Pa, Pb, Pc):
            P.free()
        ooc.ooc_release(-1)


def test_run_ops_factor_and_solve_list():
    # a 192-column panel: factor its diagonal block, solve the 500 rows below
    # against it (in two chunks through one buffer), all as one operation list
    n, b = 692, 192
    L = _int_factor(n, 8)
    A = L @ L.T
    Pa = _pinned(A)
    Ps = _pinned(np.zeros((1, 1)))
    try:
        base = b * b + 8
        ops = [ooc.make_op("h2d", 0, mat=0, rows=b, cols=b, off_c=0, ld_c=b),
               ooc.make_op("h2d", 0, mat=1, rows=1, cols=1, off_c=b * b, ld_c=1),
               ooc.make_op("potrf", 1, waits=[0, 1], rows=b, cols=b, off_c=0, ld_c=b, off_w=b * b, len_w=1),
               ooc.make_op("d2h", 2, waits=[2], mat=0, rows=b, cols=b, off_c=0, ld_c=b),
               ooc.make_op("d2h", 2, waits=[2], mat=1, rows=1, cols=1, off_c=b * b, ld_c=1)]
        for q, (r0, rr) in enumerate([(b, 250), (b + 250, 250)]):
            w = [len(ops) - 1] if q else []
            ops.append(ooc.make_op("h2d", 0, waits=w, mat=0, row0=r0, rows=rr, cols=b, off_c=base, ld_c=b))
            ops.append(ooc.make_op("trsm", 1, waits=[len(ops) - 1], rows=rr, cols=b, off_c=base, ld_c=b, off_a=0,
                                   ld_a=b))
            ops.append(ooc.make_op("d2h", 2, waits=[len(ops) - 1], mat=0, row0=r0, rows=rr, cols=b, off_c=base,
                                   ld_c=b))
        st, x, y = ooc.ooc_check_ops(ops)
        assert st == ooc.OOC_OK, (x, y)
        ooc.ooc_run_ops(ops, [Pa.array, Ps.array], (base + 250 * b) * 8)
        assert Ps.array[0, 0] == 0.0
        assert np.array_equal(np.tril(Pa.array[:, :b]), L[:, :b])
    finally:
        Pa.free(); Ps.free()
        ooc.ooc_release(-1)


def test_gemm_ex_transposed_b_split_bf16():
    # op(B) = B^T through the split-BF16 form: the stored B^T is sliced by rows
    M, N, K = 600, 520, 1300
    A = synth.matrix(M, K, synth.spec(321, 0, synth.NORMAL, row_exp=(-10, 10)))
    Bs = synth.matrix(N, K, synth.spec(321, 1, synth.NORMAL, row_exp=(-10, 10)))
    C0 = synth.matrix(M, N, synth.spec(321, 2, synth.UNIFORM))
    Pa, Pb, Pc = _pinned(A), _pinned(Bs), _pinned(C0)
    try:
        _, st = ooc.ooc_gemm_ex(1.0, Pa.array, Pb.array, 0.5, Pc.array, 8 * MiB, transb=True,
                                opts=ooc.make_opts(precision=ooc.SPLIT_BF16, slices=6))
        ref, D = oracle.gemm_rows(1.0, A, np.ascontiguousarray(Bs.T), 0.5, C0)
        lit, gen = oracle.errors(Pc.array, ref, 1.0, D, 0.5, C0)
        _say(f"split transb: error literal {lit:.3e} generalised {gen:.3e}; plan {st.plan}")
        assert st.plan.precision == ooc.SPLIT_BF16
        assert gen <= oracle.GATE
    finally:
        for P in (Pa, Pb, Pc):
            P.free()
        ooc.ooc_release(-1)


def test_gemm_ex_transposed_b_split_int8_wide_tiles():
    # op(B) = B^T through the split-INT8 form at 4096^2 with room for large
    # blocks (a 4096 x 4096 block makes 256 tiles of 256 x 256 against 512 of
    # 256 x 128, so its slice products take the wide tiles); sampled rows
    M, N, K = 4096, 4096, 2000
    A = synth.matrix(M, K, synth.spec(322, 0, synth.NORMAL, row_exp=(-10, 10)))
    Bs = synth.matrix(N, K, synth.spec(322, 1, synth.NORMAL, row_exp=(-10, 10)))
    C0 = synth.matrix(M, N, synth.spec(322, 2, synth.UNIFORM))
    Pa, Pb, Pc = _pinned(A), _pinned(Bs), _pinned(C0)
    try:
        _, st = ooc.ooc_gemm_ex(1.0, Pa.array, Pb.array, 0.5, Pc.array, 1 << 30, transb=True,
                                opts=ooc.make_opts(precision=ooc.SPLIT_INT8, slices=7))
        rows = np.unique(np.concatenate([[0, 255, 256, M - 1], np.random.default_rng(3).integers(0, M, 60)]))
        ref, D = oracle.gemm_rows(1.0, A, np.ascontiguousarray(Bs.T), 0.5, C0[rows], rows=rows)
        lit, gen = oracle.errors(Pc.array[rows], ref, 1.0, D, 0.5, C0[rows])
        _say(f"split-int8 transb: error literal {lit:.3e} generalised {gen:.3e}; plan {st.plan}")
        assert st.plan.precision == ooc.SPLIT_INT8
        assert gen <= oracle.GATE
    finally:
        for P in (Pa, Pb, Pc):
            P.free()
        ooc.ooc_release(-1)
