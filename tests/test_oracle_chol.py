"""Pins of the Cholesky and rank-k-update references (oracle/chol_ref.py)
against results the mathematics fixes: exact factors of integer SPD matrices,
closed forms, the breakdown column of indefinite matrices, the backward-error
bound, and brute force on tiny inputs."""
import numpy as np
import pytest

from oracle import chol_ref


def _int_factor(n, seed, lo=-3, hi=3, dmax=4):
    """A random integer lower-triangular L with positive diagonal."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(lo, hi + 1, (n, n)).astype(np.float64), -1)
    L[np.arange(n), np.arange(n)] = rng.integers(1, dmax + 1, n)
    return L


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (40, 3), (123, 4)])
def test_integer_factor_recovered_exactly(n, seed):
    # A = L L^T has integer entries below 2^53; every pivot is the square of
    # an integer and every quotient divides exactly, so the factor comes back
    # bit for bit (a transposed operand, a wrong index or sign breaks this)
    L = _int_factor(n, seed)
    A = L @ L.T
    assert np.array_equal(chol_ref.potrf_lower(A), L)


def test_upper_triangle_is_not_read():
    L = _int_factor(9, 5)
    A = L @ L.T
    A[np.triu_indices(9, 1)] = np.nan
    assert np.array_equal(chol_ref.potrf_lower(A), L)


def test_identity_and_diagonal():
    assert np.array_equal(chol_ref.potrf_lower(np.eye(5)), np.eye(5))
    d = np.array([4.0, 9.0, 2.0, 0.25, 1e-6])
    assert np.array_equal(chol_ref.potrf_lower(np.diag(d)), np.diag(np.sqrt(d)))


def test_tridiagonal_laplacian_closed_form():
    # tridiag(-1, 2, -1): pivots (k+1)/k (1-based), so l_kk = sqrt((k+1)/k)
    # and l_{k+1,k} = -sqrt(k/(k+1))
    n = 30
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    L = chol_ref.potrf_lower(A)
    k = np.arange(1, n + 1, dtype=np.float64)
    assert np.allclose(np.diag(L), np.sqrt((k + 1) / k), rtol=1e-15, atol=0)
    assert np.allclose(np.diag(L, -1), -np.sqrt(k[:-1] / (k[:-1] + 1)), rtol=1e-15, atol=0)
    assert np.all(np.tril(L, -2) == 0.0)


def test_two_by_two_by_hand():
    A = np.array([[4.0, 6.0], [6.0, 25.0]])
    # l11 = 2, l21 = 6/2 = 3, l22 = sqrt(25 - 9) = 4
    assert np.array_equal(chol_ref.potrf_lower(A), np.array([[2.0, 0.0], [3.0, 4.0]]))


@pytest.mark.parametrize("col", [0, 3, 6])
def test_breakdown_column(col):
    L = _int_factor(8, 7)
    A = L @ L.T
    # make pivot `col` zero: subtract its value from the diagonal entry
    A[col, col] -= L[col, col] ** 2
    with pytest.raises(chol_ref.NotPositiveDefinite) as ei:
        chol_ref.potrf_lower(A)
    assert ei.value.column == col


def test_backward_error_bound_random_spd():
    rng = np.random.default_rng(11)
    n = 200
    G = rng.standard_normal((n, n))
    A = G @ G.T / n + np.eye(n)
    L = chol_ref.potrf_lower(A)
    R = np.abs(A - L @ L.T)
    # L @ L.T itself rounds; the bound of Theorem 10.3 has room for it at this n
    assert np.all(R <= 2.0 * chol_ref.backward_bound(L))
    # and it is not vacuous: a perturbed factor fails it
    Lb = L.copy()
    Lb[n // 2, n // 3] += 1e-9
    assert not np.all(np.abs(A - Lb @ Lb.T) <= 2.0 * chol_ref.backward_bound(Lb))


def test_syrk_brute_force_and_triangles():
    rng = np.random.default_rng(3)
    n, k = 6, 5
    A = rng.integers(-4, 5, (n, k)).astype(np.float64)
    C = rng.integers(-9, 10, (n, n)).astype(np.float64)
    got = chol_ref.syrk_lower(1.5, A, -2.0, C)
    for i in range(n):
        for j in range(n):
            if i >= j:
                s = 0.0
                for kk in range(k):
                    s += A[i, kk] * A[j, kk]
                assert got[i, j] == 1.5 * s - 2.0 * C[i, j]
            else:
                assert got[i, j] == C[i, j]


def test_syrk_beta_zero_ignores_lower_c():
    A = np.arange(12, dtype=np.float64).reshape(4, 3)
    C = np.full((4, 4), np.nan)
    got = chol_ref.syrk_lower(1.0, A, 0.0, C)
    low = np.tril(np.ones((4, 4), dtype=bool))
    assert np.array_equal(got[low], (A @ A.T)[low])
    assert np.all(np.isnan(got[~low]))


def test_factor_of_syrk_result():
    # potrf(syrk(I-shifted)) round trip on integers: A = L L^T built by syrk
    L = _int_factor(17, 9)
    A = chol_ref.syrk_lower(1.0, L, 0.0, np.zeros((17, 17)))
    A = np.tril(A) + np.tril(A, -1).T
    assert np.array_equal(chol_ref.potrf_lower(A), L)


# ---- triangular solve Y L^T = X (trsm_rlt) ---------------------------------------------

@pytest.mark.parametrize("m,n,seed", [(1, 1, 0), (5, 3, 1), (40, 17, 2), (7, 90, 3)])
def test_trsm_integer_solution_recovered_exactly(m, n, seed):
    # X = Y L^T with integer Y and an integer L whose diagonal divides every
    # numerator exactly: every step of forward substitution is an exact integer
    L = _int_factor(n, seed + 20, dmax=5)
    Y = np.random.default_rng(seed).integers(-9, 10, (m, n)).astype(np.float64)
    X = Y @ L.T
    assert np.array_equal(chol_ref.trsm_rlt(L, X), Y)


def test_trsm_identity_diagonal_and_upper_not_read():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((6, 4))
    assert np.array_equal(chol_ref.trsm_rlt(np.eye(4), X), X)
    d = np.array([2.0, -0.5, 4.0, 8.0])
    assert np.array_equal(chol_ref.trsm_rlt(np.diag(d), X), X / d)
    L = np.tril(rng.standard_normal((4, 4))) + 4 * np.eye(4)
    Lu = L + np.triu(np.full((4, 4), np.nan), 1)
    assert np.array_equal(chol_ref.trsm_rlt(Lu, X), chol_ref.trsm_rlt(L, X))


def test_trsm_two_by_two_by_hand():
    # y1 = x1 / 2; y2 = (x2 - 3 y1) / 4
    L = np.array([[2.0, 0.0], [3.0, 4.0]])
    X = np.array([[4.0, 10.0], [-2.0, 1.0]])
    assert np.array_equal(chol_ref.trsm_rlt(L, X), np.array([[2.0, 1.0], [-1.0, 1.0]]))


def test_trsm_against_library_solve_and_backward_bound():
    rng = np.random.default_rng(9)
    n, m = 60, 25
    L = np.tril(rng.standard_normal((n, n))) + n ** 0.5 * np.eye(n)
    X = rng.standard_normal((m, n))
    Y = chol_ref.trsm_rlt(L, X)
    # Y L^T = X is L Y^T = X^T: a lower-triangular system per row of X
    np.testing.assert_allclose(Y, np.linalg.solve(L, X.T).T, rtol=1e-12, atol=1e-13)
    R = np.abs(X - Y @ L.T)
    assert np.all(R <= 2.0 * chol_ref.trsm_bound(L, Y))
    # and the bound is not vacuous: a perturbed solution fails it
    Yb = Y.copy()
    Yb[3, 7] += 1e-9
    assert not np.all(np.abs(X - Yb @ L.T) <= 2.0 * chol_ref.trsm_bound(L, Yb))


# ---- back substitution Y L = X (trsm_rln) and the Cholesky solve (potrs) ----------------

@pytest.mark.parametrize("m,n,seed", [(1, 1, 0), (5, 3, 1), (40, 17, 2), (7, 90, 3)])
def test_trsm_rln_integer_solution_recovered_exactly(m, n, seed):
    L = _int_factor(n, seed + 40, dmax=5)
    Y = np.random.default_rng(seed + 7).integers(-9, 10, (m, n)).astype(np.float64)
    X = Y @ L
    assert np.array_equal(chol_ref.trsm_rln(L, X), Y)


def test_trsm_rln_two_by_two_by_hand_and_upper_not_read():
    # Y L = X with L = [[2, 0], [3, 4]]: y2 = x2 / 4; y1 = (x1 - 3 y2) / 2
    L = np.array([[2.0, np.nan], [3.0, 4.0]])
    X = np.array([[7.0, 4.0], [1.0, -8.0]])
    assert np.array_equal(chol_ref.trsm_rln(L, X), np.array([[2.0, 1.0], [3.5, -2.0]]))
    d = np.array([2.0, -0.5, 4.0])
    Xr = np.random.default_rng(1).standard_normal((4, 3))
    assert np.array_equal(chol_ref.trsm_rln(np.diag(d), Xr), Xr / d)


def test_trsm_rln_against_library_solve():
    rng = np.random.default_rng(19)
    n, m = 60, 25
    L = np.tril(rng.standard_normal((n, n))) + n ** 0.5 * np.eye(n)
    X = rng.standard_normal((m, n))
    Y = chol_ref.trsm_rln(L, X)
    # Y L = X is L^T Y^T = X^T
    np.testing.assert_allclose(Y, np.linalg.solve(L.T, X.T).T, rtol=1e-12, atol=1e-13)
    # back substitution's backward error (Higham, Theorem 8.5): |X - Y L| <= gamma_n |Y| |L|
    gamma = n * chol_ref.U_FP64 / (1.0 - n * chol_ref.U_FP64)
    assert np.all(np.abs(X - Y @ L) <= 2.0 * gamma * (np.abs(Y) @ np.abs(L)))


def test_potrs_integer_and_against_library_solve():
    # A = L L^T with integer L and integer X: B = X A is solved exactly
    n, m = 30, 6
    L = _int_factor(n, 44)
    X = np.random.default_rng(2).integers(-5, 6, (m, n)).astype(np.float64)
    assert np.array_equal(chol_ref.potrs(L, X @ (L @ L.T)), X)
    rng = np.random.default_rng(3)
    G = rng.standard_normal((n, n))
    A = G @ G.T / n + np.eye(n)
    B = rng.standard_normal((m, n))
    Xs = chol_ref.potrs(chol_ref.potrf_lower(A), B)
    np.testing.assert_allclose(Xs, np.linalg.solve(A, B.T).T, rtol=1e-10, atol=1e-12)
