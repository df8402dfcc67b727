"""Cholesky factorisation and symmetric rank-k update -- TEST INFRASTRUCTURE ONLY.

The paper's closing section names, as the next use of the out-of-core
product, level-3 BLAS routines and dense factorisations whose bulk of work
is the out-of-core product (Section VII, future work).  The out-of-core
Cholesky factorisation and rank-k update built on it are checked against the
plain definitions below: FP64, row-major, no blocking.

potrf_lower(A) -> L        lower-triangular L with positive diagonal and
                            A = L L^T, column by column (Cholesky-Crout):
                              l_jj = sqrt(a_jj - sum_{k<j} l_jk^2)
                              l_ij = (a_ij - sum_{k<j} l_ik l_jk) / l_jj, i > j
                            Only the lower triangle of A is read.  A pivot
                            a_jj - sum l_jk^2 <= 0 (or not finite) raises
                            NotPositiveDefinite(j).
syrk_lower(alpha, A, beta, C) -> C'
                            C'_ij = alpha sum_k A_ik A_jk + beta C_ij for i >= j;
                            the strict upper triangle of C is returned
                            unchanged; with beta == 0 C's lower triangle is not
                            read.
trsm_rlt(L, X) -> Y         Y with Y L^T = X for lower-triangular L (n x n,
                            nonzero diagonal) and X (m x n): column by column
                            (forward substitution on every row at once),
                              y_j = (x_j - sum_{k<j} y_k l_jk) / l_jj.
                            Only the lower triangle of L is read.
trsm_rln(L, X) -> Y         Y with Y L = X (back substitution on every row at
                            once, from the last column):
                              y_j = (x_j - sum_{k>j} y_k l_kj) / l_jj.
potrs(L, B) -> X            X with X A = B for A = L L^T, i.e. each row of B
                            as a right-hand side b of A x = b (A symmetric):
                            Y L^T = B (forward), then X L = Y (backward).
trsm_bound(L, Y)            the elementwise bound gamma_n |Y| |L|^T on
                            |X - Y L^T| that forward substitution computed in
                            floating point satisfies (Higham, Theorem 8.5).
backward_bound(L)           the elementwise bound gamma_{n+1} (|L| |L|^T) on
                            |A - L L^T| that a Cholesky factorisation computed
                            in floating point with any summation order satisfies
                            (Higham, Accuracy and Stability of Numerical
                            Algorithms, 2nd ed., Theorem 10.3).
"""
import numpy as np

U_FP64 = 2.0 ** -53


class NotPositiveDefinite(ValueError):
    def __init__(self, column):
        super().__init__(f"matrix is not positive definite: pivot {column} is not positive")
        self.column = column


def potrf_lower(A):
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    assert A.shape == (n, n)
    L = np.zeros((n, n))
    for j in range(n):
        d = A[j, j] - L[j, :j] @ L[j, :j]
        if not (d > 0.0) or not np.isfinite(d):
            raise NotPositiveDefinite(j)
        L[j, j] = np.sqrt(d)
        if j + 1 < n:
            L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def syrk_lower(alpha, A, beta, C):
    A = np.asarray(A, dtype=np.float64)
    C = np.array(C, dtype=np.float64, copy=True)
    n = C.shape[0]
    assert C.shape == (n, n) and A.shape[0] == n
    S = A @ A.T
    low = np.tril(np.ones((n, n), dtype=bool))
    if beta == 0.0:
        C[low] = alpha * S[low]
    else:
        C[low] = alpha * S[low] + beta * C[low]
    return C


def trsm_rlt(L, X):
    L = np.asarray(L, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    n = L.shape[0]
    assert L.shape == (n, n) and X.shape[1] == n
    Y = np.zeros_like(X)
    for j in range(n):
        Y[:, j] = (X[:, j] - Y[:, :j] @ L[j, :j]) / L[j, j]
    return Y


def trsm_rln(L, X):
    L = np.asarray(L, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    n = L.shape[0]
    assert L.shape == (n, n) and X.shape[1] == n
    Y = np.zeros_like(X)
    for j in range(n - 1, -1, -1):
        Y[:, j] = (X[:, j] - Y[:, j + 1:] @ L[j + 1:, j]) / L[j, j]
    return Y


def potrs(L, B):
    return trsm_rln(L, trsm_rlt(L, B))


def trsm_bound(L, Y):
    """gamma_n |Y| |L|^T, gamma_n = n u / (1 - n u)."""
    n = L.shape[0]
    gamma = n * U_FP64 / (1.0 - n * U_FP64)
    return gamma * (np.abs(Y) @ np.abs(np.tril(L)).T)


def backward_bound(L):
    """gamma_{n+1} (|L| |L|^T): gamma_m = m u / (1 - m u)."""
    n = L.shape[0]
    m = n + 1
    gamma = m * U_FP64 / (1.0 - m * U_FP64)
    aL = np.abs(L)
    return gamma * (aL @ aL.T)
