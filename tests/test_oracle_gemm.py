"""Pins of the CPU reference product against facts fixed by the mathematics:
closed forms, exact integer results, exact rational arithmetic and a library
routine, so that a dropped term, a wrong sign, a transposed operand or a
mishandled alpha/beta/leading dimension fails at least one test."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

U = 2.0 ** -53


def _mat(rows, cols, seed, mat, dist=synth.UNIFORM, ld=None):
    return synth.matrix(rows, cols, synth.spec(seed, mat, dist), ld=ld)


def test_all_ones_gives_k():
    M, N, K = 7, 5, 1000
    A = np.ones((M, K))
    B = np.ones((K, N))
    C0 = np.ones((M, N))
    Cref, D = oracle.gemm_rows(1.0, A, B, 0.0, None)
    assert np.all(Cref == K)
    assert np.all(D == K)
    Cref, _ = oracle.gemm_rows(1.5, A, B, 0.5, C0)
    assert np.all(Cref == 1.5 * K + 0.5)


def test_identity_and_powers_of_two():
    K = 37
    N = 11
    B = _mat(K, N, 3, synth.MAT_B)
    C0 = _mat(K, N, 3, synth.MAT_C)
    Cref, _ = oracle.gemm_rows(1.0, np.eye(K), B, 0.0, None)
    assert np.array_equal(Cref, B)
    # alpha, beta powers of two: one rounding in the final add only
    Cref, _ = oracle.gemm_rows(2.0, np.eye(K), B, 0.5, C0)
    assert np.array_equal(Cref, 2.0 * B + 0.5 * C0)
    # diagonal 2^k scaling is exact
    d = 2.0 ** np.arange(-10, K - 10)
    Cref, _ = oracle.gemm_rows(1.0, np.diag(d), B, 0.0, None)
    assert np.array_equal(Cref, d[:, None] * B)


def test_integer_inputs_exact_and_not_transposed():
    # non-square shapes with integer entries: the exact product is known
    M, N, K = 9, 13, 7
    A = _mat(M, K, 5, synth.MAT_A, synth.INT)
    B = _mat(K, N, 5, synth.MAT_B, synth.INT)
    C0 = _mat(M, N, 5, synth.MAT_C, synth.INT)
    exact = [[sum(int(A[i, k]) * int(B[k, j]) for k in range(K)) for j in range(N)] for i in range(M)]
    Cref, D = oracle.gemm_rows(1.0, A, B, 0.0, None)
    assert np.array_equal(Cref, np.array(exact, dtype=np.float64))
    absx = [[sum(abs(int(A[i, k])) * abs(int(B[k, j])) for k in range(K)) for j in range(N)] for i in range(M)]
    assert np.array_equal(D, np.array(absx, dtype=np.float64))
    Cref, _ = oracle.gemm_rows(-3.0, A, B, 2.0, C0)
    want = np.array([[-3 * exact[i][j] + 2 * int(C0[i, j]) for j in range(N)] for i in range(M)], dtype=np.float64)
    assert np.array_equal(Cref, want)


def test_random_within_rounding_bound_of_exact():
    # exact rational result vs the reference: |err| <= gamma_K * (|A||B|)
    M, N, K = 4, 5, 64
    A = _mat(M, K, 7, synth.MAT_A, synth.NORMAL)
    B = _mat(K, N, 7, synth.MAT_B, synth.NORMAL)
    Cref, D = oracle.gemm_rows(1.0, A, B, 0.0, None)
    gamma = K * U / (1 - K * U)
    for i in range(M):
        for j in range(N):
            ex = sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(K))
            err = abs(Fraction(Cref[i, j]) - ex)
            assert err <= Fraction(gamma) * Fraction(D[i, j])


def test_against_library_matmul():
    M, N, K = 64, 48, 300
    A = _mat(M, K, 11, synth.MAT_A)
    B = _mat(K, N, 11, synth.MAT_B)
    C0 = _mat(M, N, 11, synth.MAT_C)
    Cref, D = oracle.gemm_rows(1.5, A, B, 0.5, C0)
    lib = 1.5 * (A @ B) + 0.5 * C0
    assert oracle.normalized_error(Cref, lib, np.abs(A) @ np.abs(B)) < 1e-14
    assert np.allclose(D, np.abs(A) @ np.abs(B), rtol=1e-14, atol=0)


def test_leading_dimensions_and_row_subsets():
    M, N, K = 20, 17, 23
    A = _mat(M, K, 13, synth.MAT_A, ld=K + 5)
    B = _mat(K, N, 13, synth.MAT_B, ld=N + 3)
    C0 = _mat(M, N, 13, synth.MAT_C)
    full, _ = oracle.gemm_rows(0.75, A, B, -1.25, C0)
    dense, _ = oracle.gemm_rows(0.75, np.ascontiguousarray(A), np.ascontiguousarray(B), -1.25, C0)
    assert np.array_equal(full, dense)
    rows = np.array([19, 0, 7, 7])
    sub, _ = oracle.gemm_rows(0.75, A, B, -1.25, C0[rows], rows=rows)
    assert np.array_equal(sub, full[rows])


def test_beta_zero_ignores_nan_and_alpha_zero_ignores_ab():
    M, N, K = 6, 8, 10
    A = _mat(M, K, 17, synth.MAT_A)
    B = _mat(K, N, 17, synth.MAT_B)
    Cn = np.full((M, N), np.nan)
    Cref, _ = oracle.gemm_rows(1.0, A, B, 0.0, Cn)
    assert np.all(np.isfinite(Cref))
    An = np.full((M, K), np.nan)
    C0 = _mat(M, N, 17, synth.MAT_C)
    Cref, _ = oracle.gemm_rows(0.0, An, B, 0.5, C0)
    assert np.array_equal(Cref, 0.5 * C0)
    Cref, _ = oracle.gemm_rows(0.0, An, B, 0.0, Cn)
    assert np.all(Cref == 0.0)


def test_k_zero():
    M, N = 5, 4
    C0 = _mat(M, N, 19, synth.MAT_C)
    Cref, D = oracle.gemm_rows(2.0, np.zeros((M, 0)), np.zeros((0, N)), 0.25, C0)
    assert np.array_equal(Cref, 0.25 * C0)
    assert np.all(D == 0)


def test_nan_propagates_in_ab():
    M, N, K = 3, 3, 4
    A = np.ones((M, K))
    A[1, 2] = np.nan
    Cref, _ = oracle.gemm_rows(1.0, A, np.ones((K, N)), 0.0, None)
    assert np.all(np.isnan(Cref[1])) and np.all(Cref[0] == K) and np.all(Cref[2] == K)


def test_normalized_error_metric():
    D = np.array([[2.0, 0.0]])
    assert oracle.normalized_error(np.array([[1.0, 3.0]]), np.array([[1.5, 3.0]]), D) == 0.25
    assert oracle.normalized_error(np.array([[1.0, 3.0]]), np.array([[1.0, 3.5]]), D) == math.inf


def test_generator_is_counter_based():
    sp = synth.spec(42, synth.MAT_A, synth.NORMAL, row_exp=(-20, 20))
    X = synth.matrix(50, 40, sp)
    rows = np.array([49, 3, 17])
    Y = np.empty((3, 15))
    synth.fill_rows(Y, rows, sp, col0=25)
    assert np.array_equal(Y, X[rows, 25:40])
    Z = np.empty((10, 40))
    synth.fill(Z, sp, row0=20)
    assert np.array_equal(Z, X[20:30])
    # distribution sanity: uniform in [-1,1), normal moments
    u = synth.matrix(400, 500, synth.spec(1, 0, synth.UNIFORM))
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01
    nrm = synth.matrix(400, 500, synth.spec(1, 0, synth.NORMAL))
    assert abs(nrm.mean()) < 0.01 and abs(nrm.std() - 1) < 0.01


def test_gate_denominator():
    D = np.array([[2.0, 1e-9]])
    Cin = np.array([[4.0, 0.5]])
    assert np.array_equal(oracle.gate_denominator(1.0, D, 0.0, Cin), D)
    assert np.array_equal(oracle.gate_denominator(-2.0, D, 0.5, Cin), np.array([[6.0, 0.25 + 2e-9]]))
    # one rounding of a beta*C-dominated entry is within the gate with the full denominator
    c = 0.48
    one_ulp = np.spacing(c)
    assert one_ulp / 1.2e-5 > oracle.GATE
    assert one_ulp / oracle.gate_denominator(1.5, np.array(1.2e-5), 0.5, np.array(c / 0.5)) < oracle.GATE
