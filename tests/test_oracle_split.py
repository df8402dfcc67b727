"""Pins of the split-BF16 reference: the slicing is error free (exact
reconstruction, integer slices that BF16 holds exactly), integer inputs are
reproduced exactly with one slice, and the error against the exact product
falls with the slice count and stays within the truncation bound."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import split_ref


def _mat(r, c, seed, mat, dist=synth.NORMAL, row_exp=(0, 0), col_exp=(0, 0)):
    return synth.matrix(r, c, synth.spec(seed, mat, dist, row_exp=row_exp, col_exp=col_exp))


def _bf16_exact(x):
    """True where x is exactly representable in bfloat16 (8 significant bits)."""
    m, e = np.frexp(x)
    return np.all(np.ldexp(m, 8) == np.rint(np.ldexp(m, 8)))


def test_exponent_definition():
    X = np.array([[1.0, -0.5], [0.75, 0.0], [0.0, 0.0], [-3.0, 2.0 ** -30]])
    e = split_ref.exponents(X, 1)
    # smallest e with max|x| < 2^e: 1 -> 1 (not 0), 0.75 -> 0, zero row -> 0, 3 -> 2
    assert list(e) == [1, 0, 0, 2]
    assert list(split_ref.exponents(X.T, 0)) == [1, 0, 0, 2]


@pytest.mark.parametrize("s", [1, 3, 6, 8])
def test_reconstruction_is_exact(s):
    A = _mat(40, 300, 1, 0, row_exp=(-20, 20))
    e = split_ref.exponents(A, 1)
    sl, r = split_ref.slices(A, e, s, 1)
    total = np.zeros_like(A)
    # add from the smallest part up; each partial sum is exact
    total = r.copy()
    for p in range(s, 0, -1):
        total = total + np.ldexp(sl[p - 1], (e[:, None] - 8 * p))
    assert np.array_equal(total, A)
    assert np.all(np.abs(r) <= np.ldexp(np.ones_like(r), e[:, None] - 8 * s - 1))
    for p, m in enumerate(sl, start=1):
        assert np.array_equal(m, np.rint(m))
        assert np.abs(m).max() <= (256 if p == 1 else 128)
        assert _bf16_exact(m)


def test_slice_products_exact_in_fp32_per_chunk():
    # any chunk of 256 products of slices stays below 2^24 in magnitude
    A = _mat(8, 256, 2, 0)
    B = _mat(256, 8, 2, 1)
    e, f = split_ref.exponents(A, 1), split_ref.exponents(B, 0)
    sa, _ = split_ref.slices(A, e, 4, 1)
    sb, _ = split_ref.slices(B, f, 4, 0)
    for p in range(4):
        for q in range(4):
            T = np.abs(sa[p]) @ np.abs(sb[q])
            assert T.max() <= 2 ** 24
            # FP32 accumulation reproduces the FP64 integer sum
            T32 = (sa[p].astype(np.float32) @ sb[q].astype(np.float32)).astype(np.float64)
            assert np.array_equal(T32, sa[p] @ sb[q])


def test_integer_inputs_exact_with_one_slice():
    A = _mat(9, 33, 3, 0, synth.INT)
    B = _mat(33, 7, 3, 1, synth.INT)
    C = _mat(9, 7, 3, 2, synth.INT)
    got = split_ref.split_gemm(1.0, A, B, 0.0, C, s=1)
    exact = np.array([[sum(int(A[i, k]) * int(B[k, j]) for k in range(33)) for j in range(7)] for i in range(9)],
                     dtype=np.float64)
    assert np.array_equal(got, exact)
    ones = split_ref.split_gemm(1.0, np.ones((3, 50)), np.ones((50, 4)), 0.0, None, s=1)
    assert np.all(ones == 50)


def test_error_falls_with_slices_and_meets_gate():
    M, N, K = 48, 40, 512
    A = _mat(M, K, 4, 0, row_exp=(-20, 20))
    B = _mat(K, N, 4, 1, col_exp=(-20, 20))
    ref, D = oracle.gemm_rows(1.0, A, B, 0.0, None)
    errs = []
    for s in range(1, 9):
        got = split_ref.split_gemm(1.0, A, B, 0.0, None, s=s)
        errs.append(oracle.normalized_error(got, ref, D))
    assert all(errs[i + 1] <= errs[i] * 1.01 + 1e-16 for i in range(len(errs) - 1)), errs
    assert errs[3] > 1e-12  # four slices are not enough
    assert errs[5] <= oracle.GATE  # six slices meet the gate
    assert errs[7] <= 1e-15


def test_against_exact_rational_within_truncation_bound():
    M, N, K = 3, 4, 24
    A = _mat(M, K, 5, 0, row_exp=(-5, 5))
    B = _mat(K, N, 5, 1, col_exp=(-5, 5))
    exact = [[sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(K)) for j in range(N)] for i in range(M)]
    for s in (2, 3, 5, 7):
        got = split_ref.split_gemm(1.0, A, B, 0.0, None, s=s)
        bound = split_ref.truncation_bound(A, B, s)
        for i in range(M):
            for j in range(N):
                err = abs(Fraction(got[i, j]) - exact[i][j])
                # truncation plus FP64 rounding of the final weighted sum
                allow = Fraction(bound[i, j]) + Fraction(4 * s * 2.0 ** -53) * abs(exact[i][j]) + Fraction(2.0 ** -1000)
                assert err <= allow, (s, i, j)


def test_panels_and_alpha_beta():
    M, N, K = 16, 12, 100
    A = _mat(M, K, 6, 0)
    B = _mat(K, N, 6, 1)
    C = _mat(M, N, 6, 2, synth.UNIFORM)
    ref, D = oracle.gemm_rows(1.5, A, B, 0.5, C)
    for kb in (None, 32, 100, 7):
        got = split_ref.split_gemm(1.5, A, B, 0.5, C, s=7, kb=kb)
        assert oracle.normalized_error(got, ref, D) < 1e-14
    # beta = 0 does not read C; alpha = 0 returns beta*C
    Cn = np.full((M, N), np.nan)
    assert np.all(np.isfinite(split_ref.split_gemm(1.0, A, B, 0.0, Cn, s=3)))
    assert np.array_equal(split_ref.split_gemm(0.0, A, B, 0.5, C, s=3), 0.5 * C)


# ---- INT8 slices (7 bits per slice, truncated toward zero) ----

@pytest.mark.parametrize("s", [1, 4, 7])
def test_int8_reconstruction_is_exact(s):
    A = _mat(40, 300, 7, 0, row_exp=(-20, 20))
    e = split_ref.exponents(A, 1)
    sl, r = split_ref.slices(A, e, s, 1, fmt="i8")
    total = r.copy()
    for p in range(s, 0, -1):
        total = total + np.ldexp(sl[p - 1], (e[:, None] - 7 * p))
    assert np.array_equal(total, A)
    # truncation: the remainder keeps the sign of x and is below one unit of the last digit
    assert np.all(np.abs(r) < np.ldexp(np.ones_like(r), e[:, None] - 7 * s))
    assert np.all(r * A >= 0)
    for m in sl:
        assert np.array_equal(m, np.trunc(m))
        assert np.abs(m).max() <= 127  # fits a signed byte
        assert np.all(m * A >= 0)      # every digit has the sign of x


def test_int8_digits_of_a_known_value():
    # 0.7 with exponent 0: 0.7 * 2^7 = 89.6 -> 89; remainder 0.6 * 2^-7, times 2^14 -> 76.8 -> 76
    A = np.array([[0.7, -0.7]])
    e = split_ref.exponents(A, 1)
    assert list(e) == [0]
    sl, _ = split_ref.slices(A, e, 2, 1, fmt="i8")
    assert list(sl[0][0]) == [89.0, -89.0]
    assert list(sl[1][0]) == [76.0, -76.0]


def test_int8_weight_sums_fit_int32():
    # |m_p m_q| <= 127^2 < 2^14: a weight's sum over s pairs and 8192 k stays below 2^31
    A = np.full((2, 8192), -0.99999)
    B = np.full((8192, 2), 0.99999)
    e, f = split_ref.exponents(A, 1), split_ref.exponents(B, 0)
    sa, _ = split_ref.slices(A, e, 8, 1, fmt="i8")
    sb, _ = split_ref.slices(B, f, 8, 0, fmt="i8")
    for t in range(2, 10):
        U = sum(np.abs(sa[p - 1]) @ np.abs(sb[t - p - 1]) for p in range(max(1, t - 8), min(t - 1, 8) + 1))
        assert U.max() < 2 ** 31


def test_int8_integer_inputs_exact():
    # integers below 2^7 in magnitude are one digit each (e = 7 for a row holding 64..127)
    A = _mat(9, 33, 8, 0, synth.INT)
    B = _mat(33, 7, 8, 1, synth.INT)
    exact = np.array([[sum(int(A[i, k]) * int(B[k, j]) for k in range(33)) for j in range(7)] for i in range(9)],
                     dtype=np.float64)
    assert np.array_equal(split_ref.split_gemm(1.0, A, B, 0.0, None, s=2, fmt="i8"), exact)


def test_int8_error_falls_with_slices_and_meets_gate():
    M, N, K = 48, 40, 512
    A = _mat(M, K, 4, 0, row_exp=(-20, 20))
    B = _mat(K, N, 4, 1, col_exp=(-20, 20))
    ref, D = oracle.gemm_rows(1.0, A, B, 0.0, None)
    errs = [oracle.normalized_error(split_ref.split_gemm(1.0, A, B, 0.0, None, s=s, fmt="i8"), ref, D)
            for s in range(1, 10)]
    assert all(errs[i + 1] <= errs[i] * 1.01 + 1e-16 for i in range(len(errs) - 1)), errs
    # seven bits per slice: s INT8 slices sit between s-1 and s BF16 slices
    bf = [oracle.normalized_error(split_ref.split_gemm(1.0, A, B, 0.0, None, s=s), ref, D) for s in (4, 5, 6)]
    assert errs[4] > bf[1] and errs[5] > bf[2] and errs[5] < bf[0]
    assert errs[5] > oracle.GATE and errs[6] <= oracle.GATE  # normal data: seven INT8 slices meet the gate
    assert errs[8] <= 1e-15
    # uniform data (smaller spread inside a row): six INT8 slices meet it, five do not
    A = _mat(M, K, 4, 0, synth.UNIFORM, row_exp=(-20, 20))
    B = _mat(K, N, 4, 1, synth.UNIFORM, col_exp=(-20, 20))
    ref, D = oracle.gemm_rows(1.0, A, B, 0.0, None)
    eu = [oracle.normalized_error(split_ref.split_gemm(1.0, A, B, 0.0, None, s=s, fmt="i8"), ref, D) for s in (5, 6)]
    assert eu[0] > oracle.GATE and eu[1] <= oracle.GATE, eu


def test_int8_against_exact_rational_within_truncation_bound():
    M, N, K = 3, 4, 24
    A = _mat(M, K, 9, 0, row_exp=(-5, 5))
    B = _mat(K, N, 9, 1, col_exp=(-5, 5))
    exact = [[sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(K)) for j in range(N)] for i in range(M)]
    for s in (2, 3, 5, 7):
        got = split_ref.split_gemm(1.0, A, B, 0.0, None, s=s, fmt="i8")
        bound = split_ref.truncation_bound(A, B, s, fmt="i8")
        for i in range(M):
            for j in range(N):
                err = abs(Fraction(got[i, j]) - exact[i][j])
                allow = Fraction(bound[i, j]) + Fraction(4 * s * 2.0 ** -53) * abs(exact[i][j]) + Fraction(2.0 ** -1000)
                assert err <= allow, (s, i, j)
        # the bound is not vacuous: truncating at s = 2 errs by more than a thousandth of it somewhere
        if s == 2:
            worst = max(abs(Fraction(got[i, j]) - exact[i][j]) / Fraction(bound[i, j]) for i in range(M) for j in range(N))
            assert worst > Fraction(1, 1000)


def test_int8_panels_and_alpha_beta():
    M, N, K = 16, 12, 100
    A = _mat(M, K, 6, 0)
    B = _mat(K, N, 6, 1)
    C = _mat(M, N, 6, 2, synth.UNIFORM)
    ref, D = oracle.gemm_rows(1.5, A, B, 0.5, C)
    for kb in (None, 32, 7):
        got = split_ref.split_gemm(1.5, A, B, 0.5, C, s=8, kb=kb, fmt="i8")
        assert oracle.normalized_error(got, ref, D) < 1e-14


def test_bf16_truncation_bound_is_not_vacuous():
    # random data: at s = 2 the error reaches more than a thousandth of the bound somewhere
    M, N, K = 3, 4, 24
    A = _mat(M, K, 5, 0, row_exp=(-5, 5))
    B = _mat(K, N, 5, 1, col_exp=(-5, 5))
    exact = [[sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(K)) for j in range(N)] for i in range(M)]
    got = split_ref.split_gemm(1.0, A, B, 0.0, None, s=2)
    bound = split_ref.truncation_bound(A, B, 2)
    worst = max(abs(Fraction(got[i, j]) - exact[i][j]) / Fraction(bound[i, j]) for i in range(M) for j in range(N))
    assert Fraction(1, 1000) < worst <= 1


@pytest.mark.parametrize("K", [1, 16])
def test_bf16_truncation_bound_is_tight_on_adversarial_digits(K):
    # v = 2^-1 + 2^-9 + ... + 2^-49 slices into 129, -127, -127, ...: the dropped pairs of one
    # weight all carry the same sign and add up, so the error reaches a quarter of the bound
    # at s = 1 and s = 6.  A bound with 2^(-7s) for BF16 slices, or without the factor k or
    # (s + 1), fails this test.
    v = sum(2.0 ** (-1 - 8 * p) for p in range(7))
    A, B = np.full((1, K), v), np.full((K, 1), v)
    exact = Fraction(v) * Fraction(v) * K
    for s in (1, 6):
        got = split_ref.split_gemm(1.0, A, B, 0.0, None, s=s)
        ratio = abs(Fraction(got[0, 0]) - exact) / Fraction(split_ref.truncation_bound(A, B, s)[0, 0])
        assert Fraction(1, 8) < ratio <= 1, (s, float(ratio))
