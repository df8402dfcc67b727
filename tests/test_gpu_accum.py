"""Accumulation sessions on the GPU, through the C ABI: C = beta*C_in + sum over
steps of alpha_s A_s B_s with part of C resident on the device for the whole
session and the rest streamed at every step, against the oracle applied one
step after the other (Section V: MMOOC as the local step of SUMMA / HSUMMA)."""
import sys

import numpy as np
import pytest

import oracle
import synth
import paper_1808_05056_amd as ooc

pytestmark = pytest.mark.gpu
MiB = 1 << 20


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run_session(M, N, Ks, alphas, beta, budget, dist, seed, opts=None):
    As = [ooc.PinnedMatrix(M, K) for K in Ks]
    Bs = [ooc.PinnedMatrix(K, N) for K in Ks]
    Cm = ooc.PinnedMatrix(M, N)
    try:
        for s in range(len(Ks)):
            synth.fill(As[s].array, synth.spec(seed + s, 0, dist))
            synth.fill(Bs[s].array, synth.spec(seed + s, 1, dist))
        synth.fill(Cm.array, synth.spec(seed, 2, dist))
        C0 = Cm.array.copy()
        sess = ooc.AccumSession(beta, Cm.array, budget, opts)
        for s in range(len(Ks)):
            _, st = sess.step(alphas[s], As[s].array, Bs[s].array)
            _say(f"  step {s}: K={Ks[s]} plan {st.plan} t={st.t_total_s * 1e3:.2f} ms")
        sess.end()
        got = Cm.array.copy()
        # the oracle, step after step; the last step's |A||B| and C_in give the gate's scale
        ref = C0
        Dsum = np.zeros((M, N))
        for s in range(len(Ks)):
            b = beta if s == 0 else 1.0
            ref, D = oracle.gemm_rows(alphas[s], As[s].array, Bs[s].array, b, ref if (b != 0.0) else None)
            Dsum += abs(alphas[s]) * D
        return got, ref, Dsum, C0
    finally:
        for m in As + Bs + [Cm]:
            m.free()


@pytest.mark.parametrize("case", ["partial-resident", "all-resident", "beta-zero"])
def test_session_matches_oracle(case):
    M, N, Ks, alphas, beta, budget = {
        "partial-resident": (3000, 2000, [700, 500, 900], [1.0, -0.5, 2.0], 0.5, 16 * MiB),
        "all-resident": (1000, 800, [300, 300], [1.0, 1.0], -1.0, 64 * MiB),
        "beta-zero": (2500, 1500, [1000, 200], [1.5, 1.0], 0.0, 8 * MiB),
    }[case]
    R = ooc.ooc_accum_resident_rows(M, N, budget)
    _say(f"session {case}: M={M} N={N} steps K={Ks} budget={budget} resident rows {R}")
    got, ref, D, C0 = _run_session(M, N, Ks, alphas, beta, budget, synth.UNIFORM, 70)
    # denominator: sum of |alpha_s| (|A_s||B_s|) plus |beta| |C_in| (each step's product enters once)
    den = D + (abs(beta) * np.abs(C0) if beta != 0.0 else 0.0)
    err = oracle.normalized_error(got, ref, den)
    _say(f"  normalised error {err:.3e}")
    assert err <= oracle.GATE


def test_session_integer_data_bit_exact():
    M, N, Ks, alphas, beta, budget = 2000, 1200, [300, 257, 64], [2.0, -1.0, 0.5], 1.5, 8 * MiB
    assert 0 < ooc.ooc_accum_resident_rows(M, N, budget) < M
    got, ref, _, _ = _run_session(M, N, Ks, alphas, beta, budget, synth.INT, 80)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("prec,slices", [(ooc.SPLIT_BF16, 6), (ooc.SPLIT_INT8, 7)])
def test_session_split_steps(prec, slices):
    M, N, Ks, alphas, beta, budget = 1500, 1300, [1100, 900], [1.0, 1.0], 1.0, 24 * MiB
    opts = ooc.make_opts(precision=prec, slices=slices)
    got, ref, D, C0 = _run_session(M, N, Ks, alphas, beta, budget, synth.NORMAL, 90, opts)
    den = D + abs(beta) * np.abs(C0)
    err = oracle.normalized_error(got, ref, den)
    _say(f"  split session (precision {prec}, s = {slices}) normalised error {err:.3e}")
    assert err <= oracle.GATE


def test_session_without_steps_scales_c():
    M, N, beta, budget = 900, 700, -0.75, 2 * MiB
    Cm = ooc.PinnedMatrix(M, N)
    try:
        synth.fill(Cm.array, synth.spec(5, 2))
        C0 = Cm.array.copy()
        assert 0 < ooc.ooc_accum_resident_rows(M, N, budget) < M
        sess = ooc.AccumSession(beta, Cm.array, budget)
        sess.end()
        assert np.array_equal(Cm.array, beta * C0)
    finally:
        Cm.free()
