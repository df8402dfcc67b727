"""The learned planner on the GPU: fitting a network to synthetic timings with
the library's kernels, and what the trained planner network gains over the
method without it (the paper's partition rule) on problems of the evaluation
batch, measured."""
import os

import numpy as np
import pytest

import synth
from synth import workloads as W
import paper_1808_05056_amd as ooc
from gpu_helpers import PinnedProblem, check_rows, sample_rows

pytestmark = pytest.mark.gpu
WEIGHTS = os.path.join(os.path.dirname(ooc.LIB_PATH), "planner_mlp.txt")


def test_fit_learns_a_timing_function():
    plans, model_s = ooc.ooc_plan_candidates(20000, 16000, 12000, 0.0, 2 << 30)
    X = ooc.ooc_mlp_features(20000, 16000, 12000, 0.0, 2 << 30, plans)
    # a synthetic "measured" time: the model's time with a penalty for one stream
    t = np.array(model_s) * np.where(X[:, 15] == 1, 1.8, 1.0)
    hist = ooc.ooc_mlp_fit(X, t, hidden=32, epochs=1500, lr=3e-3, weight_decay=0.0, seed=3)
    assert hist[-1] < 0.05 * hist[0]
    pred = ooc.ooc_mlp_predict(20000, 16000, 12000, 0.0, 2 << 30, plans)
    assert np.corrcoef(np.log(pred), np.log(t))[0, 1] > 0.95
    # restore the shipped network (if any) for the planner tests
    if os.path.exists(WEIGHTS):
        ooc.ooc_mlp_load(WEIGHTS)


def _subset():
    """Problems of the evaluation batch fixed by size alone, never by outcome:
    the first four under 4e12 flop."""
    return [w for w in W.problem_batch(4, count=64) if w.flops < 4e12][:4]


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained planner network shipped with the library")
def test_learned_planner_beats_the_papers_rule():
    """What the trained network gains over the method without it (the paper's
    partition rule), with its gain or regret against the cost model beside it."""
    ooc.ooc_mlp_load(WEIGHTS)
    problems = _subset()
    assert problems and all(w.beta == 0.0 for w in problems)
    gains, vs_model = [], []
    for w in problems:
        pp = PinnedProblem(w)
        try:
            times = {}
            for name, planner in (("mlp", ooc.PLAN_MLP), ("paper", ooc.PLAN_PAPER), ("model", ooc.PLAN_MODEL)):
                opts = ooc.make_opts(planner=planner)
                _, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, opts)
                assert stats.arena_bytes <= w.budget
                # beta = 0 in this batch, so every call leaves C = alpha*A*B: check it
                check_rows(w, pp, sample_rows(w.M, stats.plan.mb, count=8))
                best = min(ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, opts)[1].t_pipeline_s
                           for _ in range(2))
                times[name] = best
            gains.append(times["paper"] / times["mlp"])
            vs_model.append(times["model"] / times["mlp"])
            print(f"M={w.M} N={w.N} K={w.K} budget={w.budget >> 20} MiB: paper {times['paper']:.4f}s "
                  f"model {times['model']:.4f}s learned {times['mlp']:.4f}s", flush=True)
        finally:
            pp.free()
    print(f"learned vs paper's rule: {np.mean(gains):.3f}x; vs cost model: {np.mean(vs_model):.3f}x", flush=True)
    assert np.mean(gains) > 1.0, gains


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained planner network shipped with the library")
def test_learned_planner_on_split_plans():
    """The shipped network was also fitted to split-BF16 (s = 5) timings.  On
    the same size-fixed subset of the evaluation batch its split choice runs
    within the budget, meets the gate against the oracle and, in total, is not
    slower than the cost model's choice beyond timing noise (5 %)."""
    ooc.ooc_mlp_load(WEIGHTS)
    problems = _subset()
    assert all(w.beta == 0.0 and w.flops < 4e12 for w in problems)
    total = {"mlp": 0.0, "model": 0.0}
    differ = 0
    for w in problems:
        pp = PinnedProblem(w)
        try:
            chosen = {}
            for name, planner in (("mlp", ooc.PLAN_MLP), ("model", ooc.PLAN_MODEL)):
                opts = ooc.make_opts(planner=planner, precision=ooc.SPLIT_BF16, slices=5)
                _, stats = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, opts)
                assert stats.arena_bytes <= w.budget and stats.plan.precision == ooc.SPLIT_BF16
                check_rows(w, pp, sample_rows(w.M, stats.plan.mb, count=8))
                chosen[name] = stats.plan.as_dict()
                best = min(ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, opts)[1].t_pipeline_s
                           for _ in range(3))
                total[name] += best
                print(f"M={w.M} N={w.N} K={w.K} budget={w.budget >> 20} MiB {name}: {best:.4f}s "
                      f"{chosen[name]}", flush=True)
            differ += chosen["mlp"] != chosen["model"]
        finally:
            pp.free()
    print(f"split plans: learned {total['mlp']:.4f}s, cost model {total['model']:.4f}s; "
          f"{differ} of {len(problems)} choices differ", flush=True)
    assert total["mlp"] <= 1.05 * total["model"], total


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained planner network shipped with the library")
def test_learned_planner_declines_problems_outside_its_training_range():
    """M, N, K or budget more than four deviations (log scale) from the
    training problems' mean: the network's prediction would be an
    extrapolation and the cost model's plan stands (here a 1024^3 problem
    through 8 MiB and a 2^22-row one); the tall workload, whose shapes the
    training batch covers, is planned by the network."""
    ooc.ooc_mlp_load(WEIGHTS)
    far = W.Workload("far", 1 << 22, 8192, 8192, 1.0, 0.0, 4 << 30, seed=0)
    for w in (far, W.SMALL):
        for prec, s in ((ooc.FP64, 0), (ooc.SPLIT_BF16, 5)):
            mlp = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget,
                               ooc.make_opts(planner=ooc.PLAN_MLP, precision=prec, slices=s))
            model = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget,
                                 ooc.make_opts(planner=ooc.PLAN_MODEL, precision=prec, slices=s))
            assert mlp.as_dict() == model.as_dict(), (w.name, prec)
    w = W.TALL
    cands = ooc.ooc_plan_candidates(w.M, w.N, w.K, w.beta, w.budget)[0][:8]
    pred = ooc.ooc_mlp_predict(w.M, w.N, w.K, w.beta, w.budget, cands)
    assert np.all(np.isfinite(pred)) and np.all(np.asarray(pred) > 0)
    mlp = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, ooc.make_opts(planner=ooc.PLAN_MLP))
    assert mlp.as_dict() == cands[int(np.argmin(pred))].as_dict()


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained planner network shipped with the library")
def test_measured_sweep_and_the_learned_planners_fallback():
    """PLAN_SWEEP times the cost model's 8 best candidates on the caller's
    operands and keeps the fastest: the result meets the gate, the plan is one
    of those candidates, and a second call reuses it without timing again.  A
    problem the network declines (K = 64, far below its training range) is
    planned under PLAN_MLP by the same measured sweep."""
    MiB = 1 << 20
    sweep, mlp, model = (ooc.make_opts(planner=p) for p in (ooc.PLAN_SWEEP, ooc.PLAN_MLP, ooc.PLAN_MODEL))
    w = W.Workload("sweep", 2048, 2048, 2048, 1.0, 0.5, 64 * MiB, seed=51)
    pp = PinnedProblem(w)
    try:
        _, s1 = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, sweep)
        check_rows(w, pp, sample_rows(w.M, s1.plan.mb, count=32, seed=1))
        cands = ooc.ooc_plan_candidates(w.M, w.N, w.K, w.beta, w.budget, model)[0][:8]
        assert s1.plan.as_dict() in [c.as_dict() for c in cands]
        synth.fill(pp.C, w.spec_c())
        _, s2 = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, sweep)
        check_rows(w, pp, sample_rows(w.M, s2.plan.mb, count=32, seed=2))
        print(f"sweep: plan {s1.plan}; planning {s1.t_plan_s * 1e3:.1f} ms (timed), then {s2.t_plan_s * 1e3:.3f} ms; "
              f"product {s2.t_total_s * 1e3:.1f} ms", flush=True)
        assert s2.plan.as_dict() == s1.plan.as_dict()
        assert s1.t_plan_s > 4 * s2.t_total_s  # the first call timed the candidates (9 products)
        assert s2.t_plan_s < min(s2.t_total_s, s1.t_plan_s / 4)  # the second did not
    finally:
        pp.free()
    ooc.ooc_mlp_load(WEIGHTS)
    wd = W.Workload("declined", 4096, 4096, 64, 1.0, 0.0, 64 * MiB, seed=52)
    # the network declines: the planning-only call returns the cost model's choice
    assert (ooc.ooc_plan(wd.M, wd.N, wd.K, 0.0, wd.budget, mlp).as_dict()
            == ooc.ooc_plan(wd.M, wd.N, wd.K, 0.0, wd.budget, model).as_dict())
    pp = PinnedProblem(wd)
    try:
        _, s3 = ooc.ooc_gemm(wd.alpha, pp.A, pp.B, wd.beta, pp.C, wd.budget, mlp)
        check_rows(wd, pp, sample_rows(wd.M, s3.plan.mb, count=32, seed=3))
        _, s4 = ooc.ooc_gemm(wd.alpha, pp.A, pp.B, wd.beta, pp.C, wd.budget, sweep)
        print(f"declined: MLP planning {s3.t_plan_s * 1e3:.1f} ms, plan {s3.plan}; the sweep's remembered plan "
              f"{s4.plan}", flush=True)
        assert s4.plan.as_dict() == s3.plan.as_dict()  # the sweep the MLP call ran is remembered
        assert s3.t_plan_s > 4 * s4.t_total_s  # ... the MLP call timed the candidates
        assert s4.t_plan_s < min(s4.t_total_s, s3.t_plan_s / 4)
    finally:
        pp.free()
        ooc.ooc_release(-1)
