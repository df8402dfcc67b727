"""Race stress on the GPU: the device arena starts as NaN and waits of random
length are enqueued before random operations on their streams
(OOC_STRESS_SEED), so the copies and kernels of an operation list run in
orders its waits allow but the undelayed run rarely shows.  Every result must
be bit-identical to the undelayed run of the same plan (and that run meets the
gate against the oracle): a missing wait would show as a difference or as NaN."""
import numpy as np
import pytest

from synth import workloads as W
import paper_1808_05056_amd as ooc
from gpu_helpers import PinnedProblem, check_rows, sample_rows

pytestmark = pytest.mark.gpu
MiB = 1 << 20

PLANS = [
    ("paper-2-streams", None, ooc.PLAN_PAPER),
    ("model", None, ooc.PLAN_MODEL),
    ("rows-ksplit-2s", ooc.make_plan(256, 192, 160, ooc.ORDER_ROWS, 2, 2, 2, 2), None),
    ("rowsps-group2", ooc.make_plan(256, 192, 160, ooc.ORDER_ROWS_PS, 4, 2, 3, 3, group=2), None),
    ("colsps-staged-2s", ooc.make_plan(256, 192, 160, ooc.ORDER_COLS_PS, 2, 4, 4, 2, nbuf_d=1), None),
    ("cols-1-stream", ooc.make_plan(256, 384, 640, ooc.ORDER_COLS, 2, 1, 2, 1), None),
    ("split-rowsps", ooc.make_plan(256, 256, 320, ooc.ORDER_ROWS_PS, 2, 2, 3, 3, precision=ooc.SPLIT_BF16,
                                   slices=4, group=2), None),
    ("int8-colsp-staged-2s", ooc.make_plan(256, 192, 384, ooc.ORDER_COLS_P, 2, 2, 3, 2, precision=ooc.SPLIT_INT8,
                                           slices=4, nbuf_d=1, group=2), None),
]


@pytest.mark.parametrize("case", range(len(PLANS)))
def test_results_unchanged_under_random_delays(case, monkeypatch):
    name, plan, planner = PLANS[case]
    w = W.Workload("stress", 1024, 768, 640, 1.5, 0.5, 6 * MiB, seed=11)
    pp = PinnedProblem(w)
    try:
        C0 = pp.C.copy()
        monkeypatch.delenv("OOC_STRESS_SEED", raising=False)
        if plan is None:
            _, s = ooc.ooc_gemm(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, ooc.make_opts(planner=planner))
            plan = s.plan
        else:
            _, s = ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, plan)
        assert s.arena_bytes <= w.budget
        if plan.precision == ooc.FP64:
            check_rows(w, pp, sample_rows(w.M, plan.mb, count=8))
        ref = pp.C.copy()
        assert np.isfinite(ref).all()
        for seed in range(4):
            pp.C[...] = C0
            monkeypatch.setenv("OOC_STRESS_SEED", str(seed))
            monkeypatch.setenv("OOC_STRESS_US", "400")
            _, s = ooc.ooc_gemm_planned(w.alpha, pp.A, pp.B, w.beta, pp.C, w.budget, plan)
            same = np.array_equal(pp.C, ref)
            print(f"{name} {plan} seed {seed}: {s.t_total_s * 1e3:.2f} ms, identical {same}", flush=True)
            assert same, f"{name}: seed {seed} changed the result"
    finally:
        monkeypatch.delenv("OOC_STRESS_SEED", raising=False)
        pp.free()
