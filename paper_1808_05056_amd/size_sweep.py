"""End-to-end throughput of square products across the in-core / out-of-core boundary.

The paper sweeps square N through a fixed device memory (Section VI, Tables I and
II): up to the in-core limit the whole problem fits (3 * 8 * N^2 bytes; its
largest in-core size is N = 22528 for 12 GiB), beyond it the product runs out
of core, and the paper reports no loss of throughput across the switch.  This tool measures the same
curve for this pipeline: for every N, A, B and C (uniform[-1, 1], beta = 0) are
placed in page-locked host memory and the product is timed with the given
device budget under the paper's partitioner (in core, h = w = 1, up to the
limit) and under the cost model (which pipelines even problems that would fit:
overlapping the transfers beats loading everything first), best of `reps`
calls after a warm call, the time of the whole call with its host-device
transfers.  A product counts as in core when its plan holds each operand in
one block.

    python -m paper_1808_05056_amd.size_sweep --budget-gib 12 --report size_sweep.json
"""
import argparse
import json
import sys

import paper_1808_05056_amd as ooc

GiB = 1 << 30
DEFAULT_SIZES = (1024, 2048, 4096, 8192, 12288, 16384, 20480, 22528, 24576, 28672, 32768, 40960, 46080)


def in_core_limit(budget_bytes):
    """Largest square N whose three operands fit the budget (3 * 8 * N^2 bytes)."""
    n = int((budget_bytes / 24) ** 0.5)
    while 24 * (n + 1) ** 2 <= budget_bytes:
        n += 1
    while 24 * n * n > budget_bytes:
        n -= 1
    return n


def measure(n, budget, reps=2, seed=7, planners=(("paper", ooc.PLAN_PAPER), ("model", ooc.PLAN_MODEL)),
            check=None):
    """{planner name: (plan, best seconds, TFLOP/s)} for one square product of size n.

    check, if given, is called as check(planner_name, workload, A, B, C, plan)
    after each planner's timed calls, with C holding that planner's result."""
    import synth
    from synth import workloads as W
    w = W.Workload(f"square-{n}", n, n, n, 1.0, 0.0, budget, seed=seed)
    mats = [ooc.PinnedMatrix(n, n) for _ in range(3)]
    out = {}
    try:
        A, B, C = (m.array for m in mats)
        synth.fill(A, w.spec_a())
        synth.fill(B, w.spec_b())
        for name, planner in planners:
            opts = ooc.make_opts(planner=planner)
            _, s = ooc.ooc_gemm(1.0, A, B, 0.0, C, budget, opts)
            best = min(ooc.ooc_gemm(1.0, A, B, 0.0, C, budget, opts)[1].t_total_s for _ in range(reps))
            out[name] = (s.plan, best, w.flops / best / 1e12)
            if check is not None:
                check(name, w, A, B, C, s.plan)
        return out
    finally:
        for m in mats:
            m.free()


def is_in_core(plan, n):
    return plan.mb >= n and plan.nb >= n and plan.kb >= n


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--budget-gib", type=float, default=12.0)
    ap.add_argument("--sizes", default=",".join(str(n) for n in DEFAULT_SIZES))
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--report", default="size_sweep.json")
    args = ap.parse_args(argv)
    budget = int(args.budget_gib * GiB)
    rows = []
    print(f"[size] budget {budget / GiB:.2f} GiB, in-core limit N = {in_core_limit(budget)}", flush=True)
    for n in (int(x) for x in args.sizes.split(",")):
        for name, (plan, t, tf) in measure(n, budget, args.reps).items():
            r = {"N": n, "planner": name, "in_core": is_in_core(plan, n), "seconds": t, "tflops": tf,
                 "plan": plan.as_dict()}
            rows.append(r)
            print(f"[size] N={n} {name}: {'in core' if r['in_core'] else 'out of core'} {t:.4f}s {tf:.2f} TFLOP/s "
                  f"{plan}", flush=True)
    with open(args.report, "w") as f:
        json.dump({"budget_bytes": budget, "in_core_limit": in_core_limit(budget), "rows": rows}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
