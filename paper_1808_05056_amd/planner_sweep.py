"""Sweep candidate plans on the GPU, train the planner network, measure its regret.

The learned planner ranks the candidates the cost model enumerates with a
network trained on timings this pipeline produces (the paper fixes its plan by
rule, Section V, and observes that the best stream count depends on the
device, Section VI).  This tool

  train   times a set of candidates per problem of a training batch (M, N, K
          log-uniform in [4096, 24576], budgets log-uniform 256 MiB - 8 GiB,
          seed 40), fits the network with the library's GPU kernels
          (ooc_mlp_fit: full-batch Adam, L2 weight decay) and writes the weights;
  fit     refits the network from the timings a train run saved;
  eval    times every candidate of the evaluation batch (seed 4) that the cost
          model, the network or the paper's rule would consider, and reports
          the regret t(choice) / t(best measured) - 1 of each planner.

    python -m paper_1808_05056_amd.planner_sweep train --out planner_mlp.txt
    python -m paper_1808_05056_amd.planner_sweep eval --weights planner_mlp.txt

Timings are the pipeline time of ooc_gemm_planned (first op issued to last
op complete), best of `reps`, after one untimed call per plan.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

import paper_1808_05056_amd as ooc

GiB = 1 << 30


def _log(msg):
    print(msg, flush=True)


class Buffers:
    """Page-locked operands big enough for every problem of a batch (reused as views)."""

    def __init__(self, problems):
        self.cap = {k: max(getattr(w, a) * getattr(w, b) for w in problems)
                    for k, (a, b) in {"A": ("M", "K"), "B": ("K", "N"), "C": ("M", "N")}.items()}
        self.mats = {k: ooc.PinnedMatrix(1, v) for k, v in self.cap.items()}
        rng = np.random.default_rng(0)
        for k, m in self.mats.items():
            flat = m.array.reshape(-1)
            for s in range(0, flat.size, 1 << 26):
                flat[s:s + (1 << 26)] = rng.uniform(-1, 1, min(1 << 26, flat.size - s))

    def views(self, w):
        A = self.mats["A"].array.reshape(-1)[: w.M * w.K].reshape(w.M, w.K)
        B = self.mats["B"].array.reshape(-1)[: w.K * w.N].reshape(w.K, w.N)
        C = self.mats["C"].array.reshape(-1)[: w.M * w.N].reshape(w.M, w.N)
        return A, B, C

    def free(self):
        for m in self.mats.values():
            m.free()


def time_plan(w, views, plan, reps=1):
    A, B, C = views
    ooc.ooc_gemm_planned(w.alpha, A, B, w.beta, C, w.budget, plan)
    best = float("inf")
    for _ in range(reps):
        _, s = ooc.ooc_gemm_planned(w.alpha, A, B, w.beta, C, w.budget, plan)
        best = min(best, s.t_pipeline_s)
    return best


def _key(p):
    return tuple(p.as_dict().values())


def candidate_set(w, n_model, n_random, rng, extra=()):
    plans, model_s = ooc.ooc_plan_candidates(w.M, w.N, w.K, w.beta, w.budget)
    chosen = list(range(min(n_model, len(plans))))
    rest = list(range(len(chosen), len(plans)))
    if rest and n_random:
        chosen += list(rng.choice(rest, size=min(n_random, len(rest)), replace=False))
    out = [plans[i] for i in chosen]
    keys = {_key(p) for p in out}
    for p in extra:
        if _key(p) not in keys:
            out.append(p)
            keys.add(_key(p))
    return out, plans, model_s


def train(args):
    from synth import workloads as W
    problems = W.problem_batch(40, count=args.count)
    bufs = Buffers(problems)
    rng = np.random.default_rng(1)
    X, y, meta = [], [], []
    t0 = time.time()
    for idx, w in enumerate(problems):
        paper = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, ooc.make_opts(planner=ooc.PLAN_PAPER))
        plans, _, _ = candidate_set(w, args.n_model, args.n_random, rng, extra=[paper])
        feats = ooc.ooc_mlp_features(w.M, w.N, w.K, w.beta, w.budget, plans)
        views = bufs.views(w)
        for p, f in zip(plans, feats):
            t = time_plan(w, views, p, args.reps)
            X.append(f)
            y.append(t)
            meta.append({"problem": idx, "M": w.M, "N": w.N, "K": w.K, "budget": w.budget, "plan": p.as_dict(),
                         "seconds": t})
        _log(f"[train] problem {idx + 1}/{len(problems)} M={w.M} N={w.N} K={w.K} budget={w.budget / GiB:.2f} GiB: "
             f"{len(plans)} plans, best {min(y[-len(plans):]):.3f}s ({time.time() - t0:.0f}s elapsed)")
    bufs.free()
    X = np.array(X, dtype=np.float32)
    y = np.array(y, dtype=np.float32)
    np.savez(args.data, X=X, y=y)
    with open(args.data + ".json", "w") as f:
        json.dump(meta, f)
    fit_and_save(X, y, args)


def fit_and_save(X, y, args):
    hist = ooc.ooc_mlp_fit(X, y, hidden=args.hidden, epochs=args.epochs, lr=args.lr, weight_decay=args.weight_decay,
                           seed=args.seed)
    ooc.ooc_mlp_save(args.out)
    _log(f"[fit] {len(y)} samples; objective {hist[0]:.4f} -> {hist[-1]:.4f}; weights in {args.out}")


def fit(args):
    d = np.load(args.data)
    fit_and_save(d["X"], d["y"], args)


def evaluate(args):
    from synth import workloads as W
    if args.weights:
        ooc.ooc_mlp_load(args.weights)
    problems = W.problem_batch(4, count=args.count)
    bufs = Buffers(problems)
    rng = np.random.default_rng(2)
    rows = []
    t0 = time.time()
    for idx, w in enumerate(problems):
        pm = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, ooc.make_opts(planner=ooc.PLAN_MODEL))
        pl = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, ooc.make_opts(planner=ooc.PLAN_MLP))
        pp = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, ooc.make_opts(planner=ooc.PLAN_PAPER))
        all_plans, model_s = ooc.ooc_plan_candidates(w.M, w.N, w.K, w.beta, w.budget)
        mlp_s = ooc.ooc_mlp_predict(w.M, w.N, w.K, w.beta, w.budget, all_plans)
        by_mlp = list(np.argsort(mlp_s)[: args.n_mlp])
        sweep = [all_plans[i] for i in range(min(args.n_model, len(all_plans)))]
        sweep += [all_plans[i] for i in by_mlp]
        sweep += [pm, pl, pp]
        uniq, seen = [], set()
        for p in sweep:
            if _key(p) not in seen:
                uniq.append(p)
                seen.add(_key(p))
        views = bufs.views(w)
        times = {(_key(p)): time_plan(w, views, p, args.reps) for p in uniq}
        best = min(times.values())
        r = {"problem": idx, "M": w.M, "N": w.N, "K": w.K, "budget": w.budget, "swept": len(uniq),
             "best_s": best, "model_s": times[_key(pm)], "mlp_s": times[_key(pl)], "paper_s": times[_key(pp)],
             "flops": w.flops}
        rows.append(r)
        _log(f"[eval] {idx + 1}/{len(problems)} M={w.M} N={w.N} K={w.K} budget={w.budget / GiB:.2f} GiB: best "
             f"{best:.3f}s model {r['model_s'] / best - 1:+.3f} mlp {r['mlp_s'] / best - 1:+.3f} "
             f"paper {r['paper_s'] / best - 1:+.3f} ({time.time() - t0:.0f}s elapsed)")
    bufs.free()
    summ = {}
    for k in ("model", "mlp", "paper"):
        reg = np.array([r[f"{k}_s"] / r["best_s"] - 1 for r in rows])
        tf = np.array([r["flops"] / r[f"{k}_s"] / 1e12 for r in rows])
        summ[k] = {"mean_regret": float(reg.mean()), "median_regret": float(np.median(reg)),
                   "max_regret": float(reg.max()), "mean_tflops": float(tf.mean()),
                   "total_s": float(sum(r[f"{k}_s"] for r in rows))}
    summ["best"] = {"total_s": float(sum(r["best_s"] for r in rows)),
                    "mean_tflops": float(np.mean([r["flops"] / r["best_s"] / 1e12 for r in rows]))}
    with open(args.report, "w") as f:
        json.dump({"summary": summ, "problems": rows}, f, indent=1)
    _log(json.dumps(summ))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--count", type=int, default=48)
    t.add_argument("--n-model", type=int, default=8)
    t.add_argument("--n-random", type=int, default=6)
    t.add_argument("--reps", type=int, default=1)
    f = sub.add_parser("fit")
    for q in (t, f):
        q.add_argument("--hidden", type=int, default=64)
        q.add_argument("--epochs", type=int, default=1000)
        q.add_argument("--lr", type=float, default=3e-3)
        q.add_argument("--weight-decay", type=float, default=1e-3)
        q.add_argument("--seed", type=int, default=0)
        q.add_argument("--data", default="planner_sweep_train.npz")
        q.add_argument("--out", default="planner_mlp.txt")
    e = sub.add_parser("eval")
    e.add_argument("--count", type=int, default=64)
    e.add_argument("--n-model", type=int, default=6)
    e.add_argument("--n-mlp", type=int, default=4)
    e.add_argument("--reps", type=int, default=1)
    e.add_argument("--weights", default=None)
    e.add_argument("--report", default="planner_eval.json")
    args = ap.parse_args(argv)
    {"train": train, "fit": fit, "eval": evaluate}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
