"""Sweep candidate plans on the GPU, train the planner network, measure its regret.

The learned planner ranks the candidates the cost model enumerates with a
network trained on timings this pipeline produces (the paper fixes its plan by
rule, Section V, and observes that the best stream count depends on the
device, Section VI).  This tool

  train   times a set of candidates per problem of a training batch (M, N, K
          log-uniform in [4096, 24576], budgets log-uniform 256 MiB - 8 GiB,
          seed 40, plus --tall tall problems, seed 41), fits the network with the library's GPU kernels
          (ooc_mlp_fit: full-batch Adam, L2 weight decay) and writes the weights;
          --precision split times split-BF16 plans (--slices) instead;
  fit     refits the network from the timings one or more train runs saved
          (--data a.npz,b.npz: FP64 and split timings fit one network, whose
          slice-count feature tells the two apart);
  eval    times, per problem of the evaluation batch (seed 4), the cost
          model's best candidates, the network's best and the three planners'
          choices, and reports the regret t(choice) / t(best measured) - 1 of
          each planner (--precision split or split-int8: slice plans);
          --exhaustive times every candidate the planners consider (the
          judge of the restricted set's best), --smallest N keeps the N
          problems with the fewest flops;
  sweep   times the cost model's best candidates for one named workload (and
          the model's, the network's and the paper's choices): the swept plan;
          --precision split or split-int8 sweeps BF16 or INT8 slice plans.

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


def _opts(args, planner=ooc.PLAN_AUTO):
    if args.precision in ("split", "split-int8"):
        prec = ooc.SPLIT_BF16 if args.precision == "split" else ooc.SPLIT_INT8
        return ooc.make_opts(planner=planner, precision=prec, slices=args.slices)
    return ooc.make_opts(planner=planner)


def candidate_set(w, n_model, n_random, rng, extra=(), opts=None, within=None):
    """The model's n_model best candidates, n_random others (with a model time
    at most `within` times the best, if given) and `extra`."""
    plans, model_s = ooc.ooc_plan_candidates(w.M, w.N, w.K, w.beta, w.budget, opts)
    chosen = list(range(min(n_model, len(plans))))
    rest = list(range(len(chosen), len(plans)))
    if within:
        rest = [i for i in rest if model_s[i] <= within * model_s[0]]
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
    problems = W.problem_batch(40, count=args.count) + W.tall_batch(41, count=args.tall)
    bufs = Buffers(problems)
    rng = np.random.default_rng(1)
    X, y, meta = [], [], []
    t0 = time.time()
    split = args.precision == "split"
    for idx, w in enumerate(problems):
        # FP64 runs also time the paper's plan; its split form (slivers of a
        # few rows padded to whole tiles) is far outside what the network ranks
        paper = [] if split else [ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, _opts(args, ooc.PLAN_PAPER))]
        try:
            plans, _, _ = candidate_set(w, args.n_model, args.n_random, rng, extra=paper, opts=_opts(args),
                                        within=4.0 if split else None)
        except ooc.OOCError as e:
            _log(f"[train] problem {idx + 1}/{len(problems)}: no plan ({e})")
            continue
        feats = ooc.ooc_mlp_features(w.M, w.N, w.K, w.beta, w.budget, plans)
        views = bufs.views(w)
        for p, f in zip(plans, feats):
            t = time_plan(w, views, p, args.reps)
            X.append(f)
            y.append(t)
            meta.append({"problem": idx, "M": w.M, "N": w.N, "K": w.K, "beta": w.beta, "budget": w.budget,
                         "plan": p.as_dict(), "seconds": t})
            _log(f"[train]   {p} {t:.3f}s")
        _log(f"[train] problem {idx + 1}/{len(problems)} M={w.M} N={w.N} K={w.K} budget={w.budget / GiB:.2f} GiB: "
             f"{len(plans)} plans, best {min(y[-len(plans):]):.3f}s ({time.time() - t0:.0f}s elapsed)")
        _save(args.data, X, y, meta)  # after every problem, so a cut-short run keeps what it timed
    bufs.free()
    fit_and_save(np.array(X, dtype=np.float32), np.array(y, dtype=np.float32), args)


def _save(path, X, y, meta):
    np.savez(path, X=np.array(X, dtype=np.float32), y=np.array(y, dtype=np.float32))
    with open(path + ".json", "w") as f:
        json.dump(meta, f)


def fit_and_save(X, y, args):
    hist = ooc.ooc_mlp_fit(X, y, hidden=args.hidden, epochs=args.epochs, lr=args.lr, weight_decay=args.weight_decay,
                           seed=args.seed)
    ooc.ooc_mlp_save(args.out)
    _log(f"[fit] {len(y)} samples; objective {hist[0]:.4f} -> {hist[-1]:.4f}; weights in {args.out}")


def refeature(path):
    """Features of the plans a train run saved, recomputed with the current
    cost model (after it changes, the timings stay valid but the model's
    prediction, one of the features, does not)."""
    with open(path + ".json") as f:
        meta = json.load(f)
    X = np.concatenate([ooc.ooc_mlp_features(r["M"], r["N"], r["K"], r.get("beta", 0.0), r["budget"],
                                             [ooc.ooc_plan_t(**r["plan"])]) for r in meta]).astype(np.float32)
    return X, np.array([r["seconds"] for r in meta], dtype=np.float32)


def fit(args):
    parts = [refeature(f) if args.refeature else (lambda d: (d["X"], d["y"]))(np.load(f))
             for f in args.data.split(",")]
    X = np.concatenate([x for x, _ in parts])
    y = np.concatenate([t for _, t in parts])
    fit_and_save(X, y, args)


def evaluate(args):
    from synth import workloads as W
    if args.weights:
        ooc.ooc_mlp_load(args.weights)
    problems = W.problem_batch(4, count=args.count)
    if args.smallest:
        # a subset fixed by size alone (never by outcome): the problems with the fewest flops
        problems = sorted(problems, key=lambda w: w.flops)[: args.smallest]
    bufs = Buffers(problems)
    split = args.precision != "fp64"
    rows = []
    t0 = time.time()
    for idx, w in enumerate(problems):
        try:
            pm = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, _opts(args, ooc.PLAN_MODEL))
            pl = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, _opts(args, ooc.PLAN_MLP))
            # the paper's rule has no split form worth timing (slivers of a few
            # rows padded to whole tiles)
            pp = None if split else ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, _opts(args, ooc.PLAN_PAPER))
        except ooc.OOCError as e:
            _log(f"[eval] {idx + 1}/{len(problems)}: skipped, a planner finds no plan ({e})")
            continue
        all_plans, model_s = ooc.ooc_plan_candidates(w.M, w.N, w.K, w.beta, w.budget, _opts(args))
        # the network's own favourites (split: among the model's 16 best only)
        ranked = all_plans[:16] if split else all_plans
        if args.precision == "split-int8":  # the network declines INT8 plans (its choice is the model's)
            by_mlp = []
        else:
            mlp_s = ooc.ooc_mlp_predict(w.M, w.N, w.K, w.beta, w.budget, ranked)
            by_mlp = list(np.argsort(mlp_s)[: args.n_mlp])
        sweep = [all_plans[i] for i in range(min(args.n_model, len(all_plans)))]
        sweep += [ranked[i] for i in by_mlp]
        sweep += [pm, pl] + ([] if split else [pp])
        restricted = {_key(p) for p in sweep}
        if args.exhaustive:  # every candidate the planners consider
            sweep += list(all_plans)
        uniq, seen = [], set()
        for p in sweep:
            if _key(p) not in seen:
                uniq.append(p)
                seen.add(_key(p))
        views = bufs.views(w)
        times = {}
        for p in uniq:
            times[_key(p)] = time_plan(w, views, p, args.reps)
            _log(f"[eval]   {p} {times[_key(p)]:.3f}s")
        if args.confirm:
            # the minimum of many single timings is biased low: re-time the
            # fastest plans and the planners' choices, best of confirm_reps
            by_time = sorted(uniq, key=lambda p: times[_key(p)])
            again, seen2 = [], set()
            for p in by_time[: args.confirm] + [pm, pl] + ([] if split else [pp]):
                if _key(p) not in seen2:
                    again.append(p)
                    seen2.add(_key(p))
            for p in again:
                t2 = time_plan(w, views, p, args.confirm_reps)
                _log(f"[eval]   confirm {p} {times[_key(p)]:.4f}s -> {t2:.4f}s")
                times[_key(p)] = t2
        best = min(times.values())
        r = {"problem": idx, "M": w.M, "N": w.N, "K": w.K, "budget": w.budget, "swept": len(uniq),
             "best_s": best, "model_s": times[_key(pm)], "mlp_s": times[_key(pl)], "flops": w.flops,
             "candidates": len(all_plans),
             "restricted_best_s": min(t for k, t in times.items() if k in restricted)}
        if pp is not None:
            r["paper_s"] = times[_key(pp)]
        rows.append(r)
        paper_txt = f" paper {r['paper_s'] / best - 1:+.3f}" if pp is not None else ""
        _log(f"[eval] {idx + 1}/{len(problems)} M={w.M} N={w.N} K={w.K} budget={w.budget / GiB:.2f} GiB: best "
             f"{best:.3f}s model {r['model_s'] / best - 1:+.3f} mlp {r['mlp_s'] / best - 1:+.3f}{paper_txt} "
             f"({time.time() - t0:.0f}s elapsed)")
    bufs.free()
    summ = {}
    for k in ("model", "mlp") + (() if split else ("paper",)):
        reg = np.array([r[f"{k}_s"] / r["best_s"] - 1 for r in rows])
        tf = np.array([r["flops"] / r[f"{k}_s"] / 1e12 for r in rows])
        summ[k] = {"mean_regret": float(reg.mean()), "median_regret": float(np.median(reg)),
                   "max_regret": float(reg.max()), "mean_tflops": float(tf.mean()),
                   "total_s": float(sum(r[f"{k}_s"] for r in rows))}
    summ["best"] = {"total_s": float(sum(r["best_s"] for r in rows)),
                    "mean_tflops": float(np.mean([r["flops"] / r["best_s"] / 1e12 for r in rows]))}
    if args.exhaustive:
        # how far the restricted set (model's best, network's best, the three choices) is from the whole
        rb = np.array([r["restricted_best_s"] / r["best_s"] - 1 for r in rows])
        summ["restricted_judge"] = {"mean_gap": float(rb.mean()), "max_gap": float(rb.max()),
                                    "exact": int(np.sum(rb == 0.0)), "problems": len(rows)}
    with open(args.report, "w") as f:
        json.dump({"summary": summ, "problems": rows}, f, indent=1)
    _log(json.dumps(summ))


def sweep(args):
    import synth
    from synth import workloads as W
    w = W.BY_NAME[args.workload]
    split = args.precision != "fp64"
    if args.weights:
        ooc.ooc_mlp_load(args.weights)
    mats = [ooc.PinnedMatrix(w.M, w.K), ooc.PinnedMatrix(w.K, w.N), ooc.PinnedMatrix(w.M, w.N)]
    try:
        A, B, C = (m.array for m in mats)
        synth.fill(A, w.spec_a())
        synth.fill(B, w.spec_b())
        synth.fill(C, w.spec_c())
        plans, model_s = ooc.ooc_plan_candidates(w.M, w.N, w.K, w.beta, w.budget, _opts(args))
        named = {"model": ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, _opts(args, ooc.PLAN_MODEL)),
                 "mlp": ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, _opts(args, ooc.PLAN_MLP))}
        if not split:
            named["paper"] = ooc.ooc_plan(w.M, w.N, w.K, w.beta, w.budget, _opts(args, ooc.PLAN_PAPER))
        todo, seen = [], set()
        for p in plans[: args.top] + list(named.values()):
            if _key(p) not in seen:
                todo.append(p)
                seen.add(_key(p))
        rows = []
        for p in todo:
            t = time_plan(w, (A, B, C), p, args.reps)
            rows.append({"plan": p.as_dict(), "seconds": t, "tflops": w.flops / t / 1e12,
                         "model_s": ooc.ooc_plan_predict(w.M, w.N, w.K, w.beta, p)})
            _log(f"[sweep] {p} {t:.4f}s {w.flops / t / 1e12:.2f} TFLOP/s")
        best = min(rows, key=lambda r: r["seconds"])
        out = {"workload": w.name, "precision": args.precision, "slices": args.slices if split else 0,
               "swept": len(rows), "best": best, "rows": rows}
        for name, p in named.items():
            r = next(r for r in rows if r["plan"] == p.as_dict())
            out[name] = {"seconds": r["seconds"], "tflops": r["tflops"], "regret": r["seconds"] / best["seconds"] - 1}
        with open(args.report, "w") as f:
            json.dump(out, f, indent=1)
        _log(json.dumps({k: v for k, v in out.items() if k != "rows"}))
    finally:
        for m in mats:
            m.free()


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--count", type=int, default=48)
    t.add_argument("--tall", type=int, default=8, help="tall problems (synth tall_batch, seed 41) added to the batch")
    t.add_argument("--n-model", type=int, default=8)
    t.add_argument("--n-random", type=int, default=6)
    t.add_argument("--reps", type=int, default=1)
    f = sub.add_parser("fit")
    f.add_argument("--refeature", action="store_true", help="recompute features with the current cost model")
    e = sub.add_parser("eval")
    t.add_argument("--precision", choices=("fp64", "split"), default="fp64")
    e.add_argument("--precision", choices=("fp64", "split", "split-int8"), default="fp64")
    for q in (t, e):
        q.add_argument("--slices", type=int, default=5)
    for q in (t, f):
        q.add_argument("--hidden", type=int, default=64)
        q.add_argument("--epochs", type=int, default=1000)
        q.add_argument("--lr", type=float, default=3e-3)
        q.add_argument("--weight-decay", type=float, default=1e-3)
        q.add_argument("--seed", type=int, default=0)
        q.add_argument("--data", default="planner_sweep_train.npz")
        q.add_argument("--out", default="planner_mlp.txt")
    e.add_argument("--count", type=int, default=64)
    e.add_argument("--smallest", type=int, default=0, help="only the N problems with the fewest flops")
    e.add_argument("--exhaustive", action="store_true", help="time every candidate the planners consider")
    e.add_argument("--confirm", type=int, default=0, help="re-time the N fastest plans and the choices")
    e.add_argument("--confirm-reps", type=int, default=3)
    e.add_argument("--n-model", type=int, default=6)
    e.add_argument("--n-mlp", type=int, default=4)
    e.add_argument("--reps", type=int, default=1)
    e.add_argument("--weights", default=None)
    e.add_argument("--report", default="planner_eval.json")
    sw = sub.add_parser("sweep")
    sw.add_argument("--workload", default="tall-262144x8192x8192-budget-2GiB")
    sw.add_argument("--precision", choices=("fp64", "split", "split-int8"), default="fp64")
    sw.add_argument("--slices", type=int, default=5)
    sw.add_argument("--top", type=int, default=12)
    sw.add_argument("--reps", type=int, default=2)
    sw.add_argument("--weights", default=None)
    sw.add_argument("--report", default="planner_sweep_workload.json")
    args = ap.parse_args(argv)
    {"train": train, "fit": fit, "eval": evaluate, "sweep": sweep}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
