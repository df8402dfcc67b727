#!/usr/bin/env python3
"""Benchmark of the out-of-core FP64 product on one MI355X.

One step is one complete out-of-core product C = alpha*A*B + beta*C: the
partitioned pipeline of host-to-device tile copies, FP64 MFMA tile kernels and
device-to-host C copies (every stage of the method), with A, B and C in
page-locked host memory and device memory capped by the workload's budget.
The reported value is end-to-end TFLOP/s, 2*M*N*K / t with t including all
transfers (the paper's measure, Section VI).

Prints ONE JSON line.  Default workload: M = N = K = 32768 (8 GiB per matrix),
alpha = 1.5, beta = 0.5, entries uniform[-1, 1], device budget 4 GiB.  Beside
the FP64 figures the line carries two split legs on the same operands, the
split-BF16 form and the split-INT8 form, each with the smallest slice count
whose result meets the 1e-12 gate on the oracle's sampled rows.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "OOC DGEMM end-to-end TFLOP/s, FP64 vs split-BF16 at equal error; link GB/s"
PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak
PEAK_INT8_TOPS = 5000.0  # MI355X dense INT8 matrix peak (TOP/s)
LINK_PEAK_GBPS = 63.0  # PCIe 5.0 x16, one direction (32 GT/s x 16 lanes, 128b/130b)
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["paper_1808_05056_amd/csrc/dgemm_f64_kernel.hpp", "paper_1808_05056_amd/csrc/dgemm_f64.hip"]
SPLIT_SOURCES = ["paper_1808_05056_amd/csrc/split_bf16.hip"]


def kernel_source_hash(sources=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha1()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def measured_traffic(workload, plan):
    """HBM bytes per launch of the tile kernel from the committed rocprofv3 counter
    summary for this workload and plan, if it was taken on the current kernel source."""
    import re
    path = os.path.join(ROOT, "profiles", f"dgemm_f64_mfma_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)\s+kernel_source:\s*([0-9a-f]+)\s+plan:\s*(\S+)", text)
    if not m or m.group(2) != kernel_source_hash() or m.group(3) != plan:
        return None
    return float(m.group(1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="square-32768-budget-4GiB")
    ap.add_argument("--planner", default="model", choices=["model", "paper", "mlp", "sweep"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "split", "split-int8"])
    ap.add_argument("--slices", type=int, default=6)
    ap.add_argument("--cpu-rows", type=int, default=128, help="rows of C the CPU reference computes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", type=int, default=1, help="time every op with HIP events in the timed steps")
    ap.add_argument("--split-leg", type=int, default=1, help="1: also time the split-BF16 form (FP64 runs only)")
    ap.add_argument("--split-slices", default="4,5,6",
                    help="slice counts tried for the split leg, smallest first; the first to meet the gate is timed")
    ap.add_argument("--int8-leg", type=int, default=1, help="1: also time the split-INT8 form (FP64 runs only)")
    ap.add_argument("--int8-slices", default="5,6,7",
                    help="slice counts tried for the split-INT8 leg, smallest first; the first to meet the gate is timed")
    ap.add_argument("--copy-kernel", type=int, default=0, metavar="BYTES",
                    help="only run the library's device copy kernel once on BYTES (traffic-counter reference)")
    args = ap.parse_args()
    if args.copy_kernel:
        import paper_1808_05056_amd as ooc
        src, dst = ooc.DeviceBuffer(args.copy_kernel), ooc.DeviceBuffer(args.copy_kernel)
        ooc.ooc_device_copy(dst.ptr, src.ptr, args.copy_kernel)
        print(json.dumps({"copy_kernel_bytes": args.copy_kernel}))
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the out-of-core product is "
              f"measured per GPU, see the design notes for how it would shard", file=sys.stderr)
        sys.exit(2)

    import synth
    from synth import workloads as W
    import paper_1808_05056_amd as ooc

    if not os.path.exists(ooc.LIB_PATH):
        raise SystemExit("libooc.so is not built")
    w = W.BY_NAME[args.workload]
    planner = {"model": ooc.PLAN_MODEL, "paper": ooc.PLAN_PAPER, "mlp": ooc.PLAN_MLP, "sweep": ooc.PLAN_SWEEP}[args.planner]
    prec = {"fp64": ooc.FP64, "split": ooc.SPLIT_BF16, "split-int8": ooc.SPLIT_INT8}[args.precision]
    opts = ooc.make_opts(planner=planner, precision=prec, slices=args.slices if prec else 0)
    popts = ooc.make_opts(planner=planner, precision=prec, slices=args.slices if prec else 0,
                          profile=bool(args.profile))

    log(f"[bench] workload {w.name}: M={w.M} N={w.N} K={w.K} budget={w.budget / 2**30:.2f} GiB; "
        f"allocating {w.host_bytes() / 2**30:.1f} GiB page-locked host memory")
    t0 = time.time()
    Am = ooc.PinnedMatrix(w.M, w.K)
    Bm = ooc.PinnedMatrix(w.K, w.N)
    Cm = ooc.PinnedMatrix(w.M, w.N)
    A, B, C = Am.array, Bm.array, Cm.array
    synth.fill(A, w.spec_a())
    synth.fill(B, w.spec_b())
    synth.fill(C, w.spec_c())
    log(f"[bench] inputs ready in {time.time() - t0:.1f}s")

    # first call: checked against the CPU reference on sampled rows
    st, s1 = ooc.ooc_gemm(w.alpha, A, B, w.beta, C, w.budget, opts)
    plan = s1.plan
    log(f"[bench] plan {plan}; first call {s1.t_total_s:.3f}s (planning {s1.t_plan_s * 1e3:.1f} ms)")
    cpu = None
    ref = rows = D = Cin = None
    err = (None, None)
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(0)
        rows = np.unique(np.concatenate([[0, w.M - 1], rng.integers(0, w.M, args.cpu_rows)]))[: args.cpu_rows]
        if w.beta != 0.0:
            Cin = np.empty((len(rows), w.N))
            synth.fill_rows(Cin, rows, w.spec_c())
        tc = time.time()
        ref, D = oracle.gemm_rows(w.alpha, A, B, w.beta, Cin, rows=rows)
        tcpu = time.time() - tc
        err = oracle.errors(C[rows], ref, w.alpha, D, w.beta, Cin)
        flops = 2.0 * len(rows) * w.N * w.K
        cpu = {"value": flops / tcpu / 1e12, "unit": "TFLOP/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": f"{len(rows)} of {w.M} rows of C ({flops:.3e} flop) in {tcpu:.1f}s; "
                         f"the same plain triple loop extrapolates to {tcpu * w.M / len(rows):.0f}s for the whole product"}
        log(f"[bench] CPU reference: {len(rows)} rows in {tcpu:.1f}s, error literal {err[0]:.3e} "
            f"generalised {err[1]:.3e}")

    leg = run_leg(ooc, w, A, B, C, opts, popts, args, prec, args.slices)
    leg["first_call_plan_s"] = round(s1.t_plan_s, 6)
    roof, link = leg.pop("roofline"), leg.pop("link")
    e2e = leg.pop("end_to_end_roofline")

    split = split8 = None
    if args.split_leg and prec == ooc.FP64:
        split = split_leg(ooc, synth, w, A, B, C, args, ref, rows, D, Cin, ooc.SPLIT_BF16, args.split_slices)
    if args.int8_leg and prec == ooc.FP64:
        split8 = split_leg(ooc, synth, w, A, B, C, args, ref, rows, D, Cin, ooc.SPLIT_INT8, args.int8_slices)

    out = {
        "metric": METRIC, "value": leg["value"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": leg["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": ("f64" if prec == ooc.FP64 else
                                                 f"split-{'bf16' if prec == ooc.SPLIT_BF16 else 'int8'}x{args.slices}"),
        "data": "synthetic (seeded counter-based generator)",
        "config": {"workload": w.name, "M": w.M, "N": w.N, "K": w.K, "alpha": w.alpha, "beta": w.beta,
                   "budget_bytes": w.budget, "planner": args.planner, "plan": plan.as_dict(),
                   "arena_bytes": int(s1.arena_bytes), "parallelism": "single GPU"},
        "roofline": roof, "cpu_baseline": cpu, "link": link, "end_to_end_roofline": e2e,
        "max_error_literal": err[0], "max_normalized_error": err[1],
        "timing": {"ci95_rel": leg["ci95_rel"], "planning_first_call_s": leg["first_call_plan_s"],
                   "planning_per_step_s": leg["plan_s"], "overlap": leg["overlap"]},
        "predicted_s": round(s1.t_predicted_s, 4),
        "split_bf16": split,
        "split_int8": split8,
    }
    if split and split.get("value"):
        out["split_vs_fp64"] = round(split["value"] / leg["value"], 4)
    if split8 and split8.get("value"):
        out["split_int8_vs_fp64"] = round(split8["value"] / leg["value"], 4)
    print(json.dumps(out), flush=True)
    for m in (Am, Bm, Cm):
        m.free()
    ooc.ooc_release(-1)


def ci95_rel(times):
    """Half-width of the 95 % confidence interval of the mean step time (Student's t),
    relative to the mean: the paper repeats until this is at most 2.5 % (Section VI)."""
    n = len(times)
    if n < 2:
        return None
    from scipy import stats as sst
    m = float(np.mean(times))
    sd = float(np.std(times, ddof=1))
    return round(float(sst.t.ppf(0.975, n - 1)) * sd / np.sqrt(n) / m, 5)


def run_leg(ooc, w, A, B, C, opts, popts, args, prec, slices):
    """Warmup and timed steps of one form through ooc_gemm (planning included in
    every step's time; the plan choice is cached after the first call)."""
    for i in range(args.warmup):
        ooc.ooc_gemm(w.alpha, A, B, w.beta, C, w.budget, opts)
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    times, kbusy, hbusy, dbusy, mbusy, tplan, ovl = [], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0
    nkern = nmma = 0
    s = None
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        _, s = ooc.ooc_gemm(w.alpha, A, B, w.beta, C, w.budget, popts)
        times.append(time.perf_counter() - t0)
        kbusy += s.t_kernel_busy_s
        hbusy += s.t_h2d_busy_s
        dbusy += s.t_d2h_busy_s
        mbusy += s.t_mma_busy_s
        nmma += s.mma_launches
        tplan += s.t_plan_s
        ovl += s.overlap
        nkern += s.kernels
        log(f"[bench] step {i + 1}/{args.steps}: {times[-1]:.3f}s {w.flops / times[-1] / 1e12:.2f} TFLOP/s")
    elapsed = time.perf_counter() - t_start
    value = w.flops * args.steps / elapsed / 1e12
    plan = s.plan
    roof = None
    if args.profile and mbusy > 0:
        plan_tag = "{mb}x{nb}x{kb}/o{order}".format(**plan.as_dict())
        if prec == ooc.FP64:
            peak, work, kname = PEAK_FP64_TFLOPS, w.flops, "dgemm_f64_mfma"
            traffic = measured_traffic(w.name, plan_tag)
        else:  # BF16 or INT8 matrix work of the slice products, slicing kernels excluded
            if prec == ooc.SPLIT_BF16:
                peak, kname = PEAK_BF16_TFLOPS, "split_gemm"
            else:  # the tile width the library takes for a full block of the plan
                wide = ooc.ooc_split_int8_wide_tiles(min(plan.mb, w.M), min(plan.nb, w.N), 256)
                peak, kname = PEAK_INT8_TOPS, "split_gemm_i8w" if wide == 1 else "split_gemm_i8"
            work = w.flops * slices * (slices + 1) / 2
            traffic = None
        achieved = work * args.steps / mbusy / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TOP/s" if prec == ooc.SPLIT_INT8 else "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel_source": kernel_source_hash(KERNEL_SOURCES if prec == ooc.FP64 else SPLIT_SOURCES),
                "plan_tag": plan_tag, "kernel": kname, "launches_per_step": nmma // args.steps,
                "avg_launch_ms": round(mbusy / nmma * 1e3, 4),
                "op_busy_frac": round(kbusy / elapsed, 3)}
    link = None
    if args.profile and hbusy > 0:
        link = {"h2d_GBps": round(s.bytes_h2d * args.steps / hbusy / 1e9, 2),
                "d2h_GBps": round(s.bytes_d2h * args.steps / dbusy / 1e9, 2) if dbusy > 0 else None,
                "h2d_bytes_per_step": int(s.bytes_h2d), "d2h_bytes_per_step": int(s.bytes_d2h),
                "h2d_busy_frac": round(hbusy / elapsed, 3), "kernel_busy_frac": round(kbusy / elapsed, 3),
                "h2d_frac_of_link_peak": round(s.bytes_h2d * args.steps / hbusy / 1e9 / LINK_PEAK_GBPS, 3)}
    # end-to-end roofline: min(matrix peak, link peak x the plan's flops per host-to-device byte)
    ai = w.flops / max(s.bytes_h2d, 1)
    compute_peak = (PEAK_FP64_TFLOPS if prec == ooc.FP64  # FP64-equivalent
                    else (PEAK_BF16_TFLOPS if prec == ooc.SPLIT_BF16 else PEAK_INT8_TOPS)
                    / (slices * (slices + 1) / 2))
    e2e_roof = min(compute_peak, ai * LINK_PEAK_GBPS * 1e9 / 1e12)
    e2e = {"tflops": round(e2e_roof, 3), "flop_per_h2d_byte": round(ai, 2), "link_peak_GBps": LINK_PEAK_GBPS,
           "frac": round(value / e2e_roof, 4)}
    return {"value": round(value, 3), "ms_per_step": round(elapsed / args.steps * 1e3, 2),
            "ci95_rel": ci95_rel(times), "plan_s": round(tplan / args.steps, 6),
            "overlap": round(ovl / args.steps, 4) if args.profile else None,
            "plan": plan.as_dict(), "roofline": roof, "link": link, "end_to_end_roofline": e2e}


def split_leg(ooc, synth, w, A, B, C, args, ref, rows, D, Cin, prec, slice_list):
    """A split form (BF16 or INT8 slices) on the same workload and operands: the
    smallest slice count (from slice_list) whose result meets the gate on the
    oracle's sampled rows (literal metric when beta == 0, generalised
    otherwise), timed like the FP64 leg."""
    import oracle
    tag = "bf16" if prec == ooc.SPLIT_BF16 else "int8"
    chosen, tried = None, []
    for sl in (int(x) for x in slice_list.split(",")):
        if w.beta != 0.0:
            synth.fill(C, w.spec_c())
        o = ooc.make_opts(planner=ooc.PLAN_MODEL, precision=prec, slices=sl)
        _, st = ooc.ooc_gemm(w.alpha, A, B, w.beta, C, w.budget, o)
        lit, gen = oracle.errors(C[rows], ref, w.alpha, D, w.beta, Cin) if ref is not None else (None, None)
        gated = lit if w.beta == 0.0 else gen
        tried.append({"slices": sl, "error_literal": lit, "error_generalised": gen,
                      "first_call_s": round(st.t_total_s, 4)})
        log(f"[bench] split-{tag.upper()} s={sl}: plan {st.plan} {st.t_total_s:.3f}s error literal "
            f"{lit if lit is None else f'{lit:.3e}'} generalised {gen if gen is None else f'{gen:.3e}'}")
        if gated is not None and gated <= oracle.GATE:
            chosen = (sl, lit, gen)
            break
    if chosen is None:
        return {"value": None, "tried": tried, "note": "no slice count met the gate"}
    sl = chosen[0]
    o = ooc.make_opts(planner=ooc.PLAN_MODEL, precision=prec, slices=sl)
    po = ooc.make_opts(planner=ooc.PLAN_MODEL, precision=prec, slices=sl, profile=bool(args.profile))
    leg = run_leg(ooc, w, A, B, C, o, po, args, prec, sl)
    leg.update({"dtype": f"split-{tag}x{sl}", "slices": sl, "error_literal": chosen[1],
                "error_generalised": chosen[2], "tried": tried})
    return leg


if __name__ == "__main__":
    main()
