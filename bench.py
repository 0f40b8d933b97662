#!/usr/bin/env python3
"""Benchmark of the separated-operator apply on one MI355X.

One step = one pass of the whole hot path over one synthetic function: filter-up with
block norms, norm screening and planning, transform-and-accumulate, sum-down, and the
norm2 reduction of the result.  Inputs (the projected function and the operator with its
block cache, built during warm-up) are resident in HBM when the timed region starts.

Prints one JSON line: useful GFLOP/s (sum over kept triples of 6(2k)^4 + 6k^4 [n>0]),
boxes/s, the roofline of the dominant kernel (timed with HIP events on the library's
stream) and the FP64 oracle timed on a bounded sample on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import mra_workloads as W  # noqa: E402

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 (vector and matrix), AMD published
METRIC = "useful operator-apply GFLOP/s and boxes/s, mixed-prec batched vs FP64 @ err≤10*thresh"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="coulomb_k10",
                   choices=["coulomb_k10", "coulomb_k12_fp64", "bsh_batch_k10"])
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="approximate CPU work of the oracle baseline sample (0 = skip)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a device-to-device copy of MIB MiB (for calibrating HBM "
                        "byte counters of a profiler against a transfer of known size)")
    return p.parse_args()


def copy_calibration(mib):
    import torch
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "check": float(b[n // 2].item())}))


def cpu_baseline(name, budget_s):
    """The FP64 oracle (NumPy) timed on the host on a bounded sample of the same workload:
    whole source levels of the non-standard apply, coarsest first, until the budget is used."""
    from threadpoolctl import threadpool_info
    from oracle.apply import SeparatedOperator, nonstandard_contributions, filter_up
    from oracle.blocks import BlockFactory
    from oracle.fit import coulomb_fit, cell_r_hi
    from oracle.projection import GaussianSum, project_adaptive

    w = W.WORKLOADS[name]
    c, a, x = W.coulomb_inputs(name, 0)
    fo = project_adaptive(GaussianSum(c, a, x), w["k"], w["thresh"], W.CELL, w["initial_level"], 20)
    cc, tt = coulomb_fit(w["r_lo"], w["eps"], cell_r_hi(*W.CELL))
    op = SeparatedOperator(cc, tt)
    levels = filter_up(fo)
    bf = BlockFactory(w["k"], W.CELL[1] - W.CELL[0])
    flops, secs, done = 0.0, 0.0, []
    for n in sorted(levels):
        t0 = time.perf_counter()
        _, _, st = nonstandard_contributions(fo, op, w["tau_rel"] * w["thresh"], only_levels={n},
                                             levels=levels, blocks=bf)
        secs += time.perf_counter() - t0
        flops += st["useful_flops"]
        done.append(n)
        if secs >= budget_s:
            break
    threads = sum(i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas")
    return {"value": flops / secs / 1e9, "unit": "GFLOP/s", "cores": max(1, threads),
            "kind": "oracle",
            "sample": "source levels %s of the non-standard apply (%.1f useful GFLOP, %.1f s; "
                      "block quadrature included)" % (done, flops / 1e9, secs)}


def setup(ctx, name):
    """Functions, operators and tau for a workload; returns (funcs, ops, tau, k, config)."""
    if name == "bsh_batch_k10":
        w = W.WORKLOADS[name]
        funcs, ops, mus, ng = [], [], [], []
        for i in range(w["n_funcs"]):
            c, a, x, mu = W.bsh_inputs(i)
            funcs.append(ctx.project(c, a, x, w["k"], w["thresh"], initial_level=w["initial_level"]))
            ops.append(ctx.op_bsh(w["k"], mu, w["r_lo"], w["eps"]))
            mus.append(mu)
            ng.append(len(c))
        cfg = {"workload": name, "k": w["k"], "thresh": w["thresh"], "functions": w["n_funcs"],
               "gaussians_per_function": [min(ng), max(ng)], "operator": "bsh exp(-mu r)/r",
               "mu_range": [min(mus), max(mus)], "eps_fit": w["eps"], "r_lo": w["r_lo"],
               "tau_drop": w["tau_rel"] * w["thresh"], "precision": "fp64",
               "launch": "one batched apply (all functions per kernel launch)"}
        return funcs, ops, w["tau_rel"] * w["thresh"], w["k"], cfg
    base = "coulomb_k12_mixed" if name == "coulomb_k12_fp64" else name
    w = W.WORKLOADS[base]
    c, a, x = W.coulomb_inputs(base, 0)
    f = ctx.project(c, a, x, w["k"], w["thresh"], initial_level=w["initial_level"])
    op = ctx.op_coulomb(w["k"], w["r_lo"], w["eps"])
    cfg = {"workload": name, "k": w["k"], "thresh": w["thresh"], "gaussians": w["n_gauss"],
           "operator": "coulomb", "terms": int(op.terms()[0].size), "eps_fit": w["eps"],
           "r_lo": w["r_lo"], "tau_drop": w["tau_rel"] * w["thresh"], "precision": "fp64"}
    return [f], [op], w["tau_rel"] * w["thresh"], w["k"], cfg


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when the summary was taken on a different version of the kernel source."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1507_01888_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_pmc.md")):
        for line in open(path):
            if line.startswith("pmc: "):
                rec = json.loads(line[5:])
                if rec.get("kernel") == kernel and rec.get("kernels_hip_sha256_16") == sha:
                    return 1024.0 * (rec["fetch_kib"] * rec["fetch_factor"]
                                     + rec["write_kib"] * rec["write_factor"])
    return None


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU; --gpus %d is not supported by this build "
              "(the multi-GPU sharding is a design note, not an implementation)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1507_01888_amd as M

    ctx = M.Context(0, W.CELL)
    funcs, ops, tau, k, cfg = setup(ctx, args.workload)

    def step():
        if len(funcs) == 1:
            gs = [ctx.apply(ops[0], funcs[0], tau_drop=tau)]
        else:
            gs = ctx.apply_batch(ops, funcs, tau_drop=tau)
        st = ctx.last_stats()
        nrm = [ctx.norm2(g) for g in gs]
        for g in gs:
            g.free()
        return st, nrm

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        st, nrm = step()
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    flops = sum(s["useful_flops"] for s in stats)
    # the main kernel applies the children blocks and (for k = 8, 10, 12) the fused level-n
    # subtraction, so its algorithmic work is the full useful flop count of the step
    fused = k in (8, 10, 12)
    kernel_flops = stats[0]["useful_flops"] if fused else stats[0]["triples"] * 6.0 * (2 * k) ** 4
    main_ms = sum(s["ms_main_kernel"] for s in stats) / len(stats)
    kname = {8: "apply_ns_mfma_kernel<8>", 10: "apply_ns_mfma_kernel<10>",
             12: "apply_ns_mfma_big_kernel<12>"}.get(k, "apply_ns_kernel<%d>" % k)
    achieved = kernel_flops / (main_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": flops / elapsed / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "boxes_per_s": stats[0]["in_leaves"] * args.steps / elapsed,
        "time_to_solution_ms": elapsed / args.steps * 1e3,
        "counts": {key: stats[0][key] for key in ("triples", "targets", "in_leaves", "out_nodes",
                                                   "out_leaves")},
        "stage_ms": {key: sum(s[key] for s in stats) / len(stats)
                     for key in ("ms_filter", "ms_plan", "ms_apply", "ms_main_kernel", "ms_sumdown")},
        "norm2": nrm[0] if len(nrm) == 1 else sum(v * v for v in nrm) ** 0.5,
        "roofline": {"kernel": kname,
                     "bound": "mfma" if k in (8, 10, 12) else "alu", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(kname)},
    }
    if args.cpu_seconds > 0 and args.workload == "coulomb_k10":
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
