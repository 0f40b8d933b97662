#!/usr/bin/env python3
"""Benchmark of the separated-operator apply on one MI355X.

One step = one pass of the whole hot path over one synthetic function (or batch): filter-up
with block norms, norm screening and planning, transform-and-accumulate, sum-down, and the
norm2 reduction of the result.  Inputs (the projected functions and the operators with
their block caches, built during warm-up) are resident in HBM when the timed region starts.

Prints one JSON line: useful GFLOP/s (sum over kept triples of 6(2k)^4 + 6k^4 [n>0]),
boxes/s, the roofline of the dominant kernel (timed with HIP events on the library's
stream) and the FP64 oracle timed on a bounded sample on the host cores.  The mixed
workload (low-precision tier for triples with eta < 1e-3 thresh) also times the all-FP64
path on the same input and reports the difference between the two results.
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
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix, AMD published
METRIC = "useful operator-apply GFLOP/s and boxes/s, mixed-prec batched vs FP64 @ err≤10*thresh"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="coulomb_k10",
                   choices=["gauss_std_k8", "coulomb_k10", "coulomb_k12_fp64",
                            "coulomb_k12_mixed", "bsh_batch_k10"])
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

    base = "coulomb_k12_mixed" if name.startswith("coulomb_k12") else name
    w = W.WORKLOADS[base]
    c, a, x = W.coulomb_inputs(base, 0)
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
    if name == "gauss_std_k8":
        w = W.WORKLOADS[name]
        f = ctx.project([w["f_coeff"]], [w["f_expnt"]], [[0.0, 0.0, 0.0]], w["k"], 1.0,
                        initial_level=w["level"], max_level=w["level"])
        op = ctx.op_gaussians(w["k"], w["op_c"], w["op_t"])
        cfg = {"workload": name, "k": w["k"], "level": w["level"], "boxes": 8 ** w["level"],
               "operator": "exp(-2 x^2)", "displacements": (2 * w["disp_radius"] + 1) ** 3,
               "form": "standard", "precision": "fp64"}
        return [f], [op], None, w["k"], cfg
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
    base = "coulomb_k12_mixed" if name.startswith("coulomb_k12") else name
    w = W.WORKLOADS[base]
    c, a, x = W.coulomb_inputs(base, 0)
    f = ctx.project(c, a, x, w["k"], w["thresh"], initial_level=w["initial_level"])
    op = ctx.op_coulomb(w["k"], w["r_lo"], w["eps"])
    cfg = {"workload": name, "k": w["k"], "thresh": w["thresh"], "gaussians": w["n_gauss"],
           "operator": "coulomb", "terms": int(op.terms()[0].size), "eps_fit": w["eps"],
           "r_lo": w["r_lo"], "tau_drop": w["tau_rel"] * w["thresh"], "precision": "fp64"}
    if name == "coulomb_k12_mixed":
        cfg["precision"] = "fp64 + bf16 tier (eta < tau_tier), fp32 accumulation"
        cfg["tau_tier"] = w["tier_rel"] * w["thresh"]
    return [f], [op], w["tau_rel"] * w["thresh"], w["k"], cfg


def kernel_source_sha(kernel):
    """sha256[:16] of the source of `kernel` (its definition up to the next section rule in
    kernels.hip), so that counters stay valid while other kernels of the file change."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_1507_01888_amd", "csrc", "kernels.hip")).read()
    base = kernel.split("<")[0]
    i = src.find(" void %s(" % base)
    if i < 0:
        return None
    i = src.rfind("\ntemplate", 0, i)
    j = src.find("\n// ---", i)
    return hashlib.sha256(src[i:j].encode()).hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when the summary was taken on a different version of the kernel's source."""
    import glob
    sha = kernel_source_sha(kernel)
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_pmc.md")):
        for line in open(path):
            if line.startswith("pmc: "):
                rec = json.loads(line[5:])
                if rec.get("kernel") == kernel and rec.get("kernel_src_sha256_16") == sha:
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
    tier = cfg.get("tau_tier", 0.0)

    def step(tau_tier, keep=False):
        if tau is None:     # standard form on a uniform tree, no screening
            gs = [ctx.apply(ops[0], funcs[0], form="standard",
                            disp_radius=W.WORKLOADS[args.workload]["disp_radius"])]
        elif len(funcs) == 1:
            gs = [ctx.apply(ops[0], funcs[0], tau_drop=tau, tau_tier=tau_tier)]
        else:
            gs = ctx.apply_batch(ops, funcs, tau_drop=tau, tau_tier=tau_tier)
        st = ctx.last_stats()
        nrm = [ctx.norm2(g) for g in gs]
        if keep:
            return st, nrm, gs
        for g in gs:
            g.free()
        return st, nrm

    def timed(tau_tier):
        for _ in range(args.warmup):
            step(tau_tier)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(args.steps):
            st, nrm = step(tau_tier)
            stats.append(st)
        torch.cuda.synchronize()
        return stats, nrm, time.perf_counter() - t0

    stats, nrm, elapsed = timed(tier)
    fp64_cmp = None
    if tier > 0:
        # the all-FP64 path on the same input, and the difference of the two results
        st64, _, el64 = timed(0.0)
        _, _, g_mix = step(tier, keep=True)
        _, _, g_64 = step(0.0, keep=True)
        import numpy as np
        km, cm = g_mix[0].export()
        k6, c6 = g_64[0].export()
        assert np.array_equal(km, k6)
        fp64_cmp = {"value": sum(s["useful_flops"] for s in st64) / el64 / 1e9,
                    "ms_per_step": el64 / args.steps * 1e3,
                    "ms_main_kernel": sum(s["ms_main_kernel"] for s in st64) / len(st64),
                    "speedup_mixed_vs_fp64": el64 / elapsed,
                    "rel_l2_mixed_vs_fp64": float(np.linalg.norm(cm - c6) / np.linalg.norm(c6))}

    flops = sum(s["useful_flops"] for s in stats)
    # algorithmic work of the main kernel: the FP64 mode products it executes (children
    # blocks and, for k = 8, 10, 12, 14, the fused level-n subtraction).  For k = 10 the
    # kernel shares the y- and z-products of a target's triples, so it executes fewer flops
    # than the useful count of its triples; both rates are reported.
    fused = k in (8, 10, 12, 14)
    kernel_flops = stats[0]["flops_kernel"]
    useful_main = stats[0]["useful_flops"] - stats[0]["flops_low"]
    main_ms = sum(s["ms_main_kernel"] for s in stats) / len(stats)
    kname = {8: "apply_ns_mfma_kernel<8>", 10: "apply_ns_fac_kernel<10>",
             12: "apply_ns_own_kernel<12>", 14: "apply_ns_stream_kernel<14>"}.get(
                 k, "apply_ns_kernel<%d>" % k)
    if tau is None:        # standard form: the VALU kernel does 6 k^4 flop per triple
        fused, kernel_flops, kname = False, stats[0]["useful_flops"], "apply_std_kernel<%d>" % k
        useful_main = kernel_flops
    achieved = kernel_flops / (main_ms * 1e-3) / 1e12
    low_ms = sum(s["ms_low_kernel"] for s in stats) / len(stats)
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
                     "bound": "mfma" if fused else "alu", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(kname),
                     "useful_tflops": useful_main / (main_ms * 1e-3) / 1e12,
                     "executed_over_useful": kernel_flops / useful_main},
    }
    if tier > 0:
        s0 = stats[0]
        # the BF16 kernel evaluates 7 mode products of (2k)^3 x 2k per triple (E R R + P E R
        # + P P E with the shared R_z and E_z products) and writes nothing but the target
        low_alg = s0["triples_low"] * 14.0 * (2 * k) ** 4
        out["tiers"] = {"triples_fp64": s0["triples"] - s0["triples_low"],
                        "triples_low": s0["triples_low"],
                        "useful_flop_fraction_low": s0["flops_low"] / s0["useful_flops"],
                        "eta_low_sum": s0["eta_low"], "ms_low_kernel": low_ms,
                        "low_kernel": "apply_low_kernel<%d>" % k,
                        "low_kernel_tflops_executed": low_alg / (low_ms * 1e-3) / 1e12 if low_ms > 0 else None,
                        "low_kernel_frac_bf16_peak": (low_alg / (low_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS) if low_ms > 0 else None}
        out["fp64_path"] = fp64_cmp
    if args.cpu_seconds > 0 and args.workload.startswith("coulomb"):
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
