#!/usr/bin/env python3
"""Benchmark of the separated-operator apply on one MI355X.

One step = one pass of the whole hot path over one synthetic function or batch of
functions: filter-up with block norms, norm screening and tiering, transform-and-
accumulate, sum-down, and the norm2 reduction of every result.  Inputs (the projected
functions and the operators with their block caches, built during warm-up) are resident in
HBM when the timed region starts.

The default workload is the large batched mixed-precision apply: 16 functions of 32
unit-charge Gaussians (exponents log-uniform in [1, 1e4]), k = 14, thresh 1e-8, Coulomb
kernel fitted to 1e-8 (160 terms), one batched apply per step, with the BF16 tier for kept
triples whose norm bound eta is below 1e-3 thresh.  `value` is its useful GFLOP/s (sum over
kept triples of 6(2k)^4 + 6k^4 [n > 0]).  The same functions are also applied with every
triple in FP64 and with a wider tier (eta < thresh); the line reports both rates, the
speed-ups and the distance of each mixed result from the FP64 one.

Prints one JSON line: the metric, the roofline of the dominant kernel (timed with HIP
events on the library's stream), per-tier kernel rates, and the FP64 oracle timed on a
bounded sample on the host cores.
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

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # MI355X dense, AMD published
HBM_PEAK_GBS = 8000.0
METRIC = "useful operator-apply GFLOP/s and boxes/s, mixed-prec batched vs FP64 @ err≤10*thresh"
WORKLOAD_NAMES = ["coulomb_batch_k14", "gauss_std_k8", "coulomb_k10", "coulomb_k12_fp64",
                  "coulomb_k12_mixed", "bsh_batch_k10"]
FP64_KERNEL = {8: "apply_ns_mfma_kernel<8>", 10: "apply_ns_fac_kernel<10>",
               12: "apply_ns_own_kernel<12>", 14: "apply_ns_stream_kernel<14>"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="coulomb_batch_k14", choices=WORKLOAD_NAMES)
    p.add_argument("--cmp-steps", type=int, default=5,
                   help="timed steps of each comparison run (all-FP64 path, wide tier) of a "
                        "tiered workload, after one warm-up step (at most --steps)")
    p.add_argument("--no-tune", action="store_true",
                   help="skip the autotuner of the batched workloads' schedule")
    p.add_argument("--schedule", default=None, metavar="S,D",
                   help="run the batched workloads under sub-batches S and split divisor D "
                        "instead of tuning")
    p.add_argument("--tune-cache", default=None,
                   help="JSON file the autotuner reads and extends (default: none, tune now)")
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


# ------------------------------------------------------------------------ CPU baseline

def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(fo, op, tau, budget_s):
    """Whole source levels of the oracle's non-standard apply, coarsest first, while the
    predicted time of the next level fits the budget.  Operator blocks and their norms are
    computed before each level is timed (block quadrature is not part of the apply)."""
    from oracle.apply import filter_up, nonstandard_contributions, screen_level
    from oracle.blocks import BlockFactory
    levels = filter_up(fo)
    bf = BlockFactory(fo.k, fo.width)
    flops, secs, done, rate = 0.0, 0.0, [], None
    for n in sorted(levels):
        groups = screen_level(bf, levels[n], op, tau, fo.k)      # norms and blocks, untimed
        for (mu, d, _) in groups:
            for dd in d:
                bf.r_block(n, dd, float(op.t[mu]))
                bf.t_block(n, dd, float(op.t[mu]))
        cnt = sum(len(i) for (_, _, i) in groups)
        f_next = cnt * (6.0 * (2 * fo.k) ** 4 + (6.0 * fo.k ** 4 if n > 0 else 0.0))
        if rate is not None and secs + f_next / rate > 1.5 * budget_s:
            break
        t0 = time.perf_counter()
        _, _, st = nonstandard_contributions(fo, op, tau, only_levels={n}, levels=levels, blocks=bf)
        secs += time.perf_counter() - t0
        flops += st["useful_flops"]
        done.append(n)
        rate = flops / secs if secs > 0 else None
        if secs >= budget_s:
            break
    return flops, secs, done


def cpu_baseline(name, budget_s):
    """The FP64 oracle (NumPy) timed on the host cores on a bounded sample of the workload:
    function 0 (its own projection and operator fit), whole source levels of the
    non-standard apply (standard form: the whole apply), with every BLAS thread, and again
    on one core."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.apply import SeparatedOperator, apply_standard
    from oracle.fit import coulomb_fit, bsh_fit, cell_r_hi
    from oracle.projection import GaussianSum, project_adaptive, project_uniform

    w = W.WORKLOADS["coulomb_k12_mixed" if name.startswith("coulomb_k12") else name]
    r_hi = cell_r_hi(*W.CELL)

    if name == "gauss_std_k8":
        fo = project_uniform(GaussianSum([w["f_coeff"]], [w["f_expnt"]], [[0, 0, 0]]),
                             w["k"], W.CELL, w["level"])
        op = SeparatedOperator(w["op_c"], w["op_t"])
    else:
        if name == "bsh_batch_k10":
            c, a, x, mu = W.bsh_inputs(0)
            cc, tt = bsh_fit(mu, w["r_lo"], w["eps"], r_hi)
        else:
            c, a, x = W.coulomb_inputs(name if name in W.WORKLOADS else "coulomb_k12_mixed", 0)
            cc, tt = coulomb_fit(w["r_lo"], w["eps"], r_hi)
        fo = project_adaptive(GaussianSum(c, a, x), w["k"], w["thresh"], W.CELL,
                              w["initial_level"], 20)
        op = SeparatedOperator(cc, tt)

    def sample(limit_s):
        if name == "gauss_std_k8":
            t0 = time.perf_counter()
            _, st = apply_standard(fo, op, w["level"], w["disp_radius"])
            return st["useful_flops"], time.perf_counter() - t0, "the whole standard-form apply"
        fl, s, done = _oracle_sample(fo, op, w["tau_rel"] * w["thresh"], limit_s)
        return fl, s, "function 0, source levels %s of the non-standard apply" % done

    # several BLAS libraries may be loaded (numpy's, torch's); the oracle's products run on
    # one of them, so the thread count is the largest pool's, not the sum
    threads = max([i.get("num_threads", 0) for i in threadpool_info()
                   if i.get("user_api") == "blas"] + [1])
    fl, s, what = sample(budget_s)
    with threadpool_limits(limits=1, user_api="blas"):
        fl1, s1, what1 = sample(budget_s / 2)
    return {"value": fl / s / 1e9, "unit": "GFLOP/s", "cores": max(1, threads),
            "kind": "oracle",
            "sample": "%s (FP64 NumPy, %.1f useful GFLOP in %.1f s; screening timed, block "
                      "quadrature and projection not)" % (what, fl / 1e9, s),
            "value_1core": fl1 / s1 / 1e9,
            "sample_1core": "%s (%.1f useful GFLOP in %.1f s)" % (what1, fl1 / 1e9, s1),
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


# ---------------------------------------------------------------------------- workloads

def setup(ctx, name):
    """(funcs, ops, tau_drop, k, tau_tier, config) of a workload."""
    if name == "gauss_std_k8":
        w = W.WORKLOADS[name]
        f = ctx.project([w["f_coeff"]], [w["f_expnt"]], [[0.0, 0.0, 0.0]], w["k"], 1.0,
                        initial_level=w["level"], max_level=w["level"])
        op = ctx.op_gaussians(w["k"], w["op_c"], w["op_t"])
        cfg = {"workload": name, "k": w["k"], "level": w["level"], "boxes": 8 ** w["level"],
               "operator": "exp(-2 x^2)", "displacements": (2 * w["disp_radius"] + 1) ** 3,
               "form": "standard", "precision": "fp64"}
        return [f], [op], None, w["k"], 0.0, cfg
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
        return funcs, ops, w["tau_rel"] * w["thresh"], w["k"], 0.0, cfg
    if name == "coulomb_batch_k14":
        w = W.WORKLOADS[name]
        funcs = []
        for i in range(w["n_funcs"]):
            c, a, x = W.coulomb_inputs(name, i)
            funcs.append(ctx.project(c, a, x, w["k"], w["thresh"], initial_level=w["initial_level"]))
        op = ctx.op_coulomb(w["k"], w["r_lo"], w["eps"])
        tier = w["tier_rel"] * w["thresh"]
        cfg = {"workload": name, "k": w["k"], "thresh": w["thresh"], "functions": w["n_funcs"],
               "gaussians_per_function": w["n_gauss"], "exponent_range": [w["a_lo"], w["a_hi"]],
               "operator": "coulomb", "terms": int(op.terms()[0].size), "eps_fit": w["eps"],
               "r_lo": w["r_lo"], "tau_drop": w["tau_rel"] * w["thresh"], "tau_tier": tier,
               "precision": "fp64 + bf16 tier (eta < tau_tier), fp32 accumulation",
               "launch": "one batched apply (all functions per kernel launch)"}
        return funcs, [op] * len(funcs), w["tau_rel"] * w["thresh"], w["k"], tier, cfg
    base = "coulomb_k12_mixed" if name.startswith("coulomb_k12") else name
    w = W.WORKLOADS[base]
    c, a, x = W.coulomb_inputs(base, 0)
    f = ctx.project(c, a, x, w["k"], w["thresh"], initial_level=w["initial_level"])
    op = ctx.op_coulomb(w["k"], w["r_lo"], w["eps"])
    cfg = {"workload": name, "k": w["k"], "thresh": w["thresh"], "gaussians": w["n_gauss"],
           "operator": "coulomb", "terms": int(op.terms()[0].size), "eps_fit": w["eps"],
           "r_lo": w["r_lo"], "tau_drop": w["tau_rel"] * w["thresh"], "precision": "fp64"}
    tier = 0.0
    if name == "coulomb_k12_mixed":
        tier = w["tier_rel"] * w["thresh"]
        cfg["precision"] = "fp64 + bf16 tier (eta < tau_tier), fp32 accumulation"
        cfg["tau_tier"] = tier
    return [f], [op], w["tau_rel"] * w["thresh"], w["k"], tier, cfg


def kernel_source_sha(kernel):
    """sha256[:16] of the source of `kernel` (its definition up to the next section rule in
    kernels.hip) and of the flags kernels.hip is compiled with, so that counters stay valid
    while other kernels of the file change, and not after the code generation changed."""
    import hashlib
    from paper_1507_01888_amd import build as B
    src = open(os.path.join(ROOT, "paper_1507_01888_amd", "csrc", "kernels.hip")).read()
    base = kernel.split("<")[0]
    i = src.find(" void %s(" % base)
    if i < 0:
        return None
    i = src.rfind("\ntemplate", 0, i)
    j = src.find("\n// ---", i)
    flags = " ".join(B.COMMON + B.DEVICE_EXTRA.get("kernels.hip", []))
    return hashlib.sha256((src[i:j] + "\n" + flags).encode()).hexdigest()[:16]


def measured_traffic(kernel, workload, schedule=None):
    """HBM bytes per launch of `kernel` on `workload` from the committed rocprofv3 counter
    summaries, or None when none was taken on the current source of the kernel (and, for a
    batched workload, under the same schedule: it sets how much one launch processes)."""
    import glob
    sha = kernel_source_sha(kernel)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_pmc.md"))):
        for line in open(path):
            if line.startswith("pmc: "):
                rec = json.loads(line[5:])
                if (rec.get("kernel") == kernel and rec.get("kernel_src_sha256_16") == sha
                        and rec.get("workload", workload) == workload
                        and rec.get("schedule") == schedule):
                    return 1024.0 * (rec["fetch_kib"] * rec["fetch_factor"]
                                     + rec["write_kib"] * rec["write_factor"])
    return None


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU; --gpus %d is not supported "
              "(sharding over several GPUs is described in the design notes, not implemented)"
              % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1507_01888_amd as M

    ctx = M.Context(0, W.CELL)
    funcs, ops, tau, k, tier, cfg = setup(ctx, args.workload)
    name = args.workload
    tuning = None
    if args.schedule:
        sb, div = (int(v) for v in args.schedule.split(","))
        ctx.set_schedule(sb, div)
    elif len(funcs) > 1 and not args.no_tune:
        # the schedule of the batched apply (sub-batches, split length) picked by the
        # library's autotuner on these inputs, before warm-up
        t0 = time.perf_counter()
        sched, times = ctx.autotune_batch(ops, funcs, tau_drop=tau, tau_tier=tier,
                                          cache_path=args.tune_cache)
        tuning = {"schedule": sched, "candidate_ms": [round(float(t), 1) for t in times],
                  "seconds": time.perf_counter() - t0}

    def apply(tau_tier):
        if tau is None:     # standard form on a uniform tree, no screening
            return [ctx.apply(ops[0], funcs[0], form="standard",
                              disp_radius=W.WORKLOADS[name]["disp_radius"])]
        if len(funcs) == 1:
            return [ctx.apply(ops[0], funcs[0], tau_drop=tau, tau_tier=tau_tier)]
        return ctx.apply_batch(ops, funcs, tau_drop=tau, tau_tier=tau_tier)

    def step(tau_tier, keep=False):
        gs = apply(tau_tier)
        st = ctx.last_stats()
        nrm = [ctx.norm2(g) for g in gs]
        if keep:
            return st, nrm, gs
        for g in gs:
            g.free()
        return st, nrm

    def timed(tau_tier, steps, warmup):
        for _ in range(warmup):
            step(tau_tier)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(steps):
            st, nrm = step(tau_tier)
            stats.append(st)
        torch.cuda.synchronize()
        return stats, nrm, time.perf_counter() - t0

    def mean(stats, key):
        return sum(s[key] for s in stats) / len(stats)

    stats, nrm, elapsed = timed(tier, args.steps, args.warmup)
    s0 = stats[0]
    flops = sum(s["useful_flops"] for s in stats)

    # ---- per-kernel rates (HIP events on the library's stream), per tier
    main_ms = mean(stats, "ms_main_kernel")
    main_launch_ms = main_ms / max(1, s0["launches_main"])
    useful_main = s0["useful_flops"] - s0["flops_low"]
    if tau is None:        # standard form: matrix-core kernel for k = 8, vector ALU otherwise
        kname, bound, prec = (("apply_std_mfma_kernel<8>", "mfma", "fp64") if k == 8 else
                              ("apply_std_kernel<%d>" % k, "alu", "fp64"))
    else:
        kname, bound, prec = FP64_KERNEL.get(k, "apply_ns_kernel<%d>" % k), "mfma", "fp64"
    kernels = {"fp64": {"kernel": kname, "ms_per_apply": main_ms,
                        "launches_per_apply": s0["launches_main"],
                        "ms_per_launch": main_launch_ms,
                        "useful_tflops": useful_main / (main_ms * 1e-3) / 1e12,
                        "executed_tflops": s0["flops_kernel"] / (main_ms * 1e-3) / 1e12,
                        "triples": s0["triples"] - s0["triples_low"]}}
    kernels["fp64"]["frac"] = kernels["fp64"]["useful_tflops"] / PEAK_TFLOPS["fp64"]
    kernels["fp64"]["executed_frac"] = kernels["fp64"]["executed_tflops"] / PEAK_TFLOPS["fp64"]
    low_ms = mean(stats, "ms_low_kernel")
    if s0["triples_low"] > 0 and low_ms > 0:
        # the BF16 kernel evaluates 7 mode products of (2k)^3 x 2k per triple (E R R + P E R
        # + P P E with the shared R_z and E_z products)
        low_exec = s0["triples_low"] * 14.0 * (2 * k) ** 4
        kernels["bf16"] = {"kernel": "apply_low_kernel<%d>" % k, "ms_per_apply": low_ms,
                           "launches_per_apply": s0["launches_low"],
                           "ms_per_launch": low_ms / max(1, s0["launches_low"]),
                           "useful_tflops": s0["flops_low"] / (low_ms * 1e-3) / 1e12,
                           "executed_tflops": low_exec / (low_ms * 1e-3) / 1e12,
                           "triples": s0["triples_low"]}
        kernels["bf16"]["frac"] = kernels["bf16"]["useful_tflops"] / PEAK_TFLOPS["bf16"]
        kernels["bf16"]["executed_frac"] = kernels["bf16"]["executed_tflops"] / PEAK_TFLOPS["bf16"]
    dom = max(kernels, key=lambda t: kernels[t]["ms_per_apply"])
    dk = kernels[dom]
    peak = PEAK_TFLOPS[dom]
    alg_per_launch = (useful_main if dom == "fp64" else s0["flops_low"]) / max(1, dk["launches_per_apply"])
    achieved = alg_per_launch / (dk["ms_per_launch"] * 1e-3) / 1e12
    roofline = {"kernel": dk["kernel"], "bound": bound if dom == "fp64" else "mfma",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(dk["kernel"], name,
                                            ctx.schedule() if len(funcs) > 1 else None),
                "algorithmic_flop_per_launch": alg_per_launch,
                "ms_per_launch": dk["ms_per_launch"],
                "executed_frac": dk["executed_frac"]}

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
        "dtype": "f64+bf16" if tier > 0 else "f64",
        "data": "synthetic",
        "config": cfg,
        "boxes_per_s": s0["in_leaves"] * args.steps / elapsed,
        "time_to_solution_ms": elapsed / args.steps * 1e3,
        "counts": {key: s0[key] for key in ("triples", "triples_low", "targets", "in_leaves",
                                            "out_nodes", "out_leaves")},
        "useful_gflop_per_step": s0["useful_flops"] / 1e9,
        "stage_ms": {key: mean(stats, key) for key in ("ms_filter", "ms_plan", "ms_apply",
                                                       "ms_main_kernel", "ms_low_kernel",
                                                       "ms_sumdown")},
        "norm2": math.sqrt(sum(v * v for v in nrm)),
        "roofline": roofline,
        "kernels": kernels,
        "autotune": tuning,
        "schedule": ctx.schedule() if len(funcs) > 1 else None,
    }

    if tier > 0:
        # the same inputs with every triple in FP64, and with the wider tier eta < thresh
        n_cmp = max(1, min(args.cmp_steps, args.steps))
        thresh = cfg["thresh"]
        st64, _, el64 = timed(0.0, n_cmp, 1)
        stw, _, elw = timed(thresh, n_cmp, 1)
        ms_mixed = elapsed / args.steps * 1e3
        ms_64 = el64 / n_cmp * 1e3
        ms_w = elw / n_cmp * 1e3
        _, n64, g64 = step(0.0, keep=True)
        res = {}
        for lab, tt in (("literal", tier), ("wide", thresh)):
            _, _, gm = step(tt, keep=True)
            st = ctx.last_stats()
            d = [ctx.distance(a, b) for a, b in zip(gm, g64)]
            for g in gm:
                g.free()
            # a-priori bound of the low-tier rounding error (three BF16-rounded factors per
            # product, operators through their Frobenius norms): (3 + 3 sqrt(2k)) 2^-8 sum eta
            bound = (3 + 3 * math.sqrt(2 * k)) * 2.0 ** -8 * st["eta_low"]
            tot = math.sqrt(sum(v * v for v in n64))
            res[lab] = {"tau_tier": tt, "triples_low": st["triples_low"],
                        "useful_flop_fraction_low": st["flops_low"] / st["useful_flops"],
                        "rel_l2_vs_fp64": math.sqrt(sum(v * v for v in d)) / tot,
                        "max_rel_l2_per_function": max(dv / nv for dv, nv in zip(d, n64)),
                        "error_bound_rel": bound / tot,
                        "gate_10_thresh": 10 * thresh}
        for g in g64:
            g.free()
        res["literal"].update({"ms_per_step": ms_mixed,
                               "value": flops / elapsed / 1e9,
                               "speedup_vs_fp64": ms_64 / ms_mixed})
        res["wide"].update({"ms_per_step": ms_w,
                            "value": sum(s["useful_flops"] for s in stw) / elw / 1e9,
                            "speedup_vs_fp64": ms_64 / ms_w,
                            "ms_main_kernel": mean(stw, "ms_main_kernel"),
                            "ms_low_kernel": mean(stw, "ms_low_kernel")})
        out["fp64_path"] = {"value": sum(s["useful_flops"] for s in st64) / el64 / 1e9,
                            "ms_per_step": ms_64, "steps": n_cmp,
                            "ms_main_kernel": mean(st64, "ms_main_kernel"),
                            "kernel_useful_tflops": st64[0]["useful_flops"]
                            / (mean(st64, "ms_main_kernel") * 1e-3) / 1e12}
        out["tiers"] = res
        out["speedup_mixed_vs_fp64"] = ms_64 / ms_mixed
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(name, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
