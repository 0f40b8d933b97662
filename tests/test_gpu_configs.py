"""Parity of the HIP path at the full sizes of the benchmark workloads (through the C ABI).
Needs an MI355X.

  * k=10 Coulomb, thresh 1e-6, 4 Gaussians: every output leaf against the full oracle apply
    (<= 1e-12), the same kept triples and tree, and the potential sum_g erf(sqrt(a_g) r_g)/r_g
    of the unit charges projected on the output leaves (<= 10 thresh, Sec. 2.3 kernel);
  * k=12 Coulomb, thresh 1e-8, 4 Gaussians: the FP64 path against the full oracle
    (<= 1e-12) and the BF16 tier at 1e-3 thresh (<= 10 thresh and its rounding bound);
  * 64 batched bound-state Helmholtz functions, k=10, thresh 1e-6: sampled leaves of four
    functions against the oracle (<= 1e-12) and the Yukawa closed form (<= 10 thresh);
  * 16 batched functions of 32 Gaussians, k=14, thresh 1e-8 (FP64 and tiered): sampled
    leaves of functions 0 and 1 against the oracle (FP64 <= 1e-12, mixed <= 10 thresh), and
    every mixed result against its FP64 result within the rounding bound of the tier;
  * two runs of the same apply are bitwise equal (k = 10, 12, 14, batched).
The oracle results are computed on the host cores; each case states its cost.
"""
import math
import sys

import numpy as np
import pytest

import mra_workloads as W
from oracle.analytic import (project_callable, coulomb_potential_unit_gaussian,
                             yukawa_potential_unit_gaussian)
from oracle.apply import SeparatedOperator, apply_nonstandard, sampled_leaves
from oracle.fit import coulomb_fit, bsh_fit, cell_r_hi
from oracle.projection import GaussianSum, project_adaptive

pytestmark = pytest.mark.gpu

TOL = 1e-12
U_BF16 = 2.0 ** -8


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _key_tuple(code):
    code = int(code)
    n = (code.bit_length() - 1) // 3
    code ^= 1 << (3 * n)
    x = y = z = 0
    for b in range(n):
        x |= ((code >> (3 * b + 2)) & 1) << b
        y |= ((code >> (3 * b + 1)) & 1) << b
        z |= ((code >> (3 * b)) & 1) << b
    return (n, x, y, z)


def _as_dict(func):
    keys, co = func.export()
    return {_key_tuple(q): co[i] for i, q in enumerate(keys)}


def _rel_l2(got, ref, keys):
    num = math.sqrt(sum(float(np.sum((got[q] - ref[q]) ** 2)) for q in keys))
    den = math.sqrt(sum(float(np.sum(ref[q] ** 2)) for q in keys))
    return num / den


def _sample(keys, per_level, seed):
    rng = np.random.default_rng(seed)
    by_level = {}
    for q in sorted(keys):
        by_level.setdefault(q[0], []).append(q)
    out = []
    for n, lst in sorted(by_level.items()):
        for i in rng.choice(len(lst), min(per_level, len(lst)), replace=False):
            out.append(lst[i])
    return out


def _coulomb_potential(a, x):
    def V(p):
        out = 0.0
        for ai, xi in zip(a, x):
            out = out + coulomb_potential_unit_gaussian(ai, np.linalg.norm(p - xi, axis=-1))
        return out
    return V


@pytest.fixture(scope="module")
def M():
    import paper_1507_01888_amd as mod
    mod.load()
    return mod


@pytest.mark.timeout(900)
def test_coulomb_k10_full_every_leaf_and_closed_form(M):
    """The full k=10 Coulomb workload; the oracle apply costs about 100 GFLOP on the host."""
    name = "coulomb_k10"
    w = W.WORKLOADS[name]
    _say("case: %s full size, every leaf, closed form" % name)
    c, a, x = W.coulomb_inputs(name, 0)
    tau = w["tau_rel"] * w["thresh"]
    ctx = M.Context(0, W.CELL)
    f = ctx.project(c, a, x, w["k"], w["thresh"])
    op = ctx.op_coulomb(w["k"], w["r_lo"], w["eps"])
    g = ctx.apply(op, f, tau_drop=tau)
    st = ctx.last_stats()
    got = _as_dict(g)
    fo = project_adaptive(GaussianSum(c, a, x), w["k"], w["thresh"], W.CELL, 2, 20)
    assert set(_as_dict(f)) == set(fo.leaves)
    cc, tt = coulomb_fit(w["r_lo"], w["eps"], cell_r_hi(*W.CELL))
    ref, rst = apply_nonstandard(fo, SeparatedOperator(cc, tt), tau)
    assert st["triples"] == rst["triples"]
    assert set(got) == set(ref.leaves)
    err = _rel_l2(got, ref.leaves, ref.leaves)
    _say("%s: %d triples, %d leaves, rel L2 vs oracle %.3e" % (name, st["triples"], len(got), err))
    assert err <= TOL
    pot = project_callable(_coulomb_potential(a, x), w["k"], W.CELL, list(got),
                           npts=w["k"] + 10, panels=1)
    cerr = _rel_l2(got, pot, got)
    _say("%s: rel L2 vs sum of erf(sqrt(a) r)/r %.3e (gate %.1e)" % (name, cerr, 10 * w["thresh"]))
    assert cerr <= 10 * w["thresh"]


@pytest.mark.timeout(1200)
def test_coulomb_k12_full_fp64_and_mixed(M):
    """The full k=12, thresh 1e-8 Coulomb workload in FP64 and with the BF16 tier at
    1e-3 thresh; the oracle apply costs about 330 GFLOP on the host."""
    name = "coulomb_k12_mixed"
    w = W.WORKLOADS[name]
    _say("case: %s full size, FP64 and mixed, every leaf" % name)
    c, a, x = W.coulomb_inputs(name, 0)
    tau = w["tau_rel"] * w["thresh"]
    ctx = M.Context(0, W.CELL)
    f = ctx.project(c, a, x, w["k"], w["thresh"])
    op = ctx.op_coulomb(w["k"], w["r_lo"], w["eps"])
    g64 = _as_dict(ctx.apply(op, f, tau_drop=tau))
    st64 = ctx.last_stats()
    gmx = _as_dict(ctx.apply(op, f, tau_drop=tau, tau_tier=w["tier_rel"] * w["thresh"]))
    stmx = ctx.last_stats()
    assert stmx["triples"] == st64["triples"] and stmx["triples_low"] > 0
    fo = project_adaptive(GaussianSum(c, a, x), w["k"], w["thresh"], W.CELL, 2, 20)
    cc, tt = coulomb_fit(w["r_lo"], w["eps"], cell_r_hi(*W.CELL))
    ref, rst = apply_nonstandard(fo, SeparatedOperator(cc, tt), tau)
    assert st64["triples"] == rst["triples"]
    assert set(g64) == set(ref.leaves) == set(gmx)
    e64 = _rel_l2(g64, ref.leaves, ref.leaves)
    emx = _rel_l2(gmx, ref.leaves, ref.leaves)
    nrm = math.sqrt(sum(float(np.sum(v ** 2)) for v in ref.leaves.values()))
    bound = 1.1 * (3 + 3 * math.sqrt(2 * w["k"])) * U_BF16 * stmx["eta_low"] + 1e-12 * nrm
    _say("%s: %d triples (%d BF16), rel L2 vs oracle: FP64 %.3e, mixed %.3e (bound %.3e)"
         % (name, st64["triples"], stmx["triples_low"], e64, emx, bound / nrm))
    assert e64 <= TOL
    assert emx <= 10 * w["thresh"]
    assert emx * nrm <= bound
    pot = project_callable(_coulomb_potential(a, x), w["k"], W.CELL, list(gmx),
                           npts=w["k"] + 10, panels=1)
    cerr = _rel_l2(gmx, pot, gmx)
    _say("%s: mixed result rel L2 vs sum of erf(sqrt(a) r)/r %.3e (gate %.1e)"
         % (name, cerr, 10 * w["thresh"]))
    assert cerr <= 10 * w["thresh"]


@pytest.mark.timeout(900)
def test_bsh_batch_64_sampled_and_yukawa(M):
    """All 64 bound-state Helmholtz functions in one batched apply; sampled output leaves of
    four functions against the oracle along their root paths and the Yukawa potential of
    their unit charges on the same leaves (whole output of one function)."""
    name = "bsh_batch_k10"
    w = W.WORKLOADS[name]
    tau = w["tau_rel"] * w["thresh"]
    _say("case: %s, 64 functions batched, sampled" % name)
    ctx = M.Context(0, W.CELL)
    params = [W.bsh_inputs(i) for i in range(w["n_funcs"])]
    funcs = [ctx.project(c, a, x, w["k"], w["thresh"]) for (c, a, x, _) in params]
    ops = [ctx.op_bsh(w["k"], mu, w["r_lo"], w["eps"]) for (_, _, _, mu) in params]
    outs = ctx.apply_batch(ops, funcs, tau_drop=tau)
    st = ctx.last_stats()
    _say("%s: %d triples over %d functions" % (name, st["triples"], len(funcs)))
    r_hi = cell_r_hi(*W.CELL)
    for i in (0, 21, 42, 63):
        c, a, x, mu = params[i]
        got = _as_dict(outs[i])
        sample = _sample(got, 3, 100 + i)
        fo = project_adaptive(GaussianSum(c, a, x), w["k"], w["thresh"], W.CELL, 2, 20)
        cc, tt = bsh_fit(mu, w["r_lo"], w["eps"], r_hi)
        vals, has_acc, _ = sampled_leaves(fo, SeparatedOperator(cc, tt), tau, sample)
        assert not any(has_acc[q] for q in sample)
        err = _rel_l2(got, vals, sample)

        def V(p, a=a, x=x, mu=mu):
            out = 0.0
            for ai, xi in zip(a, x):
                out = out + yukawa_potential_unit_gaussian(ai, mu, np.linalg.norm(p - xi, axis=-1))
            return out
        keys = list(got) if i == 0 else sample
        pot = project_callable(V, w["k"], W.CELL, keys, npts=w["k"] + 10, panels=1)
        yerr = _rel_l2(got, pot, keys)
        _say("function %d (mu %.3f, %d Gaussians): %d sampled leaves rel L2 vs oracle %.3e; "
             "Yukawa closed form on %d leaves %.3e" % (i, mu, len(c), len(sample), err, len(keys), yerr))
        assert err <= TOL
        assert yerr <= 10 * w["thresh"]


@pytest.mark.timeout(1200)
def test_coulomb_batch_k14_full_sampled(M):
    """The 16 functions of 32 Gaussians at k=14, thresh 1e-8 in one batched apply, in FP64
    and with the BF16 tier at 1e-3 thresh.  Sampled output leaves of functions 0 and 1
    against the oracle along their root paths; every function's mixed result against its
    FP64 result within the tier's rounding bound (distances computed on the device)."""
    name = "coulomb_batch_k14"
    w = W.WORKLOADS[name]
    tau = w["tau_rel"] * w["thresh"]
    thresh = w["thresh"]
    _say("case: %s, 16 functions batched, FP64 and mixed" % name)
    ctx = M.Context(0, W.CELL)
    params = [W.coulomb_inputs(name, i) for i in range(w["n_funcs"])]
    funcs = [ctx.project(c, a, x, w["k"], thresh) for (c, a, x) in params]
    op = ctx.op_coulomb(w["k"], w["r_lo"], w["eps"])
    ops = [op] * len(funcs)
    g64 = ctx.apply_batch(ops, funcs, tau_drop=tau)
    st64 = ctx.last_stats()
    gmx = ctx.apply_batch(ops, funcs, tau_drop=tau, tau_tier=w["tier_rel"] * thresh)
    stmx = ctx.last_stats()
    _say("%s: %d triples (%d BF16), %.1f useful TFLOP; main kernel FP64 %.0f ms, mixed %.0f + "
         "%.0f ms" % (name, st64["triples"], stmx["triples_low"], st64["useful_flops"] / 1e12,
                      st64["ms_main_kernel"], stmx["ms_main_kernel"], stmx["ms_low_kernel"]))
    assert stmx["triples"] == st64["triples"] and stmx["triples_low"] > 0
    dist = [ctx.distance(a, b) for a, b in zip(gmx, g64)]
    norms = [ctx.norm2(g) for g in g64]
    tot = math.sqrt(sum(v * v for v in norms))
    diff = math.sqrt(sum(v * v for v in dist))
    bound = 1.1 * (3 + 3 * math.sqrt(2 * w["k"])) * U_BF16 * stmx["eta_low"]
    _say("%s: |mixed - FP64| %.3e (rel %.3e) <= bound %.3e; worst function rel %.3e"
         % (name, diff, diff / tot, bound, max(d / n for d, n in zip(dist, norms))))
    assert diff <= bound
    assert diff / tot <= 10 * thresh
    cc, tt = coulomb_fit(w["r_lo"], w["eps"], cell_r_hi(*W.CELL))
    for i in (0, 1):
        c, a, x = params[i]
        d64, dmx = _as_dict(g64[i]), _as_dict(gmx[i])
        assert set(d64) == set(dmx)
        sample = _sample(d64, 2, 200 + i)
        fo = project_adaptive(GaussianSum(c, a, x), w["k"], thresh, W.CELL, 2, 20)
        vals, has_acc, _ = sampled_leaves(fo, SeparatedOperator(cc, tt), tau, sample)
        assert not any(has_acc[q] for q in sample)
        e64 = _rel_l2(d64, vals, sample)
        emx = _rel_l2(dmx, vals, sample)
        pot = project_callable(_coulomb_potential(a, x), w["k"], W.CELL, sample,
                               npts=w["k"] + 10, panels=1)
        cerr = _rel_l2(dmx, pot, sample)
        _say("function %d: %d output leaves, %d sampled: rel L2 vs oracle FP64 %.3e, mixed %.3e;"
             " mixed vs sum of erf(sqrt(a) r)/r %.3e" % (i, len(d64), len(sample), e64, emx, cerr))
        assert e64 <= TOL
        assert emx <= 10 * thresh
        assert cerr <= 10 * thresh


@pytest.mark.parametrize("case", ["k10", "k12", "k14", "batch_k10", "batch_k14_mixed"])
def test_two_runs_bitwise_equal(M, case):
    """Results do not depend on scheduling: persistent kernels take target ranges from
    counters, but every target is owned by one workgroup and split lists are summed in a
    fixed order."""
    _say("case: determinism %s" % case)
    ctx = M.Context(0, W.CELL)
    if case.startswith("batch"):
        k = 10 if case == "batch_k10" else 14
        funcs, ops = [], []
        for i in range(3):
            c, a, x = W.unit_charge_gaussians(5, i, 3, 1.0, 100.0)
            funcs.append(ctx.project(c, a, x, k, 1e-5))
            ops.append(ctx.op_coulomb(k, 1e-5, 1e-8) if i == 0 else
                       ctx.op_bsh(k, 0.7 + i, 1e-5, 1e-8))
        tier = 1e-6 if case.endswith("mixed") else 0.0
        runs = [[_as_dict(g) for g in ctx.apply_batch(ops, funcs, tau_drop=1e-9, tau_tier=tier)]
                for _ in range(2)]
        for a_, b_ in zip(*runs):
            assert set(a_) == set(b_)
            assert all(np.array_equal(a_[q], b_[q]) for q in a_)
        return
    k = int(case[1:])
    c, a, x = W.unit_charge_gaussians(5, 9, 3, 1.0, 100.0)
    f = ctx.project(c, a, x, k, 1e-5)
    op = ctx.op_coulomb(k, 1e-5, 1e-8)
    r1 = _as_dict(ctx.apply(op, f, tau_drop=1e-9))
    n1 = ctx.last_stats()["triples"]
    r2 = _as_dict(ctx.apply(op, f, tau_drop=1e-9))
    _say("determinism %s: %d triples, %d leaves" % (case, n1, len(r1)))
    assert set(r1) == set(r2)
    assert all(np.array_equal(r1[q], r2[q]) for q in r1)
