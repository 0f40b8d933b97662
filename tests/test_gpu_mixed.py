"""Low-precision tier of the non-standard apply (BF16 transforms, FP32 accumulation, FP64
result) through the C ABI, against the FP64 oracle.  Needs an MI355X.

Gates:
  * the mixed result agrees with the FP64 oracle to relative L2 <= 10 thresh;
  * screening and trees are those of the FP64 path (the tier only changes arithmetic);
  * error model: a low-tier triple evaluates c [(R x R x R) - (P x P x P)] B_P in the
    cancellation-free form E R R + P E R + P P E, whose three terms are bounded in norm by
    the parts of N(delta) = prod(a + e) - prod(a).  Rounding the source block, each
    intermediate and each operator block to BF16 (unit roundoff u = 2^-8, operator blocks
    bounded through the Frobenius norm, <= sqrt(2k) times the spectral norm) gives at most
    (3 + 3 sqrt(2k)) u eta per triple, so ||mixed - FP64|| <= (3 + 3 sqrt(2k)) u sum(eta)
    over the low-tier triples (plus FP32 accumulation and FP64 noise, covered by a factor
    1.1 and 1e-12 ||ref||).
"""
import math
import sys

import numpy as np
import pytest

import mra_workloads as W
from oracle.apply import SeparatedOperator, apply_nonstandard
from oracle.fit import coulomb_fit, cell_r_hi
from oracle.projection import GaussianSum, project_adaptive

pytestmark = pytest.mark.gpu

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


def _l2(d, keys):
    return math.sqrt(sum(float(np.sum(d[q] ** 2)) for q in keys))


def _diff(a, b, keys):
    return math.sqrt(sum(float(np.sum((a[q] - b[q]) ** 2)) for q in keys))


@pytest.fixture(scope="module")
def M():
    import paper_1507_01888_amd as mod
    mod.load()
    return mod


CASES = {
    # k, thresh, tau_drop, gaussian generator args (workload id, seed, count, a_lo, a_hi)
    "k10": (10, 1e-5, 1e-9, (1, 7, 2, 1.0, 30.0)),
    "k12": (12, 1e-6, 1e-10, (2, 7, 1, 3.0, 3.0)),
}


@pytest.fixture(scope="module")
def oracle_refs():
    cache = {}

    def get(name):
        if name not in cache:
            k, thresh, tau, gen = CASES[name]
            c, a, x = W.unit_charge_gaussians(*gen)
            fo = project_adaptive(GaussianSum(c, a, x), k, thresh, W.CELL, 2, 20)
            cc, tt = coulomb_fit(1e-5, 1e-8, cell_r_hi(*W.CELL))
            cache[name] = apply_nonstandard(fo, SeparatedOperator(cc, tt), tau)
        return cache[name]
    return get


def _run(M, name, tau_tier):
    k, thresh, tau, gen = CASES[name]
    c, a, x = W.unit_charge_gaussians(*gen)
    ctx = M.Context(0, W.CELL)
    f = ctx.project(c, a, x, k, thresh)
    op = ctx.op_coulomb(k, 1e-5, 1e-8)
    g = ctx.apply(op, f, tau_drop=tau, tau_tier=tau_tier)
    return _as_dict(g), ctx.last_stats()


def _check(M, oracle_refs, name, tier_rel, spec_gate=True):
    k, thresh, tau, _ = CASES[name]
    _say("case: low tier %s, tau_tier = %g thresh" % (name, tier_rel))
    got, st = _run(M, name, tier_rel * thresh)
    ref, rst = oracle_refs(name)
    assert set(got) == set(ref.leaves)
    assert st["triples"] == rst["triples"]
    assert st["triples_low"] > 0
    keys = list(ref.leaves)
    nrm = _l2(ref.leaves, keys)
    diff = _diff(got, ref.leaves, keys)
    bound = 1.1 * (3 + 3 * math.sqrt(2 * k)) * U_BF16 * st["eta_low"] + 1e-12 * nrm
    _say("%s tier %g: low triples %d of %d, rel L2 vs oracle %.3e, |diff| %.3e <= bound %.3e"
         % (name, tier_rel, st["triples_low"], st["triples"], diff / nrm, diff, bound))
    assert diff > 1e-13 * nrm            # the low tier changed the arithmetic
    assert diff <= bound
    if spec_gate:
        assert diff / nrm <= 10 * thresh


def test_low_tier_k10_literal(M, oracle_refs):
    """Tier boundary 1e-3 thresh."""
    _check(M, oracle_refs, "k10", 1e-3)


def test_low_tier_k10_wide(M, oracle_refs):
    """Every triple below thresh in BF16 (most source changes and list shapes)."""
    _check(M, oracle_refs, "k10", 1.0)


def test_low_tier_k10_everything(M, oracle_refs):
    """All triples at levels n > 0 in BF16: only the error model is asserted."""
    _check(M, oracle_refs, "k10", 1e30, spec_gate=False)


def test_low_tier_k12_literal(M, oracle_refs):
    _check(M, oracle_refs, "k12", 1e-3)


def test_low_tier_k12_wide(M, oracle_refs):
    _check(M, oracle_refs, "k12", 1.0)


def test_low_tier_errors(M):
    _say("case: low tier argument errors")
    ctx = M.Context(0, W.CELL)
    c, a, x = W.unit_charge_gaussians(1, 3, 1, 2.0, 2.0)
    f = ctx.project(c, a, x, 8, 1e-4)
    op = ctx.op_coulomb(8, 1e-4, 1e-6)
    with pytest.raises(M.MraError) as e:      # no BF16 kernel for k = 8
        ctx.apply(op, f, tau_drop=1e-8, tau_tier=1e-7)
    assert e.value.code == -4
    with pytest.raises(M.MraError) as e:
        ctx.apply(op, f, tau_drop=1e-8, tau_tier=-1.0)
    assert e.value.code == -1


def test_batched_k14_mixed_sampled(M):
    """The large batched mixed workload's shape at a coarse threshold: two functions of 32
    Gaussians (exponents log-uniform in [1, 1e4]), k = 14, one batched apply with the BF16
    tier at 1e-3 thresh and one in FP64.  Output leaves sampled across levels are recomputed
    by the oracle along their root paths (FP64 path: 1e-12; mixed path: 10 thresh and the
    error model)."""
    from oracle.apply import sampled_leaves
    thresh = 1e-2
    tau = 1e-4 * thresh
    _say("case: batched k=14, 2 x 32 Gaussians, thresh %g, tiers at 1e-3 thresh" % thresh)
    ctx = M.Context(0, W.CELL)
    params = [W.coulomb_inputs("coulomb_batch_k14", i) for i in range(2)]
    funcs = [ctx.project(c, a, x, 14, thresh) for (c, a, x) in params]
    op = ctx.op_coulomb(14, 1e-5, 1e-8)
    g64 = ctx.apply_batch([op, op], funcs, tau_drop=tau)
    st64 = ctx.last_stats()
    gmx = ctx.apply_batch([op, op], funcs, tau_drop=tau, tau_tier=1e-3 * thresh)
    stmx = ctx.last_stats()
    _say("k14 batch: triples %d, low %d, useful GFLOP %.1f, main kernel %.1f ms, low kernel %.2f ms"
         % (stmx["triples"], stmx["triples_low"], stmx["useful_flops"] / 1e9,
            stmx["ms_main_kernel"], stmx["ms_low_kernel"]))
    assert stmx["triples"] == st64["triples"] and stmx["triples_low"] > 0
    d64 = [_as_dict(g) for g in g64]
    dmx = [_as_dict(g) for g in gmx]
    total_diff2 = 0.0
    for i in range(2):
        assert set(d64[i]) == set(dmx[i])
        keys = list(d64[i])
        total_diff2 += _diff(dmx[i], d64[i], keys) ** 2
    bound = 1.1 * (3 + 3 * math.sqrt(28)) * U_BF16 * stmx["eta_low"]
    _say("k14 batch: |mixed - fp64| %.3e <= bound %.3e" % (math.sqrt(total_diff2), bound))
    assert math.sqrt(total_diff2) <= bound
    # oracle on sampled output leaves of function 0
    c, a, x = params[0]
    fo = project_adaptive(GaussianSum(c, a, x), 14, thresh, W.CELL, 2, 20)
    cc, tt = coulomb_fit(1e-5, 1e-8, cell_r_hi(*W.CELL))
    keys = sorted(d64[0])
    rng = np.random.default_rng(11)
    by_level = {}
    for q in keys:
        by_level.setdefault(q[0], []).append(q)
    sample = []
    for n, lst in sorted(by_level.items()):
        for j in rng.choice(len(lst), min(2, len(lst)), replace=False):
            sample.append(lst[j])
    vals, has_acc, _ = sampled_leaves(fo, SeparatedOperator(cc, tt), tau, sample)
    for q in sample:
        assert not has_acc[q]
    num64 = math.sqrt(sum(float(np.sum((d64[0][q] - vals[q]) ** 2)) for q in sample))
    nummx = math.sqrt(sum(float(np.sum((dmx[0][q] - vals[q]) ** 2)) for q in sample))
    den = math.sqrt(sum(float(np.sum(vals[q] ** 2)) for q in sample))
    _say("k14 batch sampled (%d leaves): fp64 rel L2 %.3e, mixed rel L2 %.3e"
         % (len(sample), num64 / den, nummx / den))
    assert num64 / den <= 1e-12
    assert nummx / den <= 10 * thresh
