"""mra_norm2_noalloc (the entry point that allocates no device memory) against mra_norm2,
through the C ABI.  Needs an MI355X."""
import sys

import pytest

import mra_workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_norm2_noalloc_matches_norm2_two_calls():
    import paper_1507_01888_amd as M
    M.load()
    sizes = []
    ctx = M.Context(0, W.CELL, on_alloc=sizes.append)
    # a larger and then a smaller input: a k=10 Coulomb result and a k=6 projection
    c, a, x = W.unit_charge_gaussians(1, 7, 2, 1.0, 30.0)
    f = ctx.project(c, a, x, 10, 1e-5)
    op = ctx.op_coulomb(10, 1e-5, 1e-8)
    big = ctx.apply(op, f, tau_drop=1e-9)
    small = ctx.project([1.0], [2.0], [[0.1, 0.2, -0.3]], 6, 1e-3)
    assert big.info()["leaves"] > small.info()["leaves"]
    for g in (big, small):
        ref = ctx.norm2(g)
        sizes.clear()
        got = ctx.norm2_noalloc(g)
        _say("leaves %d: norm2 %.17g, noalloc %.17g, allocations %d"
             % (g.info()["leaves"], ref, got, len(sizes)))
        assert sizes == []                      # no device allocation through the context
        assert got == ref                       # same partials summed in the same order
    # repeated calls keep agreeing (the array keeps the last call's contents)
    assert ctx.norm2_noalloc(big) == ctx.norm2(big)
    assert ctx.norm2_noalloc(small) == ctx.norm2(small)
