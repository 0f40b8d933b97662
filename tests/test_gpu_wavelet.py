"""Wavelet form on the device (compress, reconstruct, truncate; Sec. 2.2) against the FP64
oracle, through the C ABI.  Needs an MI355X.

Bar: trees compared exactly; coefficients (every D_P, s_0, the leaves of reconstructed and
truncated functions) to relative L2 <= 1e-13 of the oracle's (the two sides filter in a
different summation order, nothing else may differ); the square root of the removed squared
norm of a truncation to 1e-13 ||f|| (it is the norm of a subset of the D_P coefficients).
Truncation thresholds are chosen away from every ||D_P|| so that the integer decisions
cannot flip on rounding (checked in the test).  The apply-result case compares against the
oracle's apply, so its bar is that of the apply (1e-12).
"""
import math
import sys

import numpy as np
import pytest

from oracle.compress import compress, truncate
from oracle.projection import GaussianSum, project_adaptive
from oracle.tree import assemble_block, children

pytestmark = pytest.mark.gpu

CELL = (-10.0, 10.0)
GAUSS = ([1.0, -0.4, 0.25], [3.0, 40.0, 400.0],
         [[0.3, -0.2, 0.1], [-1.1, 0.7, 2.0], [2.5, 2.2, -1.3]])
CASES = [(5, 1e-4), (6, 1e-4), (10, 1e-6), (14, 1e-8)]


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


def _leaves(func):
    keys, co = func.export()
    return {_key_tuple(q): co[i] for i, q in enumerate(keys)}


def _nodes(func):
    keys, co = func.export_nodes()
    return {_key_tuple(q): co[i] for i, q in enumerate(keys)}


def _rel(got, ref):
    keys = list(ref)
    num = math.sqrt(sum(float(np.sum((got[q] - ref[q]) ** 2)) for q in keys))
    den = math.sqrt(sum(float(np.sum(ref[q] ** 2)) for q in keys))
    return num / den


@pytest.fixture(scope="module")
def M():
    import paper_1507_01888_amd as mod
    mod.load()
    return mod


@pytest.fixture(scope="module")
def ctx(M):
    return M.Context(0, CELL)


_cache = {}


def _pair(ctx, k, thresh):
    if (k, thresh) not in _cache:
        f = ctx.project(*GAUSS, k, thresh)
        fo = project_adaptive(GaussianSum(*GAUSS), k, thresh, CELL, 2, 20)
        assert set(_leaves(f)) == set(fo.leaves)
        _cache[(k, thresh)] = (f, fo, compress(fo))
    return _cache[(k, thresh)]


@pytest.mark.parametrize("k,thresh", CASES)
def test_compress_matches_oracle(M, ctx, k, thresh):
    _say("case: compress, k=%d thresh=%g" % (k, thresh))
    f, fo, co = _pair(ctx, k, thresh)
    c = ctx.compress(f)
    assert c.repr() == M.REPR_WAVELET and f.repr() == M.REPR_SCALING
    slabs = _nodes(c)
    assert len(co.details) > 8
    got = {q: assemble_block([slabs[ch] for ch in children(q)], k) for q in co.details}
    ref = dict(co.details)
    got[(0, 0, 0, 0, "root")] = slabs[(0, 0, 0, 0)]
    ref[(0, 0, 0, 0, "root")] = co.root
    err = _rel(got, ref)
    _say("  %d details, rel L2 vs oracle %.3e" % (len(co.details), err))
    assert err <= 1e-13
    # Parseval over the slabs, against the scaling form's leaf norm and the oracle
    n_w, n_s = ctx.norm2(c), ctx.norm2(f)
    assert abs(n_w - n_s) <= 1e-13 * n_s
    assert abs(n_w - co.norm2()) <= 1e-13 * n_s
    # calls that need the scaling form refuse the wavelet form
    with pytest.raises(M.MraError):
        c.export()
    with pytest.raises(M.MraError):
        ctx.trace(c)
    with pytest.raises(M.MraError):
        ctx.reconstruct(f)


@pytest.mark.parametrize("k,thresh", CASES)
def test_reconstruct_round_trip(M, ctx, k, thresh):
    _say("case: reconstruct(compress(f)), k=%d thresh=%g" % (k, thresh))
    f, fo, _ = _pair(ctx, k, thresh)
    g = ctx.reconstruct(ctx.compress(f))
    assert g.repr() == M.REPR_SCALING
    got = _leaves(g)
    assert set(got) == set(fo.leaves)
    err = _rel(got, _leaves(f))
    _say("  rel L2 vs the input %.3e" % err)
    assert err <= 1e-14
    # interior slabs of the reconstruction hold the filtered coefficients
    inter = fo.filtered_interior()
    nodes = _nodes(g)
    assert _rel({q: nodes[q] for q in inter}, inter) <= 1e-13


@pytest.mark.parametrize("k,thresh", CASES)
def test_truncate_matches_oracle(M, ctx, k, thresh):
    f, fo, co = _pair(ctx, k, thresh)
    norms = np.array(sorted(math.sqrt(float(np.sum(d ** 2))) for d in co.details.values()))
    for tol in (0.0, 3 * thresh, 30 * thresh, 300 * thresh, 1e30):
        _say("case: truncate, k=%d thresh=%g tol=%g" % (k, thresh, tol))
        if 0.0 < tol < 1e30:
            assert np.min(np.abs(norms - tol)) > 1e-6 * tol, "tolerance too close to a norm"
        go, removed_o = truncate(fo, tol)
        g, removed = ctx.truncate(f, tol)
        assert g.repr() == M.REPR_SCALING
        got = _leaves(g)
        assert set(got) == set(go.leaves)
        err = _rel(got, go.leaves)
        _say("  %d -> %d leaves, rel L2 %.3e, removed %.6e (oracle %.6e)"
             % (len(fo.leaves), len(go.leaves), err, removed, removed_o))
        assert err <= 1e-13
        # the removed part is a set of D_P coefficients, each compared above to 1e-13 of
        # ||f||: by the triangle inequality its norm agrees to the same bar
        assert abs(math.sqrt(removed) - math.sqrt(removed_o)) <= 1e-13 * fo.norm2()
        if tol == 0.0:
            assert removed == 0.0 and set(got) == set(fo.leaves)
        if tol == 1e30:
            assert list(got) == [(0, 0, 0, 0)]
        # the truncated function is usable by the rest of the library
        assert ctx.norm2(g) > 0.0


def test_truncate_an_apply_result(M, ctx):
    """The output of an apply (interior slabs not yet filtered) compresses and truncates
    like a projection."""
    _say("case: truncate an apply result, k=6")
    from oracle.apply import SeparatedOperator, apply_nonstandard
    from oracle.fit import coulomb_fit, cell_r_hi
    f, fo, _ = _pair(ctx, 6, 1e-4)
    op = ctx.op_coulomb(6, 1e-3, 1e-5)
    g = ctx.apply(op, f, tau_drop=1e-8)
    cc, tt = coulomb_fit(1e-3, 1e-5, cell_r_hi(*CELL))
    go, _ = apply_nonstandard(fo, SeparatedOperator(cc, tt), 1e-8)
    assert set(_leaves(g)) == set(go.leaves)
    tol = 1e-3
    ho, removed_o = truncate(go, tol)
    norms = [math.sqrt(float(np.sum(d ** 2))) for d in compress(go).details.values()]
    assert min(abs(v - tol) for v in norms) > 1e-6 * tol
    h, removed = ctx.truncate(g, tol)
    got = _leaves(h)
    assert set(got) == set(ho.leaves) and len(ho.leaves) < len(go.leaves)
    assert _rel(got, ho.leaves) <= 1e-12
    assert abs(math.sqrt(removed) - math.sqrt(removed_o)) <= 1e-12 * go.norm2()
