"""Adaptive projection on the device (Sec. 2.1) against the FP64 oracle and the library's
host projection, through the C ABI.  Needs an MI355X.

Bar: the trees are equal (every refinement decision is taken in FP64 on both sides; the
cases are checked to have no wavelet norm within 1e-6 relative of thresh on the oracle's
side, so that rounding cannot flip one; for the 32-Gaussian function this margin is not
computed); leaf coefficients to relative L2 <= 1e-13.
"""
import math
import sys

import numpy as np
import pytest

import mra_workloads as W
from oracle.basis import filter_matrix
from oracle.projection import GaussianSum, project_adaptive, wavelet_norm
from oracle.tree import morton

pytestmark = pytest.mark.gpu

CELL = (-10.0, 10.0)
THREE = ([1.0, -0.4, 0.25], [3.0, 40.0, 400.0],
         [[0.3, -0.2, 0.1], [-1.1, 0.7, 2.0], [2.5, 2.2, -1.3]])


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def M():
    import paper_1507_01888_amd as mod
    mod.load()
    return mod


@pytest.fixture(scope="module")
def ctx(M):
    return M.Context(0, CELL)


def _dict(keys, co):
    return {int(q): co[i] for i, q in enumerate(keys)}


def _rel(got, ref):
    num = math.sqrt(sum(float(np.sum((got[q] - ref[q]) ** 2)) for q in ref))
    den = math.sqrt(sum(float(np.sum(ref[q] ** 2)) for q in ref))
    return num / den


def _margin(fo, gs, k, thresh, initial_level, max_level):
    """Smallest |norm - thresh| / thresh over every box whose refinement was tested."""
    hm = filter_matrix(k)
    tested = [q for q in list(fo.leaves) + list(fo.interior())
              if initial_level <= q[0] < max_level]
    cache = {}
    return min(abs(wavelet_norm(GaussianSum(*gs), k, CELL, q, hm, cache) - thresh) / thresh
               for q in tested)


def _check(M, ctx, gs, k, thresh, initial_level=2, max_level=20, margin=True):
    f = ctx.project(*gs, k, thresh, initial_level=initial_level, max_level=max_level)
    got = _dict(*f.export())
    fo = project_adaptive(GaussianSum(*gs), k, thresh, CELL, initial_level, max_level)
    if margin:
        assert _margin(fo, gs, k, thresh, initial_level, max_level) > 1e-6
    ref = {morton(q): v for q, v in fo.leaves.items()}
    assert sorted(got) == sorted(ref), "trees differ"
    err = _rel(got, ref)
    host = _dict(*M.host_project(CELL, *gs, k, thresh, initial_level, max_level))
    assert sorted(host) == sorted(got)
    err_h = _rel(got, host)
    _say("  %d leaves, max level %d, rel L2 vs oracle %.3e, vs host path %.3e"
         % (len(got), f.info()["max_level"], err, err_h))
    assert err <= 1e-13 and err_h <= 1e-13
    return f, fo


@pytest.mark.parametrize("k,thresh", [(4, 1e-3), (6, 1e-4), (10, 1e-6), (14, 1e-8)])
def test_projection_three_gaussians(M, ctx, k, thresh):
    _say("case: device projection, 3 Gaussians, k=%d thresh=%g" % (k, thresh))
    _check(M, ctx, THREE, k, thresh)


def test_projection_level_cap_and_level_zero_start(M, ctx):
    """A narrow Gaussian that would refine past the deepest level stops there; the
    refinement starts from the root box."""
    _say("case: device projection, cap at level 5, start at level 0")
    gs = ([1.0], [3e4], [[0.11, -0.07, 0.23]])
    f, fo = _check(M, ctx, gs, 6, 1e-6, initial_level=0, max_level=5)
    assert f.info()["max_level"] == 5 and fo.max_level() == 5


def test_projection_batch_function_k14(M, ctx):
    """Function 0 of the 16 x 32-Gaussian k=14 batch (the benchmark's inputs)."""
    _say("case: device projection, 32 Gaussians, k=14, thresh 1e-8 (batch function 0)")
    w = W.WORKLOADS["coulomb_batch_k14"]
    gs = W.coulomb_inputs("coulomb_batch_k14", 0)
    # (margin not computed here: a second oracle pass over 6,500 leaves; the tree
    # comparison itself would show a flipped decision)
    _check(M, ctx, gs, w["k"], w["thresh"], initial_level=w["initial_level"], margin=False)


def test_projection_rejects_too_many_gaussians(M, ctx):
    gs = ([1.0] * 4097, [1.0] * 4097, [[0.0, 0.0, 0.0]] * 4097)
    with pytest.raises(M.MraError):
        ctx.project(*gs, 4, 1e-3)
