"""Pins of the oracle's wavelet form, reconstruction and truncation (CPU only)."""
import math

import numpy as np
import pytest

from oracle.basis import filter_matrix
from oracle.compress import compress, reconstruct, truncate
from oracle.projection import GaussianSum, project_adaptive, project_box
from oracle.tree import filter3, unfilter3, split_block, children

CELL = (-10.0, 10.0)


def _f(k=4, thresh=1e-4):
    g = GaussianSum([1.0, -0.4], [3.0, 40.0], [[0.3, -0.2, 0.1], [-1.1, 0.7, 2.0]])
    return g, project_adaptive(g, k, thresh, CELL, 2, 20)


def test_parseval_and_round_trip():
    _, f = _f()
    c = compress(f)
    assert len(c.details) > 20
    # the transform is orthogonal: the 2-norm is the norm of root and details together
    assert abs(c.norm2() - f.norm2()) <= 1e-13 * f.norm2()
    g = reconstruct(c)
    assert set(g.leaves) == set(f.leaves)
    err = max(np.abs(g.leaves[q] - f.leaves[q]).max() for q in f.leaves)
    assert err <= 1e-14 * max(np.abs(v).max() for v in f.leaves.values())


def test_details_are_orthogonal_to_the_parent_space():
    # D_P has no component in the parent's scaling space: filtering it gives zero, and the
    # children block is the parent's polynomial plus D_P
    _, f = _f(k=5)
    hm = filter_matrix(5)
    c = compress(f)
    coeff = f.filtered_interior()
    for key, d in list(c.details.items())[:12]:
        assert np.abs(filter3(d, hm)).max() <= 1e-14 * max(1.0, np.abs(d).max())
        blk = unfilter3(coeff[key], hm) + d
        for ch, v in zip(children(key), split_block(blk, 5)):
            assert np.abs(v - coeff[ch]).max() <= 1e-14 * max(1.0, np.abs(coeff[ch]).max())


def test_truncate_below_thresh_keeps_everything():
    # every refined box of an adaptive projection at thresh has ||D|| > thresh
    _, f = _f(thresh=1e-4)
    g, removed = truncate(f, 0.5e-4)
    assert removed == 0.0 and set(g.leaves) == set(f.leaves)


def test_truncate_to_the_root_is_the_level_zero_projection():
    # with every detail removed the function is its projection on the root box, computed
    # here directly from the Gaussians
    gs, f = _f(k=4)
    g, removed = truncate(f, 1e30)
    assert list(g.leaves) == [(0, 0, 0, 0)]
    ref = project_box(gs, 4, CELL, (0, 0, 0, 0))
    assert np.abs(g.leaves[(0, 0, 0, 0)] - ref).max() <= 1e-13 * np.abs(ref).max()
    assert abs(removed - (f.norm2() ** 2 - float(np.sum(ref ** 2)))) <= 1e-12 * f.norm2() ** 2


@pytest.mark.parametrize("tol", [3e-4, 3e-3, 3e-2])
def test_truncation_error_is_the_removed_detail_norm(tol):
    # ||f - trunc(f)||^2 = sum of the squared norms of the removed D_P (orthogonality),
    # with the difference evaluated leaf by leaf on f's (finer) tree
    _, f = _f(k=4, thresh=1e-5)
    g, removed = truncate(f, tol)
    assert len(g.leaves) < len(f.leaves)
    gv = g.values_on(list(f.leaves))
    diff2 = sum(float(np.sum((f.leaves[q] - gv[q]) ** 2)) for q in f.leaves)
    assert removed > 0
    assert abs(diff2 - removed) <= 1e-9 * removed + 1e-26
    assert math.sqrt(diff2) <= tol * math.sqrt(len(f.leaves))


def test_truncate_keeps_a_small_detail_above_a_large_one():
    # a box with a small wavelet part but a refined child with a large one stays refined:
    # the rule works bottom-up and only boxes whose children are leaves can lose them
    from oracle.compress import Compressed
    k = 2
    rng = np.random.default_rng(3)
    hm = filter_matrix(k)

    def detail(scale):
        d = rng.standard_normal((2 * k, 2 * k, 2 * k))
        d -= unfilter3(filter3(d, hm), hm)          # no component in the parent space
        return scale * d / np.linalg.norm(d)

    P, Q = (0, 0, 0, 0), (1, 1, 0, 1)
    c = Compressed(k, CELL, rng.standard_normal((k, k, k)), {P: detail(1e-6), Q: detail(1.0)})
    f = reconstruct(c)
    assert len(f.leaves) == 15
    g, removed = truncate(f, 1e-3)
    assert set(g.leaves) == set(f.leaves) and removed == 0.0
    g2, removed2 = truncate(f, 2.0)
    assert list(g2.leaves) == [P] and abs(removed2 - (1.0 + 1e-12)) <= 1e-12
