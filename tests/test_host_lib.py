"""libmra on the host: the library loads, exports every declared symbol, and its FP64 host
numerics (fits, filters, blocks, projection) agree with the oracle.  No device calls."""
import math
import os
import re

import numpy as np
import pytest

import mra_workloads as W
import paper_1507_01888_amd as M
from oracle.basis import two_scale_filters
from oracle.blocks import BlockFactory
from oracle.fit import coulomb_fit, bsh_fit
from oracle.projection import GaussianSum, project_adaptive
from oracle.tree import morton

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mra.h")).read()
    return sorted(set(re.findall(r"^\s*(?:mra_status|const char\*)\s+(mra_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = M.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(M.EXPORTED)


def test_host_fits_match_oracle():
    r_hi = math.sqrt(3) * 20.0
    c, t = M.host_fit("coulomb", 1e-5, 1e-8, r_hi)
    c2, t2 = coulomb_fit(1e-5, 1e-8, r_hi)
    assert len(c) == len(c2) == 160
    assert np.abs(c / c2 - 1).max() < 1e-14 and np.abs(t / t2 - 1).max() < 1e-14
    for mu in (0.5, 2.2, 5.0):
        c, t = M.host_fit("bsh", 1e-5, 1e-8, r_hi, mu=mu)
        c2, t2 = bsh_fit(mu, 1e-5, 1e-8, r_hi)
        assert len(c) == len(c2)
        assert np.abs(c / c2 - 1).max() < 1e-13 and np.abs(t / t2 - 1).max() < 1e-14


@pytest.mark.parametrize("k", [2, 8, 14])
def test_host_filters_match_oracle(k):
    h0, h1 = M.host_filters(k)
    o0, o1 = two_scale_filters(k)
    assert np.abs(h0 - o0).max() < 1e-14 and np.abs(h1 - o1).max() < 1e-14


@pytest.mark.parametrize("n,d,t", [(2, 0, 1.0), (3, 1, 0.3), (5, 2, 100.0), (1, 0, 1e-8),
                                   (0, 0, 1e9), (7, 1, 1e4), (4, 5, 0.02)])
def test_host_blocks_match_oracle(n, d, t):
    k = 10
    bf = BlockFactory(k, 20.0)
    a = M.host_block(k, 20.0 / 2 ** n, d, t)
    b = bf.t_block(n, d, t)
    assert np.abs(a - b).max() <= 1e-14 * max(1.0, np.abs(b).max())


def test_host_spectral_norm():
    a = np.random.default_rng(0).standard_normal((28, 28))
    assert abs(M.host_spectral_norm(a) / np.linalg.norm(a, 2) - 1) < 1e-14


@pytest.mark.parametrize("case", ["example", "coulomb_k10"])
def test_host_projection_matches_oracle(case):
    if case == "example":
        cell, k, thresh = (-6.0, 6.0), 6, 1e-4
        c, a, x = [1.0], [1.0], [[0.0, 0.0, 0.0]]
    else:
        cell, k, thresh = W.CELL, 10, 1e-6
        c, a, x = W.coulomb_inputs("coulomb_k10", 0)
    keys, co = M.host_project(cell, c, a, x, k, thresh)
    f = project_adaptive(GaussianSum(c, a, x), k, thresh, cell, 2, 20)
    ok = {morton(kk): v for kk, v in f.leaves.items()}
    assert sorted(int(q) for q in keys) == sorted(ok)          # identical trees
    scale = max(np.abs(v).max() for v in ok.values())
    err = max(np.abs(co[i] - ok[int(q)]).max() for i, q in enumerate(keys))
    assert err < 1e-13 * scale


def test_host_error_codes():
    with pytest.raises(M.MraError) as e:
        M.host_fit("coulomb", -1.0, 1e-8, 10.0)
    assert e.value.code == -1
    with pytest.raises(M.MraError):
        M.host_block(15, 1.0, 0, 1.0)
    with pytest.raises(M.MraError):
        M.host_project((-1.0, 1.0), [1.0], [1.0], [[0, 0, 0]], 6, -1.0)
