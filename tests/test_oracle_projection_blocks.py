"""Pins of the oracle's projection and 1D operator blocks (CPU only)."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle.analytic import gaussian_sum_trace, gaussian_sum_norm2
from oracle.basis import gauss_legendre, phi, filter_matrix
from oracle.blocks import BlockFactory, e_bound, decay_bound
from oracle.projection import gaussian_1d, GaussianSum, project_adaptive, project_uniform


def _closed_1d(a, X, x0, h):
    """Coefficients 0 and 1 of exp(-a (x-X)^2) on the box [x0, x0+h] by erf closed forms."""
    sa = math.sqrt(a)
    i0 = math.sqrt(math.pi) / (2 * sa) * (erf(sa * (x0 + h - X)) - erf(sa * (x0 - X)))
    i1 = (math.exp(-a * (x0 - X) ** 2) - math.exp(-a * (x0 + h - X) ** 2)) / (2 * a)
    c0 = i0 / math.sqrt(h)
    c1 = math.sqrt(3) / math.sqrt(h) * ((2 / h) * (i1 + (X - x0) * i0) - i0)
    return c0, c1


@pytest.mark.parametrize("a,X,l,h", [(1.0, 0.3, 3, 1.25), (1e3, -2.01, 7, 0.15625),
                                     (50.0, 1.0, 4, 2.5), (1e6, 0.0, 512, 0.01953125)])
def test_gaussian_1d_closed_form(a, X, l, h):
    lo = -10.0
    v = gaussian_1d(6, a, X, lo, h, l)
    c0, c1 = _closed_1d(a, X, lo + l * h, h)
    scale = max(abs(c0), abs(c1), 1e-300)
    assert abs(v[0] - c0) <= 1e-13 * max(scale, math.sqrt(math.pi / a) / math.sqrt(h))
    assert abs(v[1] - c1) <= 1e-12 * max(scale, math.sqrt(math.pi / a) / math.sqrt(h))


def test_projection_trace_and_norm_adaptive():
    coeffs, expnts = [1.0, 0.5], [2.0, 40.0]
    centers = [[0.3, -0.2, 0.1], [-1.1, 0.7, 0.4]]
    f = project_adaptive(GaussianSum(coeffs, expnts, centers), 6, 1e-4, (-6.0, 6.0), 2, 12)
    # trace of a projection is exact at any level (phi_0 integrates the box)
    assert abs(f.trace() - gaussian_sum_trace(coeffs, expnts)) < 1e-12 * gaussian_sum_trace(coeffs, expnts)
    exact = gaussian_sum_norm2(coeffs, expnts, centers)
    n = f.norm2()
    assert n <= exact * (1 + 1e-14)       # projection never increases the norm
    assert exact - n < 1e-6 * exact       # and is close at this threshold


def test_projection_refinement_rule():
    # leaves satisfy ||d|| <= thresh (they are not refined): check via filtered children
    from oracle.projection import wavelet_norm
    g = GaussianSum([1.0], [5.0], [[0.2, 0.1, -0.3]])
    cell = (-6.0, 6.0)
    f = project_adaptive(g, 5, 1e-3, cell, 2, 10)
    hm = filter_matrix(5)
    rng = np.random.default_rng(0)
    keys = list(f.leaves)
    for i in rng.choice(len(keys), 20, replace=False):
        assert wavelet_norm(g, 5, cell, keys[i], hm) <= 1e-3
    for key in list(f.interior())[:10]:
        assert wavelet_norm(g, 5, cell, key, hm) > 1e-3


def _brute_block(k, h, lt, ls, texp, npan=24, npts=24):
    """Matrix element by 2D tensor quadrature with explicit box positions."""
    u, w = [], []
    for p in range(npan):
        a, b = gauss_legendre(npts, p / npan, (p + 1) / npan)
        u.append(a)
        w.append(b)
    u = np.concatenate(u)
    w = np.concatenate(w)
    x = (lt + u) * h
    y = (ls + u) * h
    K = np.exp(-texp * (x[:, None] - y[None, :]) ** 2)
    p = phi(k, u) / math.sqrt(h)
    return (p * w) @ K @ (p * w).T * h * h


@pytest.mark.parametrize("n,delta,texp", [(2, 0, 0.01), (3, 1, 0.5), (4, -2, 3.0), (5, 1, 30.0)])
def test_block_against_2d_quadrature(n, delta, texp):
    k = 5
    bf = BlockFactory(k, 20.0)
    h = bf.h(n)
    blk = bf.t_block(n, delta, texp)
    # translation invariance: two different absolute placements give the same block
    for ls in (0, 2):
        brute = _brute_block(k, h, ls + delta, ls, texp)
        assert np.abs(blk - brute).max() <= 2e-13 * max(1.0, np.abs(brute).max())


@pytest.mark.parametrize("delta,beta", [(0, 0.3), (1, 2.0), (2, 10.0), (-3, 0.05), (0, 1e6)])
def test_block_t00_closed_form(delta, beta):
    # t_00 = h int_{-1}^{1} (1 - |w|) exp(-beta (delta + w)^2) dw
    k, W, n = 4, 20.0, 3
    h = W / 2 ** n
    bf = BlockFactory(k, W)
    sb = math.sqrt(beta)

    def G(a, b):
        return math.sqrt(math.pi) / (2 * sb) * (erf(sb * b) - erf(sb * a))

    def Mm(a, b):
        return (math.exp(-beta * a * a) - math.exp(-beta * b * b)) / (2 * beta)

    d = float(delta)
    val = (1 + d) * G(d, d + 1) - Mm(d, d + 1) + (1 - d) * G(d - 1, d) + Mm(d - 1, d)
    blk = bf.t_block(n, delta, beta / h ** 2)
    assert abs(blk[0, 0] - h * val) <= 1e-13 * h * max(abs(val), 1e-3 / sb)


def test_block_symmetries_and_two_scale():
    k = 6
    bf = BlockFactory(k, 20.0)
    hm = filter_matrix(k)
    sign = np.array([[(-1.0) ** (i + j) for j in range(k)] for i in range(k)])
    for (n, d, t) in [(1, 1, 0.2), (3, 2, 4.0), (4, 0, 100.0), (2, 3, 0.01)]:
        tp, tm = bf.t_block(n, d, t), bf.t_block(n, -d, t)
        s = max(1.0, np.abs(tp).max())
        assert np.abs(tm - tp.T).max() < 1e-14 * s
        assert np.abs(tm - sign * tp).max() < 1e-14 * s
        r = bf.r_block(n, d, t)
        assert np.abs(hm @ r @ hm.T - tp).max() < 1e-14 * s


def test_screening_bounds_are_rigorous():
    rng = np.random.default_rng(3)
    for k in (6, 10):
        bf = BlockFactory(k, 20.0)
        for _ in range(25):
            n = int(rng.integers(0, 7))
            t = float(math.exp(rng.uniform(math.log(1e-4), math.log(1e6))))
            d = int(rng.integers(0, min(2 ** n, 6)))
            h = bf.h(n)
            beta = t * h * h
            a, e, r = bf.norms(n, d, t)
            # computed e carries rounding noise of order 1e-15 (a + h) (R and H^T t H cancel)
            assert e <= e_bound(k, h, beta) * (1 + 1e-12) + 1e-14 * (a + h)
            assert a + e <= decay_bound(h, beta, d) * (1 + 1e-12) + 1e-300
            assert r <= decay_bound(h, beta, d) * (1 + 1e-12) + 1e-300


def test_nonstandard_block_decay_rates():
    # Sec. 2.2: for the Poisson kernel the wavelet-wavelet part decays like r^{-2k-1} and the
    # mixed parts like r^{-k-1}.  1D check on the summed Coulomb fit in the filtered basis.
    from oracle.fit import coulomb_fit
    k = 4
    bf = BlockFactory(k, 64.0)
    c, t = coulomb_fit(1e-3, 1e-10, 200.0)
    n = 6
    h0, h1 = bf.hm[:, :k], bf.hm[:, k:]
    g0, g1 = h0.copy(), h1.copy()
    # orthonormal completion of H = [h0 h1]: rows of G span the wavelet space
    Hm = np.hstack([h0, h1])
    q, _ = np.linalg.qr(np.hstack([Hm.T, np.eye(2 * k)]))
    G = q[:, k:2 * k].T
    assert np.abs(G @ Hm.T).max() < 1e-12
    ds = np.arange(6, 14)
    dd, sd = [], []
    for d in ds:
        R = sum(ci * bf.r_block(n, int(d), ti) for ci, ti in zip(c, t))
        dd.append(np.linalg.norm(G @ R @ G.T, 2))
        sd.append(np.linalg.norm(Hm @ R @ G.T, 2))
    s_dd = np.polyfit(np.log(ds), np.log(dd), 1)[0]
    s_sd = np.polyfit(np.log(ds), np.log(sd), 1)[0]
    assert abs(s_dd + (2 * k + 1)) < 1.0
    assert abs(s_sd + (k + 1)) < 1.0
