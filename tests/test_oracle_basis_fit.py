"""Pins of the oracle's basis, two-scale filter and Gaussian-sum fits (CPU only)."""
import math

import numpy as np
import pytest

from oracle.basis import gauss_legendre, phi, two_scale_filters
from oracle.fit import coulomb_fit, bsh_fit, cell_r_hi


@pytest.mark.parametrize("k", [2, 6, 10, 14])
def test_scaling_functions_orthonormal(k):
    # eq. (scalingfunc): phi_i orthonormal on (0, 1); quadrature with 40 points is exact
    x, w = gauss_legendre(40)
    p = phi(k, x)
    g = (p * w) @ p.T
    assert np.abs(g - np.eye(k)).max() < 1e-13


def test_phi_closed_form_low_orders():
    x = np.linspace(0.01, 0.99, 17)
    p = phi(3, x)
    assert np.allclose(p[0], 1.0, atol=1e-15)
    assert np.allclose(p[1], math.sqrt(3) * (2 * x - 1), atol=1e-14)
    assert np.allclose(p[2], math.sqrt(5) * (6 * x * x - 6 * x + 1), atol=1e-13)
    assert np.all(phi(3, np.array([-0.1, 1.1])) == 0.0)


def test_filter_k2_literal_values():
    # h0 = 2^{-1/2} [[1, 0], [-sqrt(3)/2, 1/2]] for phi_0 = 1, phi_1 = sqrt(3)(2x-1)
    h0, h1 = two_scale_filters(2)
    r = 1 / math.sqrt(2)
    assert np.allclose(h0, [[r, 0.0], [-math.sqrt(3) / 2 * r, 0.5 * r]], atol=1e-15)
    assert np.allclose(h1, [[r, 0.0], [math.sqrt(3) / 2 * r, 0.5 * r]], atol=1e-15)


@pytest.mark.parametrize("k", [3, 8, 12])
def test_two_scale_relation_pointwise(k):
    # phi^0_i(x) = sum_j h0[i,j] sqrt2 phi_j(2x) + h1[i,j] sqrt2 phi_j(2x - 1), checked at
    # random points: a check of the filter against the functions themselves.
    h0, h1 = two_scale_filters(k)
    x = np.random.default_rng(1).uniform(0.0, 1.0, 200)
    lhs = phi(k, x)
    rhs = math.sqrt(2) * (h0 @ phi(k, 2 * x) + h1 @ phi(k, 2 * x - 1))
    assert np.abs(lhs - rhs).max() < 1e-11 * max(1.0, np.abs(lhs).max())


@pytest.mark.parametrize("k", [4, 10, 14])
def test_filter_identities(k):
    h0, h1 = two_scale_filters(k)
    assert np.abs(h0 @ h0.T + h1 @ h1.T - np.eye(k)).max() < 1e-14
    sign = np.array([[(-1.0) ** (i + j) for j in range(k)] for i in range(k)])
    assert np.abs(h1 - sign * h0).max() < 1e-14
    assert np.abs(np.triu(h0, 1)).max() < 1e-14


def _max_rel_err(c, t, kernel, r_lo, r_hi, n=20000):
    r = np.exp(np.linspace(math.log(r_lo), math.log(r_hi), n))
    approx = np.array([np.sum(c * np.exp(-t * rr * rr)) for rr in r])
    return float(np.max(np.abs(approx - kernel(r)) * r))


@pytest.mark.parametrize("r_lo,eps", [(1e-5, 1e-8), (1e-4, 1e-6), (1e-3, 1e-10)])
def test_coulomb_fit_accuracy(r_lo, eps):
    # Sec. 2.3: sum_mu c_mu exp(-t_mu r^2) = 1/r + O(eps / r) on the range of validity
    r_hi = cell_r_hi(-10.0, 10.0)
    c, t = coulomb_fit(r_lo, eps, r_hi)
    assert _max_rel_err(c, t, lambda r: 1.0 / r, r_lo, r_hi) <= eps


@pytest.mark.parametrize("mu", [0.5, 1.7, 5.0])
def test_bsh_fit_accuracy(mu):
    r_lo, eps, r_hi = 1e-5, 1e-8, cell_r_hi(-10.0, 10.0)
    c, t = bsh_fit(mu, r_lo, eps, r_hi)
    err = _max_rel_err(c, t, lambda r: np.exp(-mu * r) / r, r_lo, r_hi)
    assert err <= eps
    cc, _ = coulomb_fit(r_lo, eps, r_hi)
    assert len(c) < len(cc)      # the screened kernel needs fewer terms


def test_bsh_fit_reduces_to_coulomb():
    r_lo, eps, r_hi = 1e-4, 1e-8, 30.0
    c0, t0 = coulomb_fit(r_lo, eps, r_hi)
    c1, t1 = bsh_fit(0.0, r_lo, eps, r_hi)
    assert np.array_equal(t0, t1) and np.allclose(c0, c1, rtol=1e-15)


def test_fit_term_count_growth():
    # M = O(log R log 1/eps): increments in log R and log(1/eps) are uniform
    r_hi = 10.0
    ms = [len(coulomb_fit(r_hi / R, 1e-8, r_hi)[0]) for R in (1e2, 1e4, 1e6, 1e8)]
    d = np.diff(ms)
    assert np.all(d > 0) and d.max() - d.min() <= 2
    me = [len(coulomb_fit(1e-4, eps, r_hi)[0]) for eps in (1e-4, 1e-6, 1e-8, 1e-10)]
    assert np.all(np.diff(me) > 0)
    # growth with log(1/eps) is about linear times log R (within a factor 2 over the range)
    ratio = (me[-1] / me[0])
    assert 1.0 < ratio < (math.log(1e10) + 3) / (math.log(1e4) + 3) * 1.6
