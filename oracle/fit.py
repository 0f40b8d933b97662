"""Gaussian-sum fits of the Coulomb and bound-state Helmholtz kernels (paper Sec. 2.3).

The paper writes 1/r as (2/sqrt(pi)) * int exp(-r^2 e^{2s} + s) ds and discretises the
integral by quadrature into sum_mu c_mu exp(-t_mu r^2) with relative error O(eps) on a
range [1, R] (read here as [r_lo, r_hi] by scale invariance).  The quadrature is the
trapezoid rule on a uniform s-grid.

Readings (the paper gives no parameters):

* step       h = pi^2 / (2 (ln(1/eps) + 3)); the integrand is analytic in the strip
             |Im s| < pi/4, so the trapezoid error is about exp(-pi^2/(2h)), with a margin;
* upper end  s_hi = ln(erfcinv(eps/4) / r_lo): the omitted upper tail, relative to 1/r,
             is erfc(r e^{s_hi}) <= eps/4 for r >= r_lo;
* lower end  s_lo = ln(eps sqrt(pi) / (8 r_hi)): the omitted lower tail is at most
             (2/sqrt(pi)) e^{s_lo}, which times r_hi is eps/4;
* M          = ceil((s_hi - s_lo)/h) + 1 nodes s_j = s_lo + j h;
* terms      c_j = (2/sqrt(pi)) h e^{s_j},  t_j = e^{2 s_j}.

Bound-state Helmholtz kernel exp(-mu r)/r (the kernel of eq. (bshkernel) with the
distance restored in the exponent and the 1/(4 pi) dropped; mu = sqrt(-2E)):
exp(-mu r)/r = (2/sqrt(pi)) int exp(-r^2 e^{2s} - mu^2 e^{-2s}/4 + s) ds, so on the same
grid c_j = (2/sqrt(pi)) h exp(s_j - mu^2 e^{-2 s_j}/4).  The extra factor kills the lower
tail, so the first node is raised in steps of h while the omitted lower tail, bounded by
min((2/sqrt(pi)) e^s, (mu/(2 sqrt(pi))) x^{-3/2} e^{-x}) with x = mu^2 e^{-2s}/4 (the
bound Gamma(-1/2, x) <= x^{-3/2} e^{-x}), stays <= eps/(4 r_hi).  Errors are measured
relative to 1/r in both cases.
"""
import math

import numpy as np
from scipy.special import erfcinv


def _grid(r_lo, eps, r_hi):
    h = math.pi ** 2 / (2.0 * (math.log(1.0 / eps) + 3.0))
    s_hi = math.log(float(erfcinv(eps / 4.0)) / r_lo)
    s_lo = math.log(eps * math.sqrt(math.pi) / (8.0 * r_hi))
    m = int(math.ceil((s_hi - s_lo) / h)) + 1
    return h, s_lo, m


def coulomb_fit(r_lo, eps, r_hi):
    """(c, t) with 1/r ~= sum_mu c_mu exp(-t_mu r^2) to relative eps on [r_lo, r_hi]."""
    h, s_lo, m = _grid(r_lo, eps, r_hi)
    s = s_lo + h * np.arange(m)
    c = (2.0 / math.sqrt(math.pi)) * h * np.exp(s)
    t = np.exp(2.0 * s)
    return c, t


def _bsh_tail_bound(s, mu):
    coul = (2.0 / math.sqrt(math.pi)) * math.exp(s)
    x = mu * mu * math.exp(-2.0 * s) / 4.0
    if x <= 0.0:
        return coul
    return min(coul, (mu / (2.0 * math.sqrt(math.pi))) * x ** -1.5 * math.exp(-x))


def bsh_fit(mu, r_lo, eps, r_hi):
    """(c, t) with exp(-mu r)/r ~= sum c exp(-t r^2) to eps/r on [r_lo, r_hi]."""
    h, s_lo, m = _grid(r_lo, eps, r_hi)
    target = eps / (4.0 * r_hi)
    j0 = 0
    while j0 + 1 < m and _bsh_tail_bound(s_lo + (j0 + 1) * h, mu) <= target:
        j0 += 1
    s = s_lo + h * np.arange(j0, m)
    c = (2.0 / math.sqrt(math.pi)) * h * np.exp(s - mu * mu * np.exp(-2.0 * s) / 4.0)
    t = np.exp(2.0 * s)
    return c, t


def cell_r_hi(cell_lo, cell_hi):
    """Largest distance inside the cubic cell: sqrt(3) * W."""
    return math.sqrt(3.0) * (cell_hi - cell_lo)
