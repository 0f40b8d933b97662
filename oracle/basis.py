"""Scaling functions and the two-scale filter (paper Sec. 2.1, eq. scalingfunc; Sec. 2.2).

Reading (normalisation): coefficients are taken with respect to functions that are
orthonormal in user coordinates.  On a cell [lo, hi] of width W the level-n box l has
width h_n = W / 2^n and its i-th scaling function is

    phi^n_{l,i}(x) = h_n^{-1/2} phi_i((x - lo)/h_n - l),

which is the paper's 2^{n/2} phi_i(2^n x - l) after mapping the cell onto [0, 1] and
rescaling by W^{-1/2}.
"""
import numpy as np
from numpy.polynomial import legendre as _leg


def gauss_legendre(n, a=0.0, b=1.0):
    """n-point Gauss-Legendre nodes and weights on [a, b] (exact for degree 2n-1)."""
    x, w = _leg.leggauss(n)
    return a + (b - a) * (x + 1.0) * 0.5, w * (b - a) * 0.5


def phi(k, x):
    """Mother scaling functions phi_i(x) = sqrt(2i+1) P_i(2x-1) on [0,1], zero outside.

    Returns an array of shape (k,) + x.shape.  eq. (scalingfunc).
    """
    x = np.asarray(x, dtype=np.float64)
    t = 2.0 * x - 1.0
    p = np.zeros((k,) + x.shape)
    p[0] = 1.0
    if k > 1:
        p[1] = t
    for i in range(1, k - 1):
        # Bonnet recursion (i+1) P_{i+1} = (2i+1) t P_i - i P_{i-1}
        p[i + 1] = ((2 * i + 1) * t * p[i] - i * p[i - 1]) / (i + 1)
    scale = np.sqrt(2.0 * np.arange(k) + 1.0).reshape((k,) + (1,) * x.ndim)
    inside = (x >= 0.0) & (x <= 1.0)
    return p * scale * inside


def two_scale_filters(k):
    """Filters h0, h1 (k x k) relating a box to its two children (Sec. 2.2).

    phi^n_{l,i} = sum_j h0[i,j] phi^{n+1}_{2l,j} + h1[i,j] phi^{n+1}_{2l+1,j}, i.e.
    h0[i,j] = 2^{-1/2} int_0^1 phi_i(u/2) phi_j(u) du and
    h1[i,j] = 2^{-1/2} int_0^1 phi_i((u+1)/2) phi_j(u) du.
    The integrands are polynomials of degree <= 2k-2, so k-point Gauss-Legendre is exact.
    Parent scaling coefficients are s = h0 s_left + h1 s_right.
    """
    u, w = gauss_legendre(k)
    pj = phi(k, u)
    h0 = (phi(k, 0.5 * u) * w) @ pj.T / np.sqrt(2.0)
    h1 = (phi(k, 0.5 * (u + 1.0)) * w) @ pj.T / np.sqrt(2.0)
    return h0, h1


def filter_matrix(k):
    """H = [h0 | h1] (k x 2k): maps the 1D children block [s_left; s_right] to the parent s."""
    h0, h1 = two_scale_filters(k)
    return np.hstack([h0, h1])
