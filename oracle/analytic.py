"""Closed forms used to pin the oracle (not part of the method itself).

* Gaussian integrals: int exp(-a|x-X|^2) = (pi/a)^{3/2}; overlap of two Gaussians.
* Gaussian convolved with Gaussian is a Gaussian.
* Potential of a unit-charge Gaussian (a/pi)^{3/2} exp(-a r^2):
    Coulomb 1/r:         erf(sqrt(a) r) / r
    Yukawa exp(-mu r)/r: exp(-a r^2)/(2r) [erfcx(mu/(2 sqrt a) - sqrt(a) r)
                                           - erfcx(mu/(2 sqrt a) + sqrt(a) r)]
  (the second reduces to the first as mu -> 0).
* Projection of a smooth callable onto given boxes by tensor Gauss-Legendre quadrature.
"""
import math

import numpy as np
from scipy.special import erf, erfc, erfcx

from .basis import gauss_legendre, phi


def gaussian_sum_trace(coeffs, expnts):
    return float(sum(c * (math.pi / a) ** 1.5 for c, a in zip(coeffs, expnts)))


def gaussian_sum_norm2(coeffs, expnts, centers):
    """||sum_g c_g exp(-a_g |x - X_g|^2)||_2 over R^3."""
    tot = 0.0
    for c1, a1, x1 in zip(coeffs, expnts, centers):
        for c2, a2, x2 in zip(coeffs, expnts, centers):
            d2 = float(np.sum((np.asarray(x1) - np.asarray(x2)) ** 2))
            tot += c1 * c2 * (math.pi / (a1 + a2)) ** 1.5 * math.exp(-a1 * a2 / (a1 + a2) * d2)
    return math.sqrt(tot)


def gaussian_convolution(a, b):
    """(exp(-a r^2) * exp(-b r^2))(r) = (pi/(a+b))^{3/2} exp(-ab/(a+b) r^2): (coeff, expnt)."""
    return (math.pi / (a + b)) ** 1.5, a * b / (a + b)


def coulomb_potential_unit_gaussian(a, r):
    """int (a/pi)^{3/2} exp(-a|y|^2) / |x - y| dy at |x| = r."""
    r = np.asarray(r, dtype=np.float64)
    sa = math.sqrt(a)
    small = r < 1e-8
    rs = np.where(small, 1.0, r)
    return np.where(small, 2.0 * sa / math.sqrt(math.pi), erf(sa * rs) / rs)


def yukawa_potential_unit_gaussian(a, mu, r):
    """int (a/pi)^{3/2} exp(-a|y|^2) exp(-mu|x-y|) / |x - y| dy at |x| = r.

    V = [e^{mu^2/(4a) - mu r} erfc(z0 - sqrt(a) r) - e^{mu^2/(4a) + mu r} erfc(z0 + sqrt(a) r)]
        / (2r),  z0 = mu / (2 sqrt a); each term is evaluated in the form that neither
    overflows nor cancels (erfcx for positive arguments).
    """
    r = np.maximum(np.asarray(r, dtype=np.float64), 1e-6)
    sa = math.sqrt(a)
    z0 = mu / (2.0 * sa)
    u = z0 - sa * r
    g = np.exp(-a * r * r)
    t1 = np.where(u >= 0.0, erfcx(np.maximum(u, 0.0)) * g,
                  np.exp(mu * mu / (4.0 * a) - mu * r) * erfc(np.minimum(u, 0.0)))
    t2 = erfcx(z0 + sa * r) * g
    return (t1 - t2) / (2.0 * r)


def project_callable(fn, k, cell, keys, npts=None, panels=2):
    """s_T = int fn(x) phi_T(x) dx by tensor Gauss-Legendre (panels^3 sub-cubes per box).

    fn maps an (..., 3) array of points to values.  Used only to build reference
    coefficients of smooth analytic functions.
    """
    lo, hi = cell
    if npts is None:
        npts = k + 8
    u1, w1 = [], []
    for p in range(panels):
        u, w = gauss_legendre(npts, p / panels, (p + 1) / panels)
        u1.append(u)
        w1.append(w)
    u1 = np.concatenate(u1)
    w1 = np.concatenate(w1)
    ph = phi(k, u1)                      # (k, nq)
    out = {}
    for key in keys:
        n, lx, ly, lz = key
        h = (hi - lo) / 2.0 ** n
        xs = lo + h * (lx + u1)
        ys = lo + h * (ly + u1)
        zs = lo + h * (lz + u1)
        X, Y, Z = np.meshgrid(xs, ys, zs, indexing='ij')
        vals = fn(np.stack([X, Y, Z], axis=-1)) * (w1[:, None, None] * w1[None, :, None] * w1[None, None, :])
        s = np.einsum('ia,jb,mc,abc->ijm', ph, ph, ph, vals, optimize=True)
        out[key] = s * h ** 1.5
    return out
