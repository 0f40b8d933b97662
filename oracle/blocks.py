"""1D operator blocks of one Gaussian term (paper Sec. 2.2 Toeplitz structure, Sec. 2.3).

For the kernel exp(-t (x - y)^2) and level-n boxes of width h_n, the matrix element between
target box l_T (index i) and source box l_S (index j) depends only on delta = l_T - l_S
(translation invariance gives Toeplitz blocks):

  t^{n,delta}[i, j] = int int phi^n_{l_T,i}(x) exp(-t (x-y)^2) phi^n_{l_S,j}(y) dx dy
                    = h_n int_{-1}^{1} exp(-beta (delta + w)^2) C_ij(w) dw,   beta = t h_n^2,
  C_ij(w)          = int_{max(0,w)}^{min(1,1+w)} phi_i(u) phi_j(u - w) du.

Reading of the quadrature: C_ij is a polynomial in u on the overlap, evaluated exactly by
k-point Gauss-Legendre; the outer integral is split at w = 0 (where C changes form) and at
the Gaussian peak w = -delta, restricted to where the Gaussian exceeds
exp(-50)/sqrt(1+beta) of its peak, and done by composite Gauss-Legendre with 2k+20 nodes
per panel of width <= min(1, beta^{-1/2}).

The non-standard block R^{n,delta} (2k x 2k) is the level-(n+1) operator between the
children of the target and of the source: rows (b, i) for target child b, columns (a, j)
for source child a, block (b, a) = t^{n+1, 2 delta + b - a}.  Its projection onto the
parents is H R H^T = t^{n,delta} (H = [h0 | h1]).

Norms used for screening: a = ||t^{n,delta}||_2, e = ||R^{n,delta} - H^T t^{n,delta} H||_2
and r = ||R^{n,delta}||_2.
"""
import math

import numpy as np

from .basis import gauss_legendre, phi, filter_matrix


def _support_halfwidth(beta):
    if beta <= 0.0:
        return math.inf
    return math.sqrt((50.0 + 0.5 * math.log1p(beta)) / beta)


class BlockFactory:
    """Computes and caches t^{n,delta}, R^{n,delta} and their norms for one cell width."""

    def __init__(self, k, width):
        self.k = k
        self.width = float(width)
        self.hm = filter_matrix(k)
        self.xg, self.wg = gauss_legendre(k, 0.0, 1.0)
        self._t = {}
        self._r = {}
        self._norms = {}

    def h(self, n):
        return self.width / 2.0 ** n

    def corr(self, w):
        """C_ij(w) for an array of w in [-1, 1]; shape (len(w), k, k)."""
        w = np.asarray(w, dtype=np.float64)
        lo = np.maximum(0.0, w)
        hi = np.minimum(1.0, 1.0 + w)
        u = lo[:, None] + (hi - lo)[:, None] * self.xg[None, :]
        wt = (hi - lo)[:, None] * self.wg[None, :]
        pi = phi(self.k, u)            # (k, nw, ng)
        pj = phi(self.k, u - w[:, None])
        return np.einsum('ing,jng,ng->nij', pi, pj, wt)

    def t_block(self, n, delta, texp):
        """t^{n,delta} (k x k) for exp(-texp r^2), without the term's coefficient."""
        key = (n, int(delta), float(texp))
        if key in self._t:
            return self._t[key]
        h = self.h(n)
        beta = texp * h * h
        half = _support_halfwidth(beta)
        wc = -float(delta)
        width = min(1.0, 1.0 / math.sqrt(beta)) if beta > 0 else 1.0
        ws, wts = [], []
        for (a, b) in ((-1.0, 0.0), (0.0, 1.0)):
            a2, b2 = max(a, wc - half), min(b, wc + half)
            if b2 <= a2:
                continue
            cuts = [a2, b2]
            if a2 < wc < b2:
                cuts = [a2, wc, b2]
            for p in range(len(cuts) - 1):
                pa, pb = cuts[p], cuts[p + 1]
                npan = max(1, int(math.ceil((pb - pa) / width)))
                edges = np.linspace(pa, pb, npan + 1)
                for q in range(npan):
                    x, wq = gauss_legendre(2 * self.k + 20, edges[q], edges[q + 1])
                    ws.append(x)
                    wts.append(wq)
        if not ws:
            blk = np.zeros((self.k, self.k))
        else:
            w = np.concatenate(ws)
            wq = np.concatenate(wts) * np.exp(-beta * (float(delta) + w) ** 2)
            blk = h * np.einsum('n,nij->ij', wq, self.corr(w))
        self._t[key] = blk
        return blk

    def r_block(self, n, delta, texp):
        """R^{n,delta} (2k x 2k): level-(n+1) blocks between children (rows target child)."""
        key = (n, int(delta), float(texp))
        if key in self._r:
            return self._r[key]
        k = self.k
        r = np.zeros((2 * k, 2 * k))
        for b in (0, 1):
            for a in (0, 1):
                r[b * k:(b + 1) * k, a * k:(a + 1) * k] = self.t_block(n + 1, 2 * delta + b - a, texp)
        self._r[key] = r
        return r

    def norms(self, n, delta, texp):
        """(a, e, r): ||t||_2, ||R - H^T t H||_2, ||R||_2 for level n, displacement delta."""
        key = (n, abs(int(delta)), float(texp))
        if key in self._norms:
            return self._norms[key]
        t = self.t_block(n, abs(delta), texp)
        r = self.r_block(n, abs(delta), texp)
        e = r - self.hm.T @ t @ self.hm
        out = (float(np.linalg.norm(t, 2)), float(np.linalg.norm(e, 2)), float(np.linalg.norm(r, 2)))
        self._norms[key] = out
        return out


# Cramer's inequality |H_n(x)| exp(-x^2/2) <= 1.086435 sqrt(2^n n!), rounded up.
_CRAMER = 1.0865


def e_bound(k, h, beta):
    """Rigorous bound on e = ||R - H^T t H|| for any displacement.

    e <= ||(I - P^n x P^n) K||_{L2} <= ||(I-P_x)K|| + ||(I-P_y)K||, each bounded by the
    Taylor remainder of order k about the box centre: h * sup|K^(k)| (h/2)^k / k!, with
    sup|d^k/du^k exp(-t u^2)| <= 1.0865 t^{k/2} sqrt(2^k k!).  Also e <= ||K||_{L2} <= h.
    """
    v = 2.0 * _CRAMER * h * beta ** (0.5 * k) / math.sqrt(2.0 ** k * math.factorial(k))
    return min(h, v)


def decay_bound(h, beta, delta):
    """Rigorous bound on a + e (and on r) at 1D displacement delta: 2 h max K on the box pair."""
    d = abs(int(delta))
    if d == 0:
        return 2.0 * h
    return 2.0 * h * math.exp(-beta * (d - 1) ** 2)
