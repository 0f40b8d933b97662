"""Function trees for the oracle (paper Sec. 2.1; Sec. 3.1 example: trace, norm2, inner).

A function on the cubic cell [lo, hi]^3 is stored by the scaling coefficients of the
leaves of a full octree: every box that is refined has all 8 children.  Box keys are
tuples (n, lx, ly, lz) with 0 <= l < 2^n.  A leaf holds a (k, k, k) array s[i, j, m],
the coefficient of phi^n_{lx,i}(x) phi^n_{ly,j}(y) phi^n_{lz,m}(z).

Children are numbered c = 4*bx + 2*by + bz; the (2k)^3 "children block" of a box puts
child c's coefficients at rows (bx*k + i, by*k + j, bz*k + m).
"""
import numpy as np

from .basis import filter_matrix


def children(key):
    n, lx, ly, lz = key
    return [(n + 1, 2 * lx + bx, 2 * ly + by, 2 * lz + bz)
            for bx in (0, 1) for by in (0, 1) for bz in (0, 1)]


def parent(key):
    n, lx, ly, lz = key
    return (n - 1, lx >> 1, ly >> 1, lz >> 1)


def morton(key):
    """Level-prefixed Morton code: (1 << 3n) | interleave(lx, ly, lz), x in the top bit."""
    n, lx, ly, lz = key
    code = 0
    for b in range(n):
        code |= ((lx >> b) & 1) << (3 * b + 2)
        code |= ((ly >> b) & 1) << (3 * b + 1)
        code |= ((lz >> b) & 1) << (3 * b)
    return (1 << (3 * n)) | code


def assemble_block(kids, k):
    """(2k)^3 children block from the 8 child coefficient arrays (ordered c = 4bx+2by+bz)."""
    b = np.zeros((2 * k, 2 * k, 2 * k))
    for c, s in enumerate(kids):
        bx, by, bz = (c >> 2) & 1, (c >> 1) & 1, c & 1
        b[bx * k:(bx + 1) * k, by * k:(by + 1) * k, bz * k:(bz + 1) * k] = s
    return b


def split_block(b, k):
    """Inverse of assemble_block."""
    out = []
    for c in range(8):
        bx, by, bz = (c >> 2) & 1, (c >> 1) & 1, c & 1
        out.append(b[bx * k:(bx + 1) * k, by * k:(by + 1) * k, bz * k:(bz + 1) * k].copy())
    return out


def filter3(b, hm):
    """Parent scaling coefficients s = (H x H x H) B from a children block (Sec. 2.2 two-scale)."""
    return np.einsum('ia,jb,mc,abc->ijm', hm, hm, hm, b, optimize=True)


def unfilter3(s, hm):
    """Children block of the parent's polynomial: B = (H^T x H^T x H^T) s."""
    return np.einsum('ia,jb,mc,ijm->abc', hm, hm, hm, s, optimize=True)


class Function:
    """Leaves of a full octree with k^3 scaling coefficients each."""

    def __init__(self, k, cell, leaves):
        self.k = k
        self.cell = (float(cell[0]), float(cell[1]))
        self.leaves = leaves

    @property
    def width(self):
        return self.cell[1] - self.cell[0]

    def box_size(self, n):
        return self.width / 2.0 ** n

    def max_level(self):
        return max(key[0] for key in self.leaves)

    def interior(self):
        """All proper ancestors of leaves (the refined boxes)."""
        out = set()
        for key in self.leaves:
            p = key
            while p[0] > 0:
                p = parent(p)
                if p in out:
                    break
                out.add(p)
        return out

    def filtered_interior(self):
        """Scaling coefficients s of every interior box, by filtering bottom-up."""
        hm = filter_matrix(self.k)
        coeff = dict(self.leaves)
        inter = sorted(self.interior(), key=lambda kk: -kk[0])
        for key in inter:
            coeff[key] = filter3(assemble_block([coeff[c] for c in children(key)], self.k), hm)
        return coeff

    def norm2(self):
        """||f||_2 = sqrt(sum over leaves of ||s||^2) (orthonormal basis)."""
        return float(np.sqrt(sum(float(np.sum(s * s)) for s in self.leaves.values())))

    def trace(self):
        """int f = sum over leaves of s_000 h_n^{3/2}, since int phi^n_{l,0} = h_n^{1/2}."""
        return float(sum(s[0, 0, 0] * self.box_size(key[0]) ** 1.5
                         for key, s in self.leaves.items()))

    def values_on(self, keys):
        """Coefficients of this function on boxes at or below its leaves (unfiltering down)."""
        hm = filter_matrix(self.k)
        out = {}
        cache = {}

        def get(key):
            if key in self.leaves:
                return self.leaves[key]
            if key in cache:
                return cache[key]
            if key[0] == 0:
                raise KeyError("box %r is above the tree's leaves" % (key,))
            p = parent(key)
            ps = get(p)
            kids = split_block(unfilter3(ps, hm), self.k)
            for c, ck in enumerate(children(p)):
                cache[ck] = kids[c]
            return cache[key]

        for key in keys:
            out[key] = get(key)
        return out


def union_leaves(f, g):
    """Leaves of the union of two full octrees over the same cell."""
    fi, gi = f.interior(), g.interior()
    inter = fi | gi
    out = set()
    for key in list(f.leaves) + list(g.leaves):
        if key not in inter:
            out.add(key)
    return sorted(out)


def inner(f, g):
    """<f, g> on the union of the two trees (Sec. 3.1 example, 'inner')."""
    assert f.k == g.k and f.cell == g.cell
    keys = union_leaves(f, g)
    fv, gv = f.values_on(keys), g.values_on(keys)
    return float(sum(float(np.sum(fv[kk] * gv[kk])) for kk in keys))
