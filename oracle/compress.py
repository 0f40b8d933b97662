"""Wavelet (compressed) form of a function, reconstruction and truncation (paper Sec. 2.2
fast wavelet transform; Sec. 2.1 adaptive representation).  Test infrastructure: only the
test suite, the smoke check and the benchmark's CPU baseline use this package.

A function on a full octree is stored by the scaling coefficients of its leaves.  The
two-scale relation gives, for every refined box P with children block B_P (the 8
children's coefficients as one (2k)^3 block),

    s_P = (H x H x H) B_P          (filter, H = [h0 | h1])
    D_P = B_P - (H^T x H^T x H^T) s_P,

where D_P is the wavelet part of P written in the children basis: the children block is the
parent's polynomial plus D_P, and the two are orthogonal.  The compressed form is the root's
s and D_P of every refined box; reconstruction rebuilds every children block top-down as
unfilter(s_P) + D_P.  Parseval: ||f||^2 = ||s_root||^2 + sum_P ||D_P||^2.

Truncation (reading; the paper states only that small wavelet coefficients are discarded):
a refined box whose children are all leaves and whose ||D_P||_F <= tol loses its children
and becomes a leaf holding s_P; the rule is applied bottom-up, so a box can become a leaf
only after all its refined descendants have.  The same norm and the same non-strict
comparison as the refinement rule of the projection (which refines iff the norm exceeds
thresh).  The truncation error is exactly the norm of the discarded D_P (orthogonality).
"""
import numpy as np

from .basis import filter_matrix
from .tree import Function, assemble_block, children, split_block, unfilter3


class Compressed:
    """Root scaling coefficients and D_P (2k, 2k, 2k) of every refined box."""

    def __init__(self, k, cell, root, details):
        self.k = k
        self.cell = cell
        self.root = root
        self.details = details

    def norm2(self):
        tot = float(np.sum(self.root ** 2))
        tot += sum(float(np.sum(d ** 2)) for d in self.details.values())
        return float(np.sqrt(tot))


def compress(f):
    """Wavelet form of f: s at the root and D_P of every refined box."""
    hm = filter_matrix(f.k)
    coeff = f.filtered_interior()
    details = {}
    for key in f.interior():
        B = assemble_block([coeff[c] for c in children(key)], f.k)
        details[key] = B - unfilter3(coeff[key], hm)
    root = coeff[(0, 0, 0, 0)] if (0, 0, 0, 0) in coeff else f.leaves[(0, 0, 0, 0)]
    return Compressed(f.k, f.cell, root.copy(), details)


def reconstruct(c):
    """Leaves of the function whose wavelet form is c (top-down, unfilter plus details)."""
    hm = filter_matrix(c.k)
    s = {(0, 0, 0, 0): c.root}
    leaves = {}
    frontier = [(0, 0, 0, 0)]
    while frontier:
        key = frontier.pop()
        if key in c.details:
            blk = unfilter3(s[key], hm) + c.details[key]
            for ck, cv in zip(children(key), split_block(blk, c.k)):
                s[ck] = cv
                frontier.append(ck)
        else:
            leaves[key] = s[key]
    return Function(c.k, c.cell, leaves)


def truncate(f, tol):
    """f with the wavelet parts D_P <= tol of boxes whose children are leaves removed,
    bottom-up; returns (truncated function, sum of the squared norms removed)."""
    c = compress(f)
    refined = set(c.details)
    removed = 0.0
    for key in sorted(c.details, key=lambda q: -q[0]):
        if any(ch in refined for ch in children(key)):
            continue
        nrm2 = float(np.sum(c.details[key] ** 2))
        if np.sqrt(nrm2) <= tol:
            refined.discard(key)
            removed += nrm2
    kept = {q: d for q, d in c.details.items() if q in refined}
    return reconstruct(Compressed(c.k, c.cell, c.root, kept)), removed
