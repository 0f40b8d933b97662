"""Pin of the oracle's screening enumeration (CPU only).

`oracle.apply.screen_level` does not visit every (box, displacement, term) triple: it skips
terms and displacements with rigorous bounds (the Taylor bound on e and the Gaussian decay
bound on a + e) and walks the displacement cube only up to the largest 1D displacement the
bounds allow.  Here every triple of small adaptive trees is enumerated by brute force, with
eta = |c_mu| N(delta) ||B_P||_F computed for all of them (N from the block norms of every
displacement in the cube, targets outside the cell dropped), and the kept set must equal
the oracle's exactly, at thresholds that keep from a handful to most of the triples.
"""
import numpy as np
import pytest

from oracle.apply import SeparatedOperator, filter_up, screen_level
from oracle.blocks import BlockFactory
from oracle.fit import coulomb_fit, bsh_fit, cell_r_hi
from oracle.projection import GaussianSum, project_adaptive

CELL = (-10.0, 10.0)


def _brute_force(bf, lev, op, tau):
    """Every (mu, delta, P) with eta >= tau, eta evaluated for every triple."""
    n = lev.n
    nb = 2 ** n
    D = nb - 1
    kept = set()
    rng = np.arange(-D, D + 1)
    for mu in range(len(op)):
        c = abs(float(op.c[mu]))
        texp = float(op.t[mu])
        tab = np.array([bf.norms(n, d, texp) for d in range(D + 1)])
        a, e, r = tab[:, 0], tab[:, 1], tab[:, 2]
        ad, ed, rd = a[np.abs(rng)], e[np.abs(rng)], r[np.abs(rng)]
        if n > 0:
            ae = ad + ed
            N = (ae[:, None, None] * ae[None, :, None] * ae[None, None, :]
                 - ad[:, None, None] * ad[None, :, None] * ad[None, None, :])
        else:
            N = rd[:, None, None] * rd[None, :, None] * rd[None, None, :]
        for p, pos in enumerate(lev.pos):
            eta = c * N * lev.bn[p]
            ix, iy, iz = np.nonzero(eta >= tau)
            for i, j, m in zip(ix, iy, iz):
                d = (int(rng[i]), int(rng[j]), int(rng[m]))
                t = pos + np.array(d)
                if np.all((t >= 0) & (t < nb)):
                    kept.add((mu, d, p))
    return kept


def _oracle_set(bf, lev, op, tau, k):
    out = set()
    for (mu, d, idx) in screen_level(bf, lev, op, tau, k):
        for p in idx:
            out.add((mu, tuple(d), int(p)))
    return out


CASES = [
    # k, thresh, operator kind, Gaussians (coeff, expnt, centre)
    (3, 3e-2, "coulomb", [(1.0, 2.0, (0.3, -0.4, 0.2)), (0.5, 20.0, (-3.1, 2.2, 4.0))]),
    (4, 1e-2, "bsh", [(1.0, 6.0, (1.3, 0.4, -0.2))]),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_screen_level_matches_brute_force(case):
    k, thresh, kind, gs = CASES[case]
    f = project_adaptive(GaussianSum([g[0] for g in gs], [g[1] for g in gs], [g[2] for g in gs]),
                         k, thresh, CELL, 1, 4)
    r_hi = cell_r_hi(*CELL)
    if kind == "coulomb":
        c, t = coulomb_fit(1e-3, 1e-4, r_hi)
    else:
        c, t = bsh_fit(1.2, 1e-3, 1e-4, r_hi)
    op = SeparatedOperator(c, t)
    bf = BlockFactory(k, CELL[1] - CELL[0])
    levels = filter_up(f)
    assert max(levels) >= 2, "the tree should have several refined levels"
    eta_max = max(float(np.max(lev.bn)) for lev in levels.values()) * float(np.max(np.abs(c))) * 8.0
    total = 0
    for rel in (1e-2, 1e-4, 1e-6, 1e-9):
        tau = rel * eta_max
        for n, lev in sorted(levels.items()):
            ref = _brute_force(bf, lev, op, tau)
            got = _oracle_set(bf, lev, op, tau, k)
            assert got == ref, "level %d, tau %.3e: %d missing, %d extra" % (
                n, tau, len(ref - got), len(got - ref))
            total += len(ref)
    assert total > 1000      # the thresholds reach deep into the candidate cubes
