"""Separated-operator apply in standard and non-standard form (paper Sec. 2.2-2.3).

Operator: K(r) = sum_mu c_mu exp(-t_mu r^2).  Each term is a product of three 1D kernels,
so its matrix between a target box T and a source box S is the Kronecker product of three
1D blocks (Sec. 2.3: O(M (2k)^{D+1}) work instead of O((2k)^{2D})).

Standard form at level n (T^n = P^n T P^n):
    out_T = sum_{delta} sum_mu c_mu (t^{n,dx} x t^{n,dy} x t^{n,dz}) s_{T - delta}.

Non-standard form (T^N = T^0 + sum_m (A^m + B^m + C^m), Sec. 2.2), written in the children
basis: A^m + B^m + C^m = T^{m+1} - T^m restricted to the boxes that are refined at level m.
Reading of how the paper's decomposition is carried out on an adaptive tree:

  for every refined (interior) box P at level n, every displacement delta with target
  T = P + delta inside the cell (free-space boundary conditions: targets outside are
  dropped), every term mu that survives screening:
      acc_T += c_mu (R^{n,dx} x R^{n,dy} x R^{n,dz}) B_P          (children of T, level n+1)
      sub_T -= c_mu (t^{n,dx} x t^{n,dy} x t^{n,dz}) s_P          (box T, level n; n > 0 only)

and the result is reconstructed top-down (sum-down): a box's value is what it inherits
from its parent plus sub_T; its children inherit the unfiltered value plus acc_T.  On a
uniform depth-N tree without screening this equals the standard form at level N exactly.

Screening (reading; the paper only states the decay rates of A, B, C): with
a = ||t||_2, e = ||R - H^T t H||_2, r = ||R||_2 per dimension,
    N(delta) = prod_d (a_d + e_d) - prod_d a_d   (n > 0),   prod_d r_d   (n = 0),
    eta(P, delta, mu) = |c_mu| N(delta) ||B_P||_F,
eta bounds the Frobenius norm of the triple's contribution (the operator part that is not
already applied at level n is a sum of Kronecker products with at least one E = R - H^T t H
factor).  A triple is kept iff eta >= tau_drop.  Candidate displacements are enumerated with
rigorous bounds on a + e and on e (blocks.e_bound, blocks.decay_bound), which never remove a
triple with eta >= tau_drop.
"""
import numpy as np

from .basis import filter_matrix
from .blocks import BlockFactory, e_bound, decay_bound
from .tree import Function, children, parent, split_block, unfilter3, assemble_block


class SeparatedOperator:
    """sum_mu c_mu exp(-t_mu r^2)."""

    def __init__(self, c, t):
        self.c = np.asarray(c, dtype=np.float64)
        self.t = np.asarray(t, dtype=np.float64)

    def __len__(self):
        return len(self.c)


def mode_apply(rx, ry, rz, x):
    """y[p,a,b,c] = sum_{i,j,m} rx[a,i] ry[b,j] rz[c,m] x[p,i,j,m] (three mode products)."""
    p, ni, nj, nm = x.shape
    y = np.matmul(rx, x.reshape(p, ni, nj * nm)).reshape(p, rx.shape[0], nj, nm)
    y = np.matmul(ry, y)                       # (p, a, b, m)
    return np.matmul(y, rz.T)                  # (p, a, b, c)


# --------------------------------------------------------------------------- standard form

def apply_standard(f, op, level, disp_radius=1):
    """Standard-form apply on a uniform level-`level` tree, displacements |delta|_inf <= r."""
    k = f.k
    nb = 2 ** level
    bf = BlockFactory(k, f.width)
    s = np.zeros((nb, nb, nb, k, k, k))
    for (n, lx, ly, lz), v in f.leaves.items():
        assert n == level, "standard-form apply needs a uniform tree"
        s[lx, ly, lz] = v
    out = np.zeros_like(s)
    rng = range(-disp_radius, disp_radius + 1)
    triples = 0
    for mu in range(len(op)):
        for dx in rng:
            for dy in rng:
                for dz in rng:
                    # targets T with T - delta inside the cell, per axis
                    tsl, ssl = [], []
                    for d in (dx, dy, dz):
                        lo_t, hi_t = max(0, d), min(nb, nb + d)
                        tsl.append(slice(lo_t, hi_t))
                        ssl.append(slice(lo_t - d, hi_t - d))
                    if any(sl.stop <= sl.start for sl in tsl):
                        continue
                    tx = op.c[mu] * bf.t_block(level, dx, op.t[mu])
                    ty = bf.t_block(level, dy, op.t[mu])
                    tz = bf.t_block(level, dz, op.t[mu])
                    src = s[ssl[0], ssl[1], ssl[2]]
                    shp = src.shape
                    y = mode_apply(tx, ty, tz, src.reshape((-1, k, k, k)))
                    out[tsl[0], tsl[1], tsl[2]] += y.reshape(shp)
                    triples += shp[0] * shp[1] * shp[2]
    leaves = {(level, lx, ly, lz): out[lx, ly, lz].copy()
              for lx in range(nb) for ly in range(nb) for lz in range(nb)}
    stats = {"triples": triples, "useful_flops": triples * 6.0 * k ** 4}
    return Function(k, f.cell, leaves), stats


# ------------------------------------------------------------------------ non-standard form

class _Level:
    """Interior boxes of one level with their children blocks, s and block norms."""

    def __init__(self, n, keys, blocks, svals):
        self.n = n
        self.keys = keys
        self.pos = np.array([kk[1:] for kk in keys], dtype=np.int64).reshape(-1, 3)
        self.B = blocks
        self.s = svals
        self.bn = np.sqrt(np.sum(blocks.reshape(len(keys), -1) ** 2, axis=1))
        self.index = {kk: i for i, kk in enumerate(keys)}


def filter_up(f):
    """Per level: interior boxes, children blocks B_P, s_P = (H x H x H) B_P, ||B_P||_F."""
    coeff = f.filtered_interior()
    inter = f.interior()
    levels = {}
    for n in sorted({kk[0] for kk in inter}):
        keys = sorted(kk for kk in inter if kk[0] == n)
        blocks = np.stack([assemble_block([coeff[c] for c in children(kk)], f.k) for kk in keys])
        svals = np.stack([coeff[kk] for kk in keys])
        levels[n] = _Level(n, keys, blocks, svals)
    return levels


def _code(pos, n):
    return (pos[..., 0] << 42) | (pos[..., 1] << 21) | pos[..., 2]


def screen_level(bf, lev, op, tau, k, target_codes=None):
    """Kept triples of one level as groups (mu, (dx, dy, dz), source indices).

    target_codes: optional sorted array of target codes; only triples whose target is in
    the set are returned (used to evaluate sampled outputs).
    """
    n = lev.n
    nb = 2 ** n
    h = bf.h(n)
    maxb = float(lev.bn.max())
    groups = []
    for mu in range(len(op)):
        c = abs(float(op.c[mu]))
        texp = float(op.t[mu])
        beta = texp * h * h
        ab = 2.0 * h
        if n > 0:
            if c * maxb * 3.0 * e_bound(k, h, beta) * ab * ab < tau:
                continue
            fac = 3.0
        else:
            fac = 1.0
        dmax = 0
        while dmax + 1 <= nb - 1 and c * maxb * fac * ab * ab * decay_bound(h, beta, dmax + 1) >= tau:
            dmax += 1
        tab = np.array([bf.norms(n, d, texp) for d in range(dmax + 1)])  # (D+1, 3): a, e, r
        a, e, r = tab[:, 0], tab[:, 1], tab[:, 2]
        if n > 0:
            ae = a + e
            N = (ae[:, None, None] * ae[None, :, None] * ae[None, None, :]
                 - a[:, None, None] * a[None, :, None] * a[None, None, :])
        else:
            N = r[:, None, None] * r[None, :, None] * r[None, None, :]
        rng = np.arange(-dmax, dmax + 1)
        for dx in rng:
            for dy in rng:
                nxy = N[abs(dx), abs(dy)]
                for dz in rng:
                    nv = nxy[abs(dz)]
                    if c * nv * maxb < tau:
                        continue
                    sel = c * nv * lev.bn >= tau
                    delta = np.array([dx, dy, dz])
                    tgt = lev.pos + delta
                    sel &= np.all((tgt >= 0) & (tgt < nb), axis=1)
                    if target_codes is not None and sel.any():
                        codes = _code(tgt, n)
                        ix = np.searchsorted(target_codes, codes)
                        ix = np.minimum(ix, len(target_codes) - 1)
                        sel &= target_codes[ix] == codes
                    idx = np.nonzero(sel)[0]
                    if len(idx):
                        groups.append((mu, (int(dx), int(dy), int(dz)), idx))
    return groups


def nonstandard_contributions(f, op, tau_drop, sample_targets=None, only_levels=None,
                              levels=None, blocks=None):
    """acc_T (children basis) and sub_T for every target (or for the sampled targets).

    Returns (levels, contrib, stats) where contrib[n] = (target_keys, acc, sub) with
    acc of shape (NT, 2k, 2k, 2k) and sub of shape (NT, k, k, k).  only_levels restricts
    the source levels that are processed; levels / blocks may pass a previous filter_up
    result and BlockFactory.
    """
    k = f.k
    bf = blocks if blocks is not None else BlockFactory(k, f.width)
    if levels is None:
        levels = filter_up(f)
    contrib = {}
    stats = {"triples": 0, "useful_flops": 0.0, "per_level": {}}
    for n, lev in levels.items():
        if only_levels is not None and n not in only_levels:
            continue
        tcodes = None
        if sample_targets is not None:
            want = np.array([kk[1:] for kk in sample_targets if kk[0] == n], dtype=np.int64).reshape(-1, 3)
            if len(want) == 0:
                continue
            tcodes = np.unique(_code(want, n))
        groups = screen_level(bf, lev, op, tau_drop, k, tcodes)
        if not groups:
            continue
        allt = np.concatenate([_code(lev.pos[idx] + np.array(d), n) for (_, d, idx) in groups])
        tcode_u = np.unique(allt)
        nt = len(tcode_u)
        acc = np.zeros((nt, 2 * k, 2 * k, 2 * k))
        sub = np.zeros((nt, k, k, k))
        count = 0
        for (mu, d, idx) in groups:
            cmu, texp = float(op.c[mu]), float(op.t[mu])
            ti = np.searchsorted(tcode_u, _code(lev.pos[idx] + np.array(d), n))
            rx = cmu * bf.r_block(n, d[0], texp)
            ry = bf.r_block(n, d[1], texp)
            rz = bf.r_block(n, d[2], texp)
            acc[ti] += mode_apply(rx, ry, rz, lev.B[idx])      # targets distinct within a group
            if n > 0:
                tx = cmu * bf.t_block(n, d[0], texp)
                ty = bf.t_block(n, d[1], texp)
                tz = bf.t_block(n, d[2], texp)
                sub[ti] -= mode_apply(tx, ty, tz, lev.s[idx])
            count += len(idx)
        keys = [(n, int(cc >> 42), int((cc >> 21) & ((1 << 21) - 1)), int(cc & ((1 << 21) - 1)))
                for cc in tcode_u]
        contrib[n] = (keys, acc, sub)
        flops = count * (6.0 * (2 * k) ** 4 + (6.0 * k ** 4 if n > 0 else 0.0))
        stats["triples"] += count
        stats["useful_flops"] += flops
        stats["per_level"][n] = {"triples": count, "targets": nt, "groups": len(groups)}
    return levels, contrib, stats


def output_tree_nodes(contrib):
    """Nodes of the output tree: targets, their 8 children, ancestors, closed under siblings.
    The root is always present (it is the ancestor of every box; with no target at all the
    result is the zero function on the root)."""
    nodes = {(0, 0, 0, 0)}
    for n, (keys, acc, sub) in contrib.items():
        for kk in keys:
            nodes.add(kk)
            nodes.update(children(kk))
    # ancestors and siblings
    frontier = list(nodes)
    while frontier:
        kk = frontier.pop()
        if kk[0] == 0:
            continue
        p = parent(kk)
        for sib in children(p):
            if sib not in nodes:
                nodes.add(sib)
                frontier.append(sib)
        if p not in nodes:
            nodes.add(p)
            frontier.append(p)
    return nodes


def sum_down(k, cell, contrib, nodes):
    """Top-down reconstruction of the result on the leaves of the output tree."""
    hm = filter_matrix(k)
    accd, subd = {}, {}
    for n, (keys, acc, sub) in contrib.items():
        for i, kk in enumerate(keys):
            accd[kk] = acc[i]
            subd[kk] = sub[i]
    has_kids = {parent(kk) for kk in nodes if kk[0] > 0}
    inherited = {}
    leaves = {}
    for kk in sorted(nodes, key=lambda q: q[0]):
        v = inherited.pop(kk, np.zeros((k, k, k)))
        if kk in subd:
            v = v + subd[kk]
        if kk in has_kids:
            blk = unfilter3(v, hm)
            if kk in accd:
                blk = blk + accd[kk]
            for ck, cv in zip(children(kk), split_block(blk, k)):
                inherited[ck] = cv
        else:
            assert kk not in accd
            leaves[kk] = v
    return Function(k, cell, leaves)


def apply_nonstandard(f, op, tau_drop):
    """Full non-standard apply: filter-up, screening, contributions, sum-down."""
    _, contrib, stats = nonstandard_contributions(f, op, tau_drop)
    nodes = output_tree_nodes(contrib)
    return sum_down(f.k, f.cell, contrib, nodes), stats


def sampled_leaves(f, op, tau_drop, leaf_keys):
    """Result on selected output leaves, computing only the contributions on their paths.

    Every leaf's value depends only on sub_A for A on its root path (A = leaf included) and
    on acc_A of its proper ancestors.  Returns ({leaf: coeffs}, {leaf: has_acc}) where
    has_acc tells whether the box received children contributions (then it is not a leaf).
    """
    k = f.k
    hm = filter_matrix(k)
    want = set()
    for kk in leaf_keys:
        p = kk
        want.add(p)
        while p[0] > 0:
            p = parent(p)
            want.add(p)
    _, contrib, stats = nonstandard_contributions(f, op, tau_drop, sample_targets=want)
    accd, subd = {}, {}
    for n, (keys, acc, sub) in contrib.items():
        for i, kk in enumerate(keys):
            accd[kk] = acc[i]
            subd[kk] = sub[i]
    out, has_acc = {}, {}
    for leaf in leaf_keys:
        path = [leaf]
        while path[-1][0] > 0:
            path.append(parent(path[-1]))
        path.reverse()
        v = np.zeros((k, k, k))
        for depth, kk in enumerate(path):
            if kk in subd:
                v = v + subd[kk]
            if depth + 1 < len(path):
                blk = unfilter3(v, hm)
                if kk in accd:
                    blk = blk + accd[kk]
                child = path[depth + 1]
                c = children(kk).index(child)
                v = split_block(blk, k)[c]
        out[leaf] = v
        has_acc[leaf] = leaf in accd
    return out, has_acc, stats
