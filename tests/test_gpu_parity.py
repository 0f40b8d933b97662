"""Parity of the HIP path (through the C ABI) against the FP64 oracle.  Needs an MI355X.

Tolerances: the pure-FP64 path must agree with the oracle to relative L2 <= 1e-12 over the
compared leaves (summation order differs; nothing else may).  Trees are compared exactly.
"""
import math
import sys

import numpy as np
import pytest

import mra_workloads as W
from oracle.analytic import gaussian_convolution
from oracle.apply import SeparatedOperator, apply_standard, apply_nonstandard, sampled_leaves
from oracle.fit import coulomb_fit, bsh_fit, cell_r_hi
from oracle.projection import GaussianSum, project_adaptive, project_uniform
from oracle.tree import morton, inner

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _key_tuple(code):
    code = int(code)
    n = (code.bit_length() - 1) // 3
    code ^= 1 << (3 * n)
    x = y = z = 0
    for b in range(n):
        x |= ((code >> (3 * b + 2)) & 1) << b
        y |= ((code >> (3 * b + 1)) & 1) << b
        z |= ((code >> (3 * b)) & 1) << b
    return (n, x, y, z)


def _as_dict(func):
    keys, co = func.export()
    return {_key_tuple(q): co[i] for i, q in enumerate(keys)}


def _rel_l2(got, ref, keys):
    num = math.sqrt(sum(float(np.sum((got[q] - ref[q]) ** 2)) for q in keys))
    den = math.sqrt(sum(float(np.sum(ref[q] ** 2)) for q in keys))
    return num / den


@pytest.fixture(scope="module")
def M():
    import paper_1507_01888_amd as mod
    mod.load()
    return mod


def test_standard_form_gaussian_k8(M):
    """Single-term k=8 standard-form apply on the uniform level-4 tree (4096 boxes)."""
    _say("case: standard form, k=8, level 4, 27 displacements")
    w = W.WORKLOADS["gauss_std_k8"]
    ctx = M.Context(0, W.CELL)
    f = ctx.project([w["f_coeff"]], [w["f_expnt"]], [[0, 0, 0]], w["k"], 1.0,
                    initial_level=w["level"], max_level=w["level"])
    op = ctx.op_gaussians(w["k"], w["op_c"], w["op_t"])
    g = ctx.apply(op, f, form="standard", disp_radius=w["disp_radius"])
    st = ctx.last_stats()
    assert st["triples"] == 46 ** 3
    fo = project_uniform(GaussianSum([w["f_coeff"]], [w["f_expnt"]], [[0, 0, 0]]), w["k"],
                         W.CELL, w["level"])
    fin = _as_dict(f)
    assert set(fin) == set(fo.leaves)
    assert _rel_l2(fin, fo.leaves, fo.leaves) < 1e-13
    go, _ = apply_standard(fo, SeparatedOperator(w["op_c"], w["op_t"]), w["level"], 1)
    got = _as_dict(g)
    assert set(got) == set(go.leaves)
    err = _rel_l2(got, go.leaves, go.leaves)
    _say("standard k=8 rel L2 vs oracle", err)
    assert err <= TOL
    # analytic check of the GPU result (27 displacements: truncation ~8e-3, see oracle test)
    cc, ee = gaussian_convolution(w["f_expnt"], w["op_t"][0])
    ex = project_uniform(GaussianSum([w["f_coeff"] * cc], [ee], [[0, 0, 0]]), w["k"], W.CELL, w["level"])
    assert 5e-3 < _rel_l2(got, ex.leaves, ex.leaves) < 1.2e-2
    # a wider displacement cube reaches the projection floor
    g3 = ctx.apply(op, f, form="standard", disp_radius=3)
    assert _rel_l2(_as_dict(g3), ex.leaves, ex.leaves) < 2e-6



def test_standard_form_clamped_radius_two_terms(M):
    """Standard form on the uniform level-2 tree (4^3 boxes), two terms, a displacement
    radius beyond the cube (the library clamps it to 2^level - 1; the oracle skips the
    empty displacements): every box then sees every box, per term."""
    _say("case: standard form, k=6, level 2, radius 5, 2 terms")
    k, level, radius = 6, 2, 5
    c, t = [1.0, 0.25], [0.05, 0.4]
    ctx = M.Context(0, W.CELL)
    f = ctx.project([1.0], [0.5], [[0.3, -0.2, 0.1]], k, 1.0, initial_level=level,
                    max_level=level)
    op = ctx.op_gaussians(k, c, t)
    g = ctx.apply(op, f, form="standard", disp_radius=radius)
    assert ctx.last_stats()["triples"] == 4 ** 3 * 4 ** 3 * len(c)
    fo = project_uniform(GaussianSum([1.0], [0.5], [[0.3, -0.2, 0.1]]), k, W.CELL, level)
    go, _ = apply_standard(fo, SeparatedOperator(c, t), level, radius)
    got = _as_dict(g)
    assert set(got) == set(go.leaves)
    err = _rel_l2(got, go.leaves, go.leaves)
    _say("standard clamped radius rel L2 vs oracle", err)
    assert err <= TOL

def test_paper_example_on_gpu(M):
    """Sec. 3.1 example: trace, norm2 and self-energy of exp(-r^2), and leaf parity."""
    _say("case: paper example, k=6, thresh 1e-4, Coulomb(1e-4, 1e-6)")
    cell = (-6.0, 6.0)
    ctx = M.Context(0, cell)
    g = ctx.project([1.0], [1.0], [[0, 0, 0]], 6, 1e-4)
    op = ctx.op_coulomb(6, 1e-4, 1e-6)
    vg = ctx.apply(op, g, tau_drop=1e-8)
    tr, nrm, en = ctx.trace(g), ctx.norm2(g), ctx.inner(g, vg)
    _say("trace", tr, "norm2", nrm, "energy", en)
    assert abs(tr - math.pi ** 1.5) < 1e-6 * math.pi ** 1.5
    assert abs(nrm - (math.pi / 2) ** 0.75) < 1e-6
    assert abs(en - math.pi ** 2.5 * math.sqrt(2)) < 1e-6 * 24.74
    # full parity of the output tree against the oracle
    go = project_adaptive(GaussianSum([1.0], [1.0], [[0, 0, 0]]), 6, 1e-4, cell, 2, 20)
    c, t = coulomb_fit(1e-4, 1e-6, cell_r_hi(*cell))
    ref, st = apply_nonstandard(go, SeparatedOperator(c, t), 1e-8)
    got = _as_dict(vg)
    assert set(got) == set(ref.leaves)
    assert ctx.last_stats()["triples"] == st["triples"]
    err = _rel_l2(got, ref.leaves, ref.leaves)
    _say("paper example rel L2 vs oracle", err)
    assert err <= TOL
    assert abs(en - inner(go, ref)) < 1e-12 * en


def test_coulomb_k10_reduced_full_parity(M):
    """k=10 Coulomb non-standard apply, 2 Gaussians at thresh 1e-5: every leaf compared."""
    _say("case: coulomb k=10 reduced (2 Gaussians, thresh 1e-5)")
    c, a, x = W.unit_charge_gaussians(1, 7, 2, 1.0, 30.0)
    ctx = M.Context(0, W.CELL)
    f = ctx.project(c, a, x, 10, 1e-5)
    op = ctx.op_coulomb(10, 1e-5, 1e-8)
    g = ctx.apply(op, f, tau_drop=1e-9)
    fo = project_adaptive(GaussianSum(c, a, x), 10, 1e-5, W.CELL, 2, 20)
    assert set(_as_dict(f)) == set(fo.leaves)
    cc, tt = coulomb_fit(1e-5, 1e-8, cell_r_hi(*W.CELL))
    oc, ot = op.terms()
    assert np.array_equal(oc.size, cc.size) and np.abs(oc / cc - 1).max() < 1e-14
    ref, st = apply_nonstandard(fo, SeparatedOperator(cc, tt), 1e-9)
    got = _as_dict(g)
    assert set(got) == set(ref.leaves)
    assert ctx.last_stats()["triples"] == st["triples"]
    err = _rel_l2(got, ref.leaves, ref.leaves)
    _say("coulomb k10 reduced rel L2 vs oracle", err, "triples", st["triples"])
    assert err <= TOL
    # norm2 through the reduction kernel
    assert abs(ctx.norm2(g) - ref.norm2()) < 1e-12 * ref.norm2()


def test_bsh_k10_reduced_full_parity(M):
    """k=10 bound-state Helmholtz apply of one batched-workload function (reduced thresh)."""
    c, a, x, mu = W.bsh_inputs(0)
    _say("case: bsh k=10, mu=%.3f, %d Gaussians, thresh 1e-4" % (mu, len(c)))
    ctx = M.Context(0, W.CELL)
    f = ctx.project(c, a, x, 10, 1e-4)
    op = ctx.op_bsh(10, mu, 1e-5, 1e-8)
    g = ctx.apply(op, f, tau_drop=1e-8)
    fo = project_adaptive(GaussianSum(c, a, x), 10, 1e-4, W.CELL, 2, 20)
    cc, tt = bsh_fit(mu, 1e-5, 1e-8, cell_r_hi(*W.CELL))
    ref, st = apply_nonstandard(fo, SeparatedOperator(cc, tt), 1e-8)
    got = _as_dict(g)
    assert set(got) == set(ref.leaves)
    err = _rel_l2(got, ref.leaves, ref.leaves)
    _say("bsh rel L2 vs oracle", err)
    assert err <= TOL


def test_deterministic_and_errors(M):
    _say("case: determinism and error codes")
    ctx = M.Context(0, W.CELL)
    c, a, x = W.unit_charge_gaussians(1, 3, 1, 2.0, 2.0)
    f = ctx.project(c, a, x, 8, 1e-4)
    op = ctx.op_coulomb(8, 1e-4, 1e-6)
    g1 = _as_dict(ctx.apply(op, f, tau_drop=1e-8))
    g2 = _as_dict(ctx.apply(op, f, tau_drop=1e-8))
    assert all(np.array_equal(g1[q], g2[q]) for q in g1)
    op6 = ctx.op_coulomb(6, 1e-4, 1e-6)
    with pytest.raises(M.MraError) as e:
        ctx.apply(op6, f, tau_drop=1e-8)
    assert e.value.code == -5
    f13 = ctx.project(c, a, x, 13, 1e-3)
    op13 = ctx.op_coulomb(13, 1e-4, 1e-6)
    with pytest.raises(M.MraError) as e:
        ctx.apply(op13, f13, tau_drop=1e-8)
    assert e.value.code == -4
    with pytest.raises(M.MraError) as e:
        ctx.project(c, a, x, 15, 1e-3)
    assert e.value.code == -1


def test_batched_bsh_matches_single_and_oracle(M):
    """Several functions with their own Helmholtz kernels in one batched apply: the same
    triples and trees as the one-at-a-time applies, values equal up to the summation order
    of split target lists (the split size depends on the batch), and parity with the oracle."""
    _say("case: batched bsh, 4 functions, k=10, thresh 1e-4")
    ctx = M.Context(0, W.CELL)
    funcs, ops, params = [], [], []
    for i in range(4):
        c, a, x, mu = W.bsh_inputs(i)
        funcs.append(ctx.project(c, a, x, 10, 1e-4))
        ops.append(ctx.op_bsh(10, mu, 1e-5, 1e-8))
        params.append((c, a, x, mu))
    outs = ctx.apply_batch(ops, funcs, tau_drop=1e-8)
    st = ctx.last_stats()
    tot = 0
    for i in range(4):
        single = ctx.apply(ops[i], funcs[i], tau_drop=1e-8)
        tot += ctx.last_stats()["triples"]
        a, b = _as_dict(outs[i]), _as_dict(single)
        assert set(a) == set(b)
        assert _rel_l2(a, b, b) <= 1e-14
    assert st["triples"] == tot
    c, a, x, mu = params[2]
    fo = project_adaptive(GaussianSum(c, a, x), 10, 1e-4, W.CELL, 2, 20)
    cc, tt = bsh_fit(mu, 1e-5, 1e-8, cell_r_hi(*W.CELL))
    ref, _ = apply_nonstandard(fo, SeparatedOperator(cc, tt), 1e-8)
    got = _as_dict(outs[2])
    assert set(got) == set(ref.leaves)
    err = _rel_l2(got, ref.leaves, ref.leaves)
    _say("batched bsh function 2 rel L2 vs oracle", err)
    assert err <= TOL


def test_pipelined_batch_plan(M, monkeypatch):
    """The chunked plan (target sets from the screening pre-pass, level-units planned and
    launched in chunks) forced on the small batched Helmholtz case: the same triples and
    trees as the one-piece plan, values equal up to the summation order of split lists, and
    parity with the oracle."""
    _say("case: batched bsh, 4 functions, chunked plan forced")
    ctx = M.Context(0, W.CELL)
    funcs, ops, params = [], [], []
    for i in range(4):
        c, a, x, mu = W.bsh_inputs(i)
        funcs.append(ctx.project(c, a, x, 10, 1e-4))
        ops.append(ctx.op_bsh(10, mu, 1e-5, 1e-8))
        params.append((c, a, x, mu))
    monkeypatch.setenv("MRA_PIPELINE_MIN", "1e30")
    one = ctx.apply_batch(ops, funcs, tau_drop=1e-8)
    st1 = ctx.last_stats()
    monkeypatch.setenv("MRA_PIPELINE_MIN", "0")
    piped = ctx.apply_batch(ops, funcs, tau_drop=1e-8)
    st2 = ctx.last_stats()
    monkeypatch.delenv("MRA_PIPELINE_MIN")
    assert st1["triples"] == st2["triples"] and st1["out_nodes"] == st2["out_nodes"]
    worst = 0.0
    for i in range(4):
        a, b = _as_dict(piped[i]), _as_dict(one[i])
        assert set(a) == set(b)
        worst = max(worst, _rel_l2(a, b, b))
    _say("chunked vs one-piece plan: worst rel L2 %.3e over 4 functions" % worst)
    assert worst <= 1e-14
    c, a, x, mu = params[1]
    fo = project_adaptive(GaussianSum(c, a, x), 10, 1e-4, W.CELL, 2, 20)
    cc, tt = bsh_fit(mu, 1e-5, 1e-8, cell_r_hi(*W.CELL))
    ref, _ = apply_nonstandard(fo, SeparatedOperator(cc, tt), 1e-8)
    got = _as_dict(piped[1])
    assert set(got) == set(ref.leaves)
    err = _rel_l2(got, ref.leaves, ref.leaves)
    _say("chunked plan, function 1 rel L2 vs oracle", err)
    assert err <= TOL


def test_coulomb_k12_reduced_full_parity(M):
    """k=12 non-standard apply (the mixed-precision workload's order) in FP64, every leaf."""
    _say("case: coulomb k=12 reduced (1 Gaussian, thresh 1e-6)")
    c, a, x = W.unit_charge_gaussians(2, 7, 1, 3.0, 3.0)
    ctx = M.Context(0, W.CELL)
    f = ctx.project(c, a, x, 12, 1e-6)
    op = ctx.op_coulomb(12, 1e-5, 1e-8)
    g = ctx.apply(op, f, tau_drop=1e-10)
    fo = project_adaptive(GaussianSum(c, a, x), 12, 1e-6, W.CELL, 2, 20)
    assert set(_as_dict(f)) == set(fo.leaves)
    cc, tt = coulomb_fit(1e-5, 1e-8, cell_r_hi(*W.CELL))
    ref, st = apply_nonstandard(fo, SeparatedOperator(cc, tt), 1e-10)
    got = _as_dict(g)
    assert set(got) == set(ref.leaves)
    assert ctx.last_stats()["triples"] == st["triples"]
    err = _rel_l2(got, ref.leaves, ref.leaves)
    _say("coulomb k12 reduced rel L2 vs oracle", err, "triples", st["triples"])
    assert err <= TOL


def test_coulomb_k14_reduced_full_parity(M):
    """k=14 non-standard apply (the order of the large batched workload) in FP64, every
    leaf: the source block is streamed through LDS in z-quad slabs."""
    _say("case: coulomb k=14 reduced (2 Gaussians, thresh 1e-5)")
    c, a, x = W.unit_charge_gaussians(4, 3, 2, 1.0, 30.0)
    ctx = M.Context(0, W.CELL)
    f = ctx.project(c, a, x, 14, 1e-5)
    op = ctx.op_coulomb(14, 1e-5, 1e-8)
    g = ctx.apply(op, f, tau_drop=1e-9)
    fo = project_adaptive(GaussianSum(c, a, x), 14, 1e-5, W.CELL, 2, 20)
    assert set(_as_dict(f)) == set(fo.leaves)
    cc, tt = coulomb_fit(1e-5, 1e-8, cell_r_hi(*W.CELL))
    ref, st = apply_nonstandard(fo, SeparatedOperator(cc, tt), 1e-9)
    got = _as_dict(g)
    assert set(got) == set(ref.leaves)
    assert ctx.last_stats()["triples"] == st["triples"]
    err = _rel_l2(got, ref.leaves, ref.leaves)
    _say("coulomb k14 reduced rel L2 vs oracle", err, "triples", st["triples"])
    assert err <= TOL


@pytest.mark.parametrize("k,thresh", [(3, 1e-3), (5, 1e-4), (7, 1e-5), (9, 1e-6)])
def test_small_and_odd_orders_full_parity(M, k, thresh):
    """Non-standard Coulomb apply at orders without a matrix-core kernel (the vector
    transform, the separate level-n subtraction and the sum-down at odd and small k): input
    tree, kept triples, output tree and every output leaf against the oracle."""
    _say("case: coulomb k=%d, thresh %g, 2 Gaussians" % (k, thresh))
    cell = (-6.0, 6.0)
    gs = ([1.0, 0.5], [1.0, 4.0], [[0, 0, 0], [0.5, -0.25, 0.3]])
    ctx = M.Context(0, cell)
    g = ctx.project(*gs, k, thresh)
    go = project_adaptive(GaussianSum(*gs), k, thresh, cell, 2, 20)
    assert set(_as_dict(g)) == set(go.leaves)
    c, t = coulomb_fit(1e-4, 1e-6, cell_r_hi(*cell))
    op = ctx.op_coulomb(k, 1e-4, 1e-6)
    vg = ctx.apply(op, g, tau_drop=1e-2 * thresh)
    ref, st = apply_nonstandard(go, SeparatedOperator(c, t), 1e-2 * thresh)
    got = _as_dict(vg)
    assert set(got) == set(ref.leaves)
    assert ctx.last_stats()["triples"] == st["triples"]
    err = _rel_l2(got, ref.leaves, ref.leaves)
    _say("k=%d: %d output leaves, %d triples, rel L2 vs oracle %.3e" % (k, len(got), st["triples"], err))
    assert err <= TOL


def test_degenerate_inputs(M):
    """Edge cases of the non-standard apply: an input whose root is a leaf is rejected; with
    every triple screened out the result is the zero function on the root box (as in the
    oracle); a single refined root (level-1 leaves only) is applied exactly."""
    _say("case: degenerate inputs")
    ctx = M.Context(0, W.CELL)
    c, a, x = W.unit_charge_gaussians(1, 3, 1, 2.0, 2.0)
    op = ctx.op_coulomb(6, 1e-4, 1e-6)
    root_leaf = ctx.project(c, a, x, 6, 1e3, initial_level=0)
    assert root_leaf.info()["leaves"] == 1
    with pytest.raises(M.MraError) as e:
        ctx.apply(op, root_leaf, tau_drop=1e-8)
    assert e.value.code == -1
    f = ctx.project(c, a, x, 6, 1e-3)
    g = ctx.apply(op, f, tau_drop=1e30)
    assert ctx.last_stats()["triples"] == 0
    got = _as_dict(g)
    assert list(got) == [(0, 0, 0, 0)] and not np.any(got[(0, 0, 0, 0)])
    fo = project_adaptive(GaussianSum(c, a, x), 6, 1e-3, W.CELL, 2, 20)
    cc, tt = coulomb_fit(1e-4, 1e-6, cell_r_hi(*W.CELL))
    ref, st = apply_nonstandard(fo, SeparatedOperator(cc, tt), 1e30)
    assert st["triples"] == 0 and set(ref.leaves) == {(0, 0, 0, 0)}
    # refined root only: every box at level 1 is a leaf
    f1 = ctx.project(c, a, x, 6, 1e3, initial_level=1, max_level=1)
    g1 = ctx.apply(op, f1, tau_drop=0.0)
    fo1 = project_adaptive(GaussianSum(c, a, x), 6, 1e3, W.CELL, 1, 1)
    ref1, st1 = apply_nonstandard(fo1, SeparatedOperator(cc, tt), 0.0)
    got1 = _as_dict(g1)
    assert set(got1) == set(ref1.leaves) and ctx.last_stats()["triples"] == st1["triples"]
    err = _rel_l2(got1, ref1.leaves, ref1.leaves)
    _say("refined root only: rel L2 vs oracle", err, "triples", st1["triples"])
    assert err <= TOL


def test_allocator_null_gives_nomem_without_leak(M):
    """An allocator that returns NULL after a given number of allocations: every call ends
    with MRA_OK or MRA_E_NOMEM (-2), never anything else, and once the handles and the
    context are freed every allocation has been returned."""
    import ctypes
    import torch
    _say("case: allocator returning NULL")
    lib = M.load()
    stream = torch.cuda.current_stream(0).cuda_stream
    c, a, x = W.unit_charge_gaussians(1, 3, 2, 2.0, 20.0)
    garr, ng = M._binding._gaussians(c, a, x)
    outcomes = []
    for budget in (0, 1, 2, 3, 5, 8, 13, 21, 34, 1000):
        live, left = {}, [budget]

        def _alloc(nbytes, user):
            if left[0] <= 0:
                return None
            left[0] -= 1
            p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream)
            live[p] = int(nbytes)
            return p

        def _free(ptr, user):
            assert ptr in live
            del live[ptr]
            torch.cuda.caching_allocator_delete(ptr)

        af, ff = M._binding.ALLOC_FN(_alloc), M._binding.FREE_FN(_free)
        h = ctypes.c_void_p()
        assert lib.mra_ctx_create(0, ctypes.c_void_p(stream), af, ff, None, W.CELL[0], W.CELL[1],
                                  ctypes.byref(h)) == 0
        steps = []
        fh, oh, gh = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        p = M._binding.ProjectParams(8, 1e-4, 2, 20)
        rc = lib.mra_project(h, garr, ng, ctypes.byref(p), ctypes.byref(fh))
        steps.append(rc)
        if rc == 0:
            rc = lib.mra_op_coulomb(h, 8, 1e-4, 1e-6, ctypes.byref(oh))
            steps.append(rc)
        if rc == 0:
            ap = M._binding.ApplyParams(0, 1, 1e-8, 0.0, 1)
            rc = lib.mra_apply(h, oh, fh, ctypes.byref(ap), ctypes.byref(gh))
            steps.append(rc)
        if rc == 0:
            v = ctypes.c_double()
            rc = lib.mra_norm2(h, gh, ctypes.byref(v))
            steps.append(rc)
        assert all(s in (0, -2) for s in steps), steps
        if steps[-1] == -2:
            assert "allocation" in lib.mra_last_error(h).decode()
        for hh, fn in ((gh, lib.mra_func_free), (fh, lib.mra_func_free), (oh, lib.mra_op_free)):
            if hh.value:
                fn(hh)
        lib.mra_ctx_free(h)
        torch.cuda.synchronize()
        outcomes.append((budget, steps[-1], len(steps)))
        assert live == {}, "budget %d: %d allocations not returned" % (budget, len(live))
    _say("allocator budget -> (last status, calls made):", outcomes)
    assert outcomes[0][1] == -2 and outcomes[-1][1] == 0


def test_autotuned_schedule(M, tmp_path):
    """The autotuner times the batched apply under each candidate schedule and keeps the
    fastest; its JSON cache is reused on the next call.  Results under different schedules
    agree up to the summation order of split lists, and the tuned one matches the oracle."""
    _say("case: autotuner, 4 batched Helmholtz functions")
    ctx = M.Context(0, W.CELL)
    funcs, ops, params = [], [], []
    for i in range(4):
        c, a, x, mu = W.bsh_inputs(i)
        funcs.append(ctx.project(c, a, x, 10, 1e-4))
        ops.append(ctx.op_bsh(10, mu, 1e-5, 1e-8))
        params.append((c, a, x, mu))
    cache = str(tmp_path / "tune.json")
    best, times = ctx.autotune_batch(ops, funcs, tau_drop=1e-8, cache_path=cache)
    _say("tuned schedule", best, "times ms", [round(t, 2) for t in times])
    assert best["sub_batches"] in (1, 2, 4) and best["split_div"] in (256, 512, 1024)
    assert np.all(times > 0) and ctx.schedule() == best
    ctx2 = M.Context(0, W.CELL)
    best2, times2 = ctx2.autotune_batch(ops, funcs, tau_drop=1e-8, cache_path=cache)
    assert best2 == best and np.all(times2 == -1.0)
    outs = [_as_dict(g) for g in ctx.apply_batch(ops, funcs, tau_drop=1e-8)]
    ctx.set_schedule(1, 256)
    other = [_as_dict(g) for g in ctx.apply_batch(ops, funcs, tau_drop=1e-8)]
    for a_, b_ in zip(outs, other):
        assert set(a_) == set(b_)
        assert _rel_l2(a_, b_, b_) <= 1e-14
    c, a, x, mu = params[3]
    fo = project_adaptive(GaussianSum(c, a, x), 10, 1e-4, W.CELL, 2, 20)
    cc, tt = bsh_fit(mu, 1e-5, 1e-8, cell_r_hi(*W.CELL))
    ref, _ = apply_nonstandard(fo, SeparatedOperator(cc, tt), 1e-8)
    assert set(outs[3]) == set(ref.leaves)
    assert _rel_l2(outs[3], ref.leaves, ref.leaves) <= TOL
    with pytest.raises(M.MraError):
        ctx.set_schedule(-1, 512)
