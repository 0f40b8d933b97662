"""ctypes binding of libmra (argument marshalling only).

Every computation happens inside libmra.so (host planner in C++, kernels in HIP).  PyTorch
is used for two things only: the caching allocator that backs the library's device memory,
and the current HIP stream on which the library issues its work.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmra.so")

MRA_OK = 0
ERRORS = {-1: "MRA_E_INVALID", -2: "MRA_E_NOMEM", -3: "MRA_E_DEVICE", -4: "MRA_E_UNSUPPORTED",
          -5: "MRA_E_MISMATCH"}
FORM_NONSTANDARD = 0
FORM_STANDARD = 1
REPR_SCALING = 0
REPR_WAVELET = 1

# every symbol declared in include/mra.h
EXPORTED = [
    "mra_ctx_create", "mra_ctx_free", "mra_last_error", "mra_project", "mra_func_info",
    "mra_func_export", "mra_func_free", "mra_op_coulomb", "mra_op_bsh", "mra_op_gaussians",
    "mra_op_terms", "mra_op_free", "mra_apply", "mra_apply_batch", "mra_norm2", "mra_trace",
    "mra_inner", "mra_distance", "mra_norm2_noalloc", "mra_set_schedule", "mra_get_schedule",
    "mra_autotune_batch", "mra_func_repr", "mra_compress", "mra_reconstruct", "mra_truncate",
    "mra_func_export_nodes",
    "mra_last_stats", "mra_host_fit", "mra_host_block", "mra_host_filters",
    "mra_host_spectral_norm", "mra_host_project",
]


class MraError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "MRA_E_?"), code, msg))


class Gaussian(ctypes.Structure):
    _fields_ = [("coeff", ctypes.c_double), ("expnt", ctypes.c_double),
                ("center", ctypes.c_double * 3)]


class ProjectParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("thresh", ctypes.c_double),
                ("initial_level", ctypes.c_int), ("max_level", ctypes.c_int)]


LOW_BF16 = 1


class ApplyParams(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("disp_radius", ctypes.c_int),
                ("tau_drop", ctypes.c_double), ("tau_tier", ctypes.c_double),
                ("low_precision", ctypes.c_int)]


class Schedule(ctypes.Structure):
    _fields_ = [("sub_batches", ctypes.c_int), ("split_div", ctypes.c_int)]


class ApplyStats(ctypes.Structure):
    _fields_ = [("triples", ctypes.c_int64), ("targets", ctypes.c_int64),
                ("in_leaves", ctypes.c_int64), ("out_nodes", ctypes.c_int64),
                ("out_leaves", ctypes.c_int64), ("useful_flops", ctypes.c_double),
                ("ms_filter", ctypes.c_double), ("ms_plan", ctypes.c_double),
                ("ms_apply", ctypes.c_double), ("ms_sumdown", ctypes.c_double),
                ("ms_main_kernel", ctypes.c_double), ("triples_low", ctypes.c_int64),
                ("flops_low", ctypes.c_double), ("eta_low", ctypes.c_double),
                ("ms_low_kernel", ctypes.c_double), ("flops_kernel", ctypes.c_double),
                ("launches_main", ctypes.c_int64), ("launches_low", ctypes.c_int64)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load():
    """Load libmra.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmra.so is not built (run paper_1507_01888_amd.build.build())")
    # torch is imported first so that its HIP runtime is the one in the process: libmra's
    # libamdhip64.so.7 dependency then resolves to that same runtime, and streams and device
    # memory handed over by torch are valid inside the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i64p = P(ctypes.c_int64)
    dp = P(ctypes.c_double)
    lib.mra_ctx_create.argtypes = [ctypes.c_int, vp, ALLOC_FN, FREE_FN, vp, ctypes.c_double,
                                   ctypes.c_double, P(vp)]
    lib.mra_ctx_free.argtypes = [vp]
    lib.mra_last_error.argtypes = [vp]
    lib.mra_last_error.restype = ctypes.c_char_p
    lib.mra_project.argtypes = [vp, P(Gaussian), ctypes.c_int, P(ProjectParams), P(vp)]
    lib.mra_func_info.argtypes = [vp, P(ctypes.c_int), i64p, i64p, P(ctypes.c_int)]
    lib.mra_func_export.argtypes = [vp, vp, ctypes.c_int64, P(ctypes.c_uint64), dp, i64p]
    lib.mra_func_free.argtypes = [vp]
    lib.mra_op_coulomb.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, P(vp)]
    lib.mra_op_bsh.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, P(vp)]
    lib.mra_op_gaussians.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, dp, P(vp)]
    lib.mra_op_terms.argtypes = [vp, P(ctypes.c_int), dp, dp]
    lib.mra_op_free.argtypes = [vp]
    lib.mra_apply.argtypes = [vp, vp, vp, P(ApplyParams), P(vp)]
    lib.mra_apply_batch.argtypes = [vp, ctypes.c_int, P(vp), P(vp), P(ApplyParams), P(vp)]
    lib.mra_norm2.argtypes = [vp, vp, dp]
    lib.mra_trace.argtypes = [vp, vp, dp]
    lib.mra_inner.argtypes = [vp, vp, vp, dp]
    lib.mra_distance.argtypes = [vp, vp, vp, dp]
    lib.mra_norm2_noalloc.argtypes = [vp, vp, dp]
    lib.mra_set_schedule.argtypes = [vp, P(Schedule)]
    lib.mra_get_schedule.argtypes = [vp, P(Schedule)]
    lib.mra_autotune_batch.argtypes = [vp, ctypes.c_int, P(vp), P(vp), P(ApplyParams),
                                       ctypes.c_char_p, P(Schedule), dp]
    lib.mra_func_repr.argtypes = [vp, P(ctypes.c_int)]
    lib.mra_compress.argtypes = [vp, vp, P(vp)]
    lib.mra_reconstruct.argtypes = [vp, vp, P(vp)]
    lib.mra_truncate.argtypes = [vp, vp, ctypes.c_double, P(vp), dp]
    lib.mra_func_export_nodes.argtypes = [vp, vp, ctypes.c_int64, P(ctypes.c_uint64), dp, i64p]
    lib.mra_last_stats.argtypes = [vp, P(ApplyStats)]
    lib.mra_host_fit.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int, dp, dp, P(ctypes.c_int)]
    lib.mra_host_block.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, dp]
    lib.mra_host_filters.argtypes = [ctypes.c_int, dp, dp]
    lib.mra_host_spectral_norm.argtypes = [ctypes.c_int, dp, dp]
    lib.mra_host_project.argtypes = [ctypes.c_double, ctypes.c_double, P(Gaussian), ctypes.c_int,
                                     P(ProjectParams), ctypes.c_int64, P(ctypes.c_uint64), dp, i64p]
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _gaussians(coeffs, expnts, centers):
    coeffs = np.asarray(coeffs, dtype=np.float64).ravel()
    expnts = np.asarray(expnts, dtype=np.float64).ravel()
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, 3)
    n = len(coeffs)
    arr = (Gaussian * n)()
    for i in range(n):
        arr[i].coeff = coeffs[i]
        arr[i].expnt = expnts[i]
        for d in range(3):
            arr[i].center[d] = centers[i, d]
    return arr, n


# ------------------------------------------------------------------------ host-only helpers

def host_fit(kind, lo, eps, r_hi, mu=0.0):
    """Gaussian-sum fit computed by the library's host code (kind 'coulomb' or 'bsh')."""
    lib = load()
    m = ctypes.c_int()
    code = 0 if kind == "coulomb" else 1
    rc = lib.mra_host_fit(code, mu, lo, eps, r_hi, 0, None, None, ctypes.byref(m))
    if rc != MRA_OK:
        raise MraError(rc, "host_fit")
    c = np.zeros(m.value)
    t = np.zeros(m.value)
    rc = lib.mra_host_fit(code, mu, lo, eps, r_hi, m.value, _dptr(c), _dptr(t), ctypes.byref(m))
    if rc != MRA_OK:
        raise MraError(rc, "host_fit")
    return c, t


def host_block(k, h, delta, texp):
    out = np.zeros((k, k))
    rc = load().mra_host_block(k, h, delta, texp, _dptr(out))
    if rc != MRA_OK:
        raise MraError(rc, "host_block")
    return out


def host_filters(k):
    h0 = np.zeros((k, k))
    h1 = np.zeros((k, k))
    rc = load().mra_host_filters(k, _dptr(h0), _dptr(h1))
    if rc != MRA_OK:
        raise MraError(rc, "host_filters")
    return h0, h1


def host_spectral_norm(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = ctypes.c_double()
    rc = load().mra_host_spectral_norm(a.shape[0], _dptr(a), ctypes.byref(out))
    if rc != MRA_OK:
        raise MraError(rc, "host_spectral_norm")
    return out.value


def host_project(cell, coeffs, expnts, centers, k, thresh, initial_level=2, max_level=20):
    """Adaptive projection by the library's host code: (keys, coeffs (n, k, k, k))."""
    lib = load()
    arr, ng = _gaussians(coeffs, expnts, centers)
    p = ProjectParams(k, thresh, initial_level, max_level)
    n = ctypes.c_int64()
    rc = lib.mra_host_project(cell[0], cell[1], arr, ng, ctypes.byref(p), 0, None, None,
                              ctypes.byref(n))
    if rc != MRA_OK:
        raise MraError(rc, "host_project")
    keys = np.zeros(n.value, dtype=np.uint64)
    co = np.zeros((n.value, k, k, k))
    rc = lib.mra_host_project(cell[0], cell[1], arr, ng, ctypes.byref(p), n.value,
                              keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _dptr(co),
                              ctypes.byref(n))
    if rc != MRA_OK:
        raise MraError(rc, "host_project")
    return keys, co


# ------------------------------------------------------------------------ device objects

class Context:
    """A libmra context on one HIP device, backed by torch's caching allocator and stream."""

    def __init__(self, device=0, cell=(-10.0, 10.0), use_torch_allocator=True, on_alloc=None):
        """on_alloc: optional callable(nbytes) told of every device allocation the library
        asks for (diagnostics; needs use_torch_allocator)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libmra needs a HIP device")
        self._lib = load()
        self.device = device
        self.cell = (float(cell[0]), float(cell[1]))
        torch.cuda.set_device(device)
        stream = torch.cuda.current_stream(device)
        self._stream = stream
        if use_torch_allocator:
            dev = device
            sptr = stream.cuda_stream

            def _alloc(nbytes, user):
                if on_alloc is not None:
                    on_alloc(int(nbytes))
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, sptr)
                except Exception:  # noqa: BLE001 - reported to the library as NULL
                    return None

            delete = torch.cuda.caching_allocator_delete

            def _free(ptr, user):
                try:
                    delete(ptr)
                except Exception:  # noqa: BLE001 - torch already torn down at exit
                    pass

            self._alloc = ALLOC_FN(_alloc)
            self._free = FREE_FN(_free)
        else:
            self._alloc = ALLOC_FN()
            self._free = FREE_FN()
        h = ctypes.c_void_p()
        rc = self._lib.mra_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), self._alloc,
                                      self._free, None, self.cell[0], self.cell[1], ctypes.byref(h))
        if rc != MRA_OK:
            msg = self._lib.mra_last_error(None)
            raise MraError(rc, "mra_ctx_create: %s" % (msg.decode() if msg else ""))
        self.h = h

    def _check(self, rc, what):
        if rc != MRA_OK:
            msg = self._lib.mra_last_error(self.h)
            raise MraError(rc, "%s: %s" % (what, msg.decode() if msg else ""))

    def close(self):
        if getattr(self, "h", None):
            self._lib.mra_ctx_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    # -- functions
    def project(self, coeffs, expnts, centers, k, thresh, initial_level=2, max_level=20):
        arr, ng = _gaussians(coeffs, expnts, centers)
        p = ProjectParams(k, thresh, initial_level, max_level)
        h = ctypes.c_void_p()
        self._check(self._lib.mra_project(self.h, arr, ng, ctypes.byref(p), ctypes.byref(h)),
                    "mra_project")
        return Function(self, h)

    # -- operators
    def op_coulomb(self, k, lo, eps):
        h = ctypes.c_void_p()
        self._check(self._lib.mra_op_coulomb(self.h, k, lo, eps, ctypes.byref(h)), "mra_op_coulomb")
        return Operator(self, h)

    def op_bsh(self, k, mu, lo, eps):
        h = ctypes.c_void_p()
        self._check(self._lib.mra_op_bsh(self.h, k, mu, lo, eps, ctypes.byref(h)), "mra_op_bsh")
        return Operator(self, h)

    def op_gaussians(self, k, c, t):
        c = np.ascontiguousarray(c, dtype=np.float64)
        t = np.ascontiguousarray(t, dtype=np.float64)
        h = ctypes.c_void_p()
        self._check(self._lib.mra_op_gaussians(self.h, k, len(c), _dptr(c), _dptr(t),
                                               ctypes.byref(h)), "mra_op_gaussians")
        return Operator(self, h)

    # -- apply and reductions
    def apply(self, op, f, form="nonstandard", tau_drop=0.0, disp_radius=1, tau_tier=0.0):
        """op(f).  tau_tier > 0: triples at levels n > 0 with eta < tau_tier run in BF16."""
        p = ApplyParams(FORM_STANDARD if form == "standard" else FORM_NONSTANDARD,
                        disp_radius, tau_drop, tau_tier, LOW_BF16)
        h = ctypes.c_void_p()
        self._check(self._lib.mra_apply(self.h, op.h, f.h, ctypes.byref(p), ctypes.byref(h)),
                    "mra_apply")
        return Function(self, h)

    def apply_batch(self, ops, funcs, tau_drop=0.0, tau_tier=0.0):
        """[op_i(f_i)] in one batched pass (non-standard form)."""
        n = len(funcs)
        if len(ops) != n:
            raise ValueError("need one operator per function")
        oarr = (ctypes.c_void_p * n)(*[o.h.value for o in ops])
        farr = (ctypes.c_void_p * n)(*[f.h.value for f in funcs])
        outs = (ctypes.c_void_p * n)()
        p = ApplyParams(FORM_NONSTANDARD, 1, tau_drop, tau_tier, LOW_BF16)
        self._check(self._lib.mra_apply_batch(self.h, n, oarr, farr, ctypes.byref(p), outs),
                    "mra_apply_batch")
        return [Function(self, ctypes.c_void_p(outs[i])) for i in range(n)]

    def set_schedule(self, sub_batches=0, split_div=512):
        sch = Schedule(sub_batches, split_div)
        self._check(self._lib.mra_set_schedule(self.h, ctypes.byref(sch)), "mra_set_schedule")

    def schedule(self):
        sch = Schedule()
        self._check(self._lib.mra_get_schedule(self.h, ctypes.byref(sch)), "mra_get_schedule")
        return {"sub_batches": sch.sub_batches, "split_div": sch.split_div}

    def autotune_batch(self, ops, funcs, tau_drop=0.0, tau_tier=0.0, cache_path=None):
        """Times the batched apply under the library's candidate schedules and keeps the
        fastest (see mra_autotune_batch); returns (schedule dict, times in ms)."""
        n = len(funcs)
        oarr = (ctypes.c_void_p * n)(*[o.h.value for o in ops])
        farr = (ctypes.c_void_p * n)(*[f.h.value for f in funcs])
        p = ApplyParams(FORM_NONSTANDARD, 1, tau_drop, tau_tier, LOW_BF16)
        best = Schedule()
        times = np.zeros(9)
        path = cache_path.encode() if cache_path else None
        self._check(self._lib.mra_autotune_batch(self.h, n, oarr, farr, ctypes.byref(p), path,
                                                 ctypes.byref(best), _dptr(times)),
                    "mra_autotune_batch")
        return {"sub_batches": best.sub_batches, "split_div": best.split_div}, times

    def norm2(self, f):
        v = ctypes.c_double()
        self._check(self._lib.mra_norm2(self.h, f.h, ctypes.byref(v)), "mra_norm2")
        return v.value

    def norm2_noalloc(self, f):
        """norm2 through the entry point that allocates no device memory."""
        v = ctypes.c_double()
        self._check(self._lib.mra_norm2_noalloc(self.h, f.h, ctypes.byref(v)), "mra_norm2_noalloc")
        return v.value

    def trace(self, f):
        v = ctypes.c_double()
        self._check(self._lib.mra_trace(self.h, f.h, ctypes.byref(v)), "mra_trace")
        return v.value

    def inner(self, f, g):
        v = ctypes.c_double()
        self._check(self._lib.mra_inner(self.h, f.h, g.h, ctypes.byref(v)), "mra_inner")
        return v.value

    def distance(self, f, g):
        """||f - g||_2 of two functions on the same tree (computed on the device)."""
        v = ctypes.c_double()
        self._check(self._lib.mra_distance(self.h, f.h, g.h, ctypes.byref(v)), "mra_distance")
        return v.value

    def compress(self, f):
        """Wavelet form of f on the same tree (new function)."""
        h = ctypes.c_void_p()
        self._check(self._lib.mra_compress(self.h, f.h, ctypes.byref(h)), "mra_compress")
        return Function(self, h)

    def reconstruct(self, c):
        """Scaling form of a function in wavelet form (new function)."""
        h = ctypes.c_void_p()
        self._check(self._lib.mra_reconstruct(self.h, c.h, ctypes.byref(h)), "mra_reconstruct")
        return Function(self, h)

    def truncate(self, f, tol):
        """(truncated function, sum of the squared norms of the dropped wavelet parts)."""
        h = ctypes.c_void_p()
        rem = ctypes.c_double()
        self._check(self._lib.mra_truncate(self.h, f.h, tol, ctypes.byref(h), ctypes.byref(rem)),
                    "mra_truncate")
        return Function(self, h), rem.value

    def last_stats(self):
        s = ApplyStats()
        self._check(self._lib.mra_last_stats(self.h, ctypes.byref(s)), "mra_last_stats")
        return {name: getattr(s, name) for name, _ in ApplyStats._fields_}


class Function:
    def __init__(self, ctx, h):
        self.ctx = ctx
        self.h = h

    def info(self):
        k = ctypes.c_int()
        nodes = ctypes.c_int64()
        leaves = ctypes.c_int64()
        ml = ctypes.c_int()
        self.ctx._check(self.ctx._lib.mra_func_info(self.h, ctypes.byref(k), ctypes.byref(nodes),
                                                    ctypes.byref(leaves), ctypes.byref(ml)),
                        "mra_func_info")
        return {"k": k.value, "nodes": nodes.value, "leaves": leaves.value, "max_level": ml.value}

    def export(self):
        """(keys uint64 level-prefixed Morton codes, coeffs (nleaves, k, k, k))."""
        inf = self.info()
        n, k = inf["leaves"], inf["k"]
        keys = np.zeros(n, dtype=np.uint64)
        co = np.zeros((n, k, k, k))
        cnt = ctypes.c_int64()
        self.ctx._check(self.ctx._lib.mra_func_export(
            self.ctx.h, self.h, n, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
            _dptr(co), ctypes.byref(cnt)), "mra_func_export")
        return keys, co

    def repr(self):
        """REPR_SCALING or REPR_WAVELET."""
        r = ctypes.c_int()
        self.ctx._check(self.ctx._lib.mra_func_repr(self.h, ctypes.byref(r)), "mra_func_repr")
        return r.value

    def export_nodes(self):
        """(keys of every node, level-major, coeffs (nnodes, k, k, k)): the slab of every node."""
        inf = self.info()
        n, k = inf["nodes"], inf["k"]
        keys = np.zeros(n, dtype=np.uint64)
        co = np.zeros((n, k, k, k))
        cnt = ctypes.c_int64()
        self.ctx._check(self.ctx._lib.mra_func_export_nodes(
            self.ctx.h, self.h, n, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
            _dptr(co), ctypes.byref(cnt)), "mra_func_export_nodes")
        return keys, co

    def free(self):
        if self.h:
            self.ctx._lib.mra_func_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:  # noqa: BLE001
            pass


class Operator:
    def __init__(self, ctx, h):
        self.ctx = ctx
        self.h = h

    def terms(self):
        m = ctypes.c_int()
        self.ctx._check(self.ctx._lib.mra_op_terms(self.h, ctypes.byref(m), None, None), "mra_op_terms")
        c = np.zeros(m.value)
        t = np.zeros(m.value)
        self.ctx._check(self.ctx._lib.mra_op_terms(self.h, ctypes.byref(m), _dptr(c), _dptr(t)),
                        "mra_op_terms")
        return c, t

    def free(self):
        if self.h:
            self.ctx._lib.mra_op_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:  # noqa: BLE001
            pass
