"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws parameters (Gaussian exponents, centres, charges, kernel
parameters) from seeded generators and names the workload sizes.  It holds none of the
method's arithmetic: no basis, projection, fit, block or apply code.

Recipe (the paper uses no dataset; everything is synthetic):
  * RNG numpy.random.default_rng(1000 + 100 * workload_id + function_index);
  * Gaussians are unit charges (a/pi)^{3/2} exp(-a |x - X|^2) with a log-uniform in the
    stated range and X uniform in [-5, 5]^3, on the cell [-10, 10]^3;
  * bound-state Helmholtz parameters mu are log-uniform in [0.5, 5].
"""
import math

import numpy as np

CELL = (-10.0, 10.0)


def rng(workload_id, index=0):
    return np.random.default_rng(1000 + 100 * workload_id + index)


def unit_charge_gaussians(workload_id, index, count, a_lo, a_hi, box=5.0):
    """(coeffs, expnts, centers) of `count` unit-charge Gaussians."""
    g = rng(workload_id, index)
    expnts = np.exp(g.uniform(math.log(a_lo), math.log(a_hi), size=count))
    centers = g.uniform(-box, box, size=(count, 3))
    coeffs = (expnts / math.pi) ** 1.5
    return coeffs, expnts, centers


def bsh_mu(workload_id, index, lo=0.5, hi=5.0):
    g = rng(workload_id, 10_000 + index)
    return float(math.exp(g.uniform(math.log(lo), math.log(hi))))


# Workload definitions.  Sizes are those of the stated configurations; `reduced` variants
# keep the structure at sizes the FP64 oracle finishes in seconds.
WORKLOADS = {
    # plain FP64 single-term standard-form apply, k=8, uniform level 4 (4096 boxes)
    "gauss_std_k8": dict(id=0, k=8, level=4, f_coeff=(10.0 / math.pi) ** 1.5, f_expnt=10.0,
                         op_c=[1.0], op_t=[2.0], disp_radius=1),
    # plain FP64 Coulomb non-standard apply, k=10, thresh 1e-6, 4 Gaussians a in [1, 1e3]
    "coulomb_k10": dict(id=1, k=10, thresh=1e-6, n_gauss=4, a_lo=1.0, a_hi=1e3,
                        r_lo=1e-5, eps=1e-8, tau_rel=1e-4, initial_level=2),
    # mixed precision Coulomb, k=12, thresh 1e-8
    "coulomb_k12_mixed": dict(id=2, k=12, thresh=1e-8, n_gauss=4, a_lo=1.0, a_hi=1e3,
                              r_lo=1e-5, eps=1e-8, tau_rel=1e-4, tier_rel=1e-3,
                              initial_level=2),
    # batched bound-state Helmholtz, 64 functions of 1-8 Gaussians, k=10
    "bsh_batch_k10": dict(id=3, k=10, thresh=1e-6, n_funcs=64, n_gauss_lo=1, n_gauss_hi=8,
                          a_lo=1.0, a_hi=1e3, r_lo=1e-5, eps=1e-8, tau_rel=1e-4,
                          initial_level=2),
    # large batched mixed, 16 functions x 32 Gaussians, a in [1, 1e4], k=14, thresh 1e-8
    "coulomb_batch_k14": dict(id=4, k=14, thresh=1e-8, n_funcs=16, n_gauss=32, a_lo=1.0,
                              a_hi=1e4, r_lo=1e-5, eps=1e-8, tau_rel=1e-4, tier_rel=1e-3,
                              initial_level=2),
}


def coulomb_inputs(name, index=0):
    """Gaussians of function `index` of a Coulomb workload."""
    w = WORKLOADS[name]
    return unit_charge_gaussians(w["id"], index, w["n_gauss"], w["a_lo"], w["a_hi"])


def bsh_inputs(index):
    """(coeffs, expnts, centers, mu) of function `index` of the batched BSH workload."""
    w = WORKLOADS["bsh_batch_k10"]
    g = rng(w["id"], 20_000 + index)
    count = int(g.integers(w["n_gauss_lo"], w["n_gauss_hi"] + 1))
    c, a, x = unit_charge_gaussians(w["id"], index, count, w["a_lo"], w["a_hi"])
    return c, a, x, bsh_mu(w["id"], index)
