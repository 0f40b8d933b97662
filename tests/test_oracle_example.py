"""The paper's worked example (Sec. 3.1): trace, 2-norm and Coulomb self-energy of
exp(-|x|^2) on [-6, 6]^3 with the default k = 6, thresh = 1e-4 and the Coulomb operator
built with lo = 1e-4, eps = 1e-6.  The printed values and the closed forms are in
tests/golden/paper_example.json; the paper reports agreement to six significant figures."""
import json
import math
import os

import pytest

from oracle.apply import SeparatedOperator, apply_nonstandard
from oracle.fit import coulomb_fit, cell_r_hi
from oracle.projection import GaussianSum, project_adaptive
from oracle.tree import inner

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")


@pytest.fixture(scope="module")
def example():
    cell = (-6.0, 6.0)
    g = project_adaptive(GaussianSum([1.0], [1.0], [[0.0, 0.0, 0.0]]), 6, 1e-4, cell, 2, 20)
    c, t = coulomb_fit(1e-4, 1e-6, cell_r_hi(*cell))
    vg, _ = apply_nonstandard(g, SeparatedOperator(c, t), 1e-4 * 1e-4)
    return g, vg


def test_printed_and_closed_form_values(example):
    g, vg = example
    gold = json.load(open(GOLDEN))
    closed = {"trace": math.pi ** 1.5, "norm2": (math.pi / 2) ** 0.75,
              "self_energy": math.pi ** 2.5 * math.sqrt(2.0)}
    got = {"trace": g.trace(), "norm2": g.norm2(), "self_energy": inner(g, vg)}
    for name in closed:
        # printed values are the closed forms rounded to the digits shown
        assert abs(gold["printed"][name] - closed[name]) < 1e-6 * closed[name]
        # six significant figures
        assert abs(got[name] - closed[name]) <= 1e-6 * closed[name], name
