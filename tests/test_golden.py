"""The golden fixtures (written by tests/golden/make_golden.py from the
oracle) still match the oracle's CG reference route, and the closed-form
condition-number bounds of the five workloads hold."""

import json
import os

import numpy as np
import pytest

from workloads import spectrum
from oracle import reference_solve, kappa_ub

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("name", ["periodic_L8", "padded_L8", "periodic_L4", "padded_L2"])
def test_golden_cases(name):
    with open(os.path.join(GOLD, name + ".json")) as f:
        g = json.load(f)
    L, M = g["L"], g["M"]
    d = np.array(g["d"]).reshape(L, L)
    b = np.array(g["b"]).reshape(L, L)
    xg = np.array(g["x"]).reshape(L, L)
    x, info = reference_solve(spectrum(M, g["eps"]), d, b, g["padded"])
    assert np.linalg.norm(x - xg) <= 2e-12 * np.linalg.norm(xg)


@pytest.mark.parametrize("M,eps,dmin,dmax,expect", [
    (64, 1e-2, 0.5, 1.5, 13.48),     # periodic L=64
    (1024, 1e-3, 0.0, 1.5, 93.7),    # padded L=512 with zeros in d
    (4096, 1e-4, 0.0, 1.5, 287.1),   # padded L=2048
])
def test_condition_bounds(M, eps, dmin, dmax, expect):
    # closed forms: max ghat = 1/sqrt(eps), min ghat = 1/sqrt(8 + eps)
    k = (dmax + 1 / np.sqrt(eps)) / (dmin + 1 / np.sqrt(8 + eps))
    assert k == pytest.approx(expect, rel=2e-3)
    gh = spectrum(min(M, 256), eps)
    d = np.array([[dmin, dmax]])
    assert kappa_ub(gh, d) == pytest.approx(k, rel=1e-12)
