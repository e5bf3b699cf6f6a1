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


@pytest.mark.parametrize("s", [0, 1, 2])
def test_large_samples_structure(s):
    """The stored samples of the L = 2048 oracle solutions sit at the seeded
    positions and carry a certified oracle solution."""
    import sys
    sys.path.insert(0, GOLD)
    from make_c3_samples import sample_positions
    with open(os.path.join(GOLD, f"padded_L2048_seed{s}_samples.json")) as f:
        g = json.load(f)
    assert g["pos"] == sample_positions(s, 2048 * 2048).tolist()
    assert len(g["x"]) == len(g["pos"]) and np.all(np.isfinite(g["x"]))
    assert g["bound"] < 1e-12 and g["xnorm"] > 0


@pytest.mark.slow
def test_large_samples_regenerate():
    """Re-solving the first L = 2048 instance reproduces its stored samples."""
    from workloads import c3_instance
    with open(os.path.join(GOLD, "padded_L2048_seed0_samples.json")) as f:
        g = json.load(f)
    inst = c3_instance(0)
    x, info = reference_solve(inst["ghat"], inst["d"], inst["b"], 1, route="fft")
    assert np.max(np.abs(x.ravel()[g["pos"]] - np.array(g["x"]))) <= 1e-12 * g["xnorm"]
