"""The seeded input recipes: shapes, determinism and the spectrum's
closed-form properties (real, even in each index, symmetric, max 1/sqrt(eps)
at the origin, min 1/sqrt(8+eps) at (M/2, M/2))."""

import numpy as np
import pytest

from workloads import (spectrum, c1_instance, c2_instance, c4_schedule,
                       c4_request, c5_sequence, padded_instance)


@pytest.mark.parametrize("M,eps", [(4, 1e-2), (64, 1e-2), (1024, 1e-3)])
def test_spectrum_properties(M, eps):
    gh = spectrum(M, eps)
    idx = (-np.arange(M)) % M
    assert np.array_equal(gh, gh[idx, :])
    assert np.array_equal(gh, gh[:, idx])
    assert np.array_equal(gh, gh.T)
    assert gh.max() == gh[0, 0] == pytest.approx(1 / np.sqrt(eps), rel=1e-15)
    assert gh.min() == gh[M // 2, M // 2] == pytest.approx(1 / np.sqrt(8 + eps), rel=1e-15)


def test_c1_deterministic():
    a, b = c1_instance(3), c1_instance(3)
    assert np.array_equal(a["d"], b["d"]) and np.array_equal(a["b"], b["b"])
    assert a["d"].shape == (64, 64) and a["M"] == 64 and a["padded"] == 0
    assert 0.5 <= a["d"].min() and a["d"].max() <= 1.5


def test_c2_zero_fraction():
    inst = c2_instance(0)
    frac = np.mean(inst["d"] == 0)
    assert 0.28 < frac < 0.32
    assert inst["M"] == 1024


def test_schedule():
    t, sizes = c4_schedule(2000)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 2000 - 0.5e-3) < 0.05e-3
    assert set(np.unique(sizes)) <= {128, 256, 512, 1024}
    r = c4_request(5, 256)
    assert r["d"].shape == (128, 128)


def test_c5():
    s = c5_sequence(0, L=32)
    assert np.all(s["d"] == 1) and np.all(s["b"] == 1) and s["t"].shape == (32, 32)


def test_normal_b():
    inst = padded_instance(16, [3, 0], eps=1e-4, normal_b=True)
    assert inst["b"].min() < 0
