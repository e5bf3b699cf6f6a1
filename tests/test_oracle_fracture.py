"""Pins of the oracle's fracture driver (Sec. 2).

* the restricted solve equals the dense solve of the intact submatrix
  (Cholesky of A_II, A assembled entrywise), with zeros on broken fibres;
* periodic grid, uniform thresholds, nothing broken: all forces equal the
  closed form 1 / (1/k + ghat(0, 0)) (translation invariance), so the first
  fibre to break is index 0 (tie rule) at D = t (1/k + ghat(0, 0));
* the total force at unit displacement never increases as fibres break (the
  restricted energy maximum is taken over a shrinking subspace);
* a whole sequence on a 4 x 4 grid equals brute force (dense restricted
  solves and argmax at every step).
"""

import numpy as np
import pytest

from workloads import spectrum, fracture_instance
from oracle import kernel_table, assemble_dense, restricted_solve, fracture_sequence


def _dense_restricted(ghat, k, mask, padded):
    M = ghat.shape[0]
    L = M // 2 if padded else M
    A = assemble_dense(kernel_table(ghat), np.full((L, L), 1.0 / k), padded)
    I = np.flatnonzero(mask.ravel() > 0)
    f = np.zeros(L * L)
    f[I] = np.linalg.solve(A[np.ix_(I, I)], np.ones(len(I)))
    return f.reshape(L, L)


@pytest.mark.parametrize("padded", [0, 1])
def test_restricted_solve_dense(padded):
    L = 8
    M = 2 * L if padded else L
    gh = spectrum(M, 1e-2)
    rng = np.random.default_rng([80, padded])
    mask = (rng.random((L, L)) > 0.3).astype(float)
    f, _ = restricted_solve(gh, 2.0, mask, padded)
    ref = _dense_restricted(gh, 2.0, mask, padded)
    assert np.max(np.abs(f - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.all(f[mask == 0] == 0.0)


def test_uniform_periodic_first_step():
    L, k, tval = 16, 2.0, 0.7
    gh = spectrum(L, 1e-2)
    t = np.full((L, L), tval)
    f, _ = restricted_solve(gh, k, np.ones((L, L)), 0)
    np.testing.assert_allclose(f, 1.0 / (1.0 / k + gh[0, 0]), rtol=1e-13)
    broken, dbreak, _, _ = fracture_sequence(gh, k, t, 1, 0)
    assert broken[0] == 0
    assert dbreak[0] == pytest.approx(tval * (1.0 / k + gh[0, 0]), rel=1e-12)


def test_total_force_decreases():
    inst = fracture_instance(0, L=16)
    gh = spectrum(32, 1e-3)
    L = inst["L"]
    mask = np.ones((L, L))
    prev = np.inf
    broken, _, _, _ = fracture_sequence(gh, inst["k"], inst["t"], 12, 1)
    for i in broken:
        f, _ = restricted_solve(gh, inst["k"], mask, 1)
        assert f.sum() <= prev * (1 + 1e-13)
        prev = f.sum()
        mask.ravel()[i] = 0.0


def test_sequence_bruteforce():
    L = 4
    gh = spectrum(2 * L, 1e-2)
    inst = fracture_instance(1, L=L)
    broken, dbreak, f, _ = fracture_sequence(gh, inst["k"], inst["t"], 10, 1)
    mask = np.ones((L, L))
    for s in range(10):
        fd = _dense_restricted(gh, inst["k"], mask, 1)
        rho = np.where(mask > 0, fd / inst["t"], -np.inf).ravel()
        i = int(np.argmax(rho))
        assert broken[s] == i
        assert dbreak[s] == pytest.approx(1.0 / rho[i], rel=1e-12)
        mask.ravel()[i] = 0.0
    assert np.max(np.abs(f - _dense_restricted(gh, inst["k"], np.where(np.isin(np.arange(L * L), broken[:-1]).reshape(L, L), 0.0, 1.0), 1))) <= 1e-12
