"""Pins of the oracle's preconditioned CG (Fourier-space circulant
preconditioner, an extension beyond the paper's unpreconditioned solver).

* the preconditioner equals crop(S^{-1} pad(r)) with S = mean(d) I + C_M built
  as an explicit dense matrix from the cosine-matrix kernel table (no FFT)
  and inverted densely, on padded and periodic grids; a planted mistake
  (no zero padding) fails this pin;
* periodic grid with uniform d: the preconditioner is exactly A^{-1}, so PCG
  converges in one iteration to the dense solution;
* symmetric positive definite on random vectors;
* PCG agrees with the dense Cholesky solution (zeros in d included);
* conjugacy in the preconditioned inner product: r_i . z_j ~ 0 for i != j;
* it converges in fewer iterations than CG on a padded grid.
"""

import numpy as np
import pytest

from workloads import spectrum, periodic_instance, padded_instance
from oracle import (kernel_table, assemble_dense, apply_direct, apply_fft, cg, pcg, circulant_precond,
                    solve_dense)


def _dense_precond(ghat, d, padded):
    M = ghat.shape[0]
    L = M // 2 if padded else M
    g = kernel_table(ghat)
    S = assemble_dense(g, np.full((M, M), float(np.mean(d))), 0)  # M^2 x M^2 circulant + dbar I
    Sinv = np.linalg.inv(S)
    i1, i2 = np.divmod(np.arange(L * L), L)
    sites = i1 * M + i2  # the L x L corner inside the M x M grid
    return Sinv[np.ix_(sites, sites)]


@pytest.mark.parametrize("L,padded", [(4, 1), (8, 1), (8, 0), (16, 0)])
def test_precond_equals_dense_inverse(L, padded):
    inst = padded_instance(L, [70, L], eps=1e-3) if padded else periodic_instance(L, [71, L], eps=1e-2)
    P = _dense_precond(inst["ghat"], inst["d"], padded)
    apply = circulant_precond(inst["ghat"], inst["d"], padded)
    rng = np.random.default_rng([72, L, padded])
    for _ in range(3):
        r = rng.standard_normal((L, L))
        z = apply(r)
        ref = (P @ r.ravel()).reshape(L, L)
        assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_precond_planted_mistake_fails():
    """Without the zero padding (circulant on the L grid) the pin above fails."""
    L = 8
    inst = padded_instance(L, [70, L], eps=1e-3)
    P = _dense_precond(inst["ghat"], inst["d"], 1)
    gh = inst["ghat"]
    dbar = float(np.mean(inst["d"]))
    r = np.random.default_rng(3).standard_normal((L, L))
    wrong = np.fft.ifft2(np.fft.fft2(r) / (dbar + gh[::2, ::2])).real
    ref = (P @ r.ravel()).reshape(L, L)
    assert np.max(np.abs(wrong - ref)) > 1e-3 * np.max(np.abs(ref))


def test_periodic_uniform_is_exact_inverse():
    L, eps = 32, 1e-2
    gh = spectrum(L, eps)
    d = np.full((L, L), 0.8)
    b = np.random.default_rng(5).uniform(0, 1, (L, L))
    g = kernel_table(gh)
    xs = solve_dense(g, d, b, 0)
    apply = circulant_precond(gh, d, 0)
    assert np.max(np.abs(apply(b) - xs)) <= 1e-12 * np.max(np.abs(xs))
    x, info = pcg(lambda v: apply_direct(g, d, v, 0), apply, b, tol=1e-13)
    assert info["iterations"] == 1
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("padded", [0, 1])
def test_precond_spd(padded):
    L = 16
    inst = padded_instance(L, [73, L], eps=1e-3) if padded else periodic_instance(L, [74, L], eps=1e-2)
    apply = circulant_precond(inst["ghat"], inst["d"], padded)
    rng = np.random.default_rng([75, padded])
    for _ in range(5):
        u, v = rng.standard_normal((2, L, L))
        assert abs(np.sum(apply(u) * v) - np.sum(u * apply(v))) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(v)
        assert np.sum(u * apply(u)) > 0.0


@pytest.mark.parametrize("L,padded", [(8, 1), (16, 1), (16, 0)])
def test_pcg_matches_cholesky(L, padded):
    inst = padded_instance(L, [76, L], eps=1e-3) if padded else periodic_instance(L, [77, L], eps=1e-2)
    g = kernel_table(inst["ghat"])
    xs = solve_dense(g, inst["d"], inst["b"], padded)
    apply = circulant_precond(inst["ghat"], inst["d"], padded)
    x, info = pcg(lambda v: apply_direct(g, inst["d"], v, padded), apply, inst["b"], tol=1e-14)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_pcg_conjugacy_and_speed():
    L = 64
    inst = padded_instance(L, [78, L], eps=1e-3)
    mv = lambda v: apply_fft(inst["ghat"], inst["d"], v, 1)  # noqa: E731
    apply = circulant_precond(inst["ghat"], inst["d"], 1)
    x, info = pcg(mv, apply, inst["b"], tol=1e-10, record=True)
    R, Z = info["residuals"], info["zs"]
    for i in range(min(6, len(R))):
        for j in range(i):
            rz = np.sum(R[i] * Z[j])
            scale = np.sqrt(np.sum(R[i] * Z[i]) * np.sum(R[j] * Z[j]))
            assert abs(rz) <= 1e-8 * scale
    _, cinfo = cg(mv, inst["b"], tol=1e-10)
    assert info["converged"]
    assert info["iterations"] * 2 <= cinfo["iterations"]
