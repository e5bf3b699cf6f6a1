"""Pins of the oracle's operator A = diag(d) + C.

* dense assembly vs the direct real-space sum vs the FFT route (L <= 64,
  and padded L = 512);
* symmetry and positive definiteness, eigenvalues inside the closed-form
  bounds;
* plane waves are eigenvectors of the periodic operator with eigenvalue
  d + ghat(m, n) (eq. (3): C is diagonal in Fourier space);
* the padded operator equals P^T Circ_M P + diag(d) with Circ_M built from
  explicit complex DFT matrices.
"""

import numpy as np
import pytest

from workloads import spectrum, periodic_instance, padded_instance
from oracle import (kernel_table, conv_direct, apply_direct, apply_direct_at,
                    assemble_dense, apply_fft, lambda_lb, lambda_ub)
import oracle.operator as op_mod


def _inst(L, padded, seed=0):
    if padded:
        return padded_instance(L, [90, L, seed], eps=1e-3)
    return periodic_instance(L, [91, L, seed], eps=1e-2)


@pytest.mark.parametrize("L", [2, 4, 8, 16])
@pytest.mark.parametrize("padded", [0, 1])
def test_dense_equals_direct(L, padded):
    inst = _inst(L, padded)
    g = kernel_table(inst["ghat"])
    A = assemble_dense(g, inst["d"], padded)
    rng = np.random.default_rng(1)
    for _ in range(3):
        x = rng.standard_normal((L, L))
        np.testing.assert_allclose(apply_direct(g, inst["d"], x, padded),
                                   (A @ x.ravel()).reshape(L, L), rtol=0,
                                   atol=1e-13 * np.abs(A).sum(1).max() * np.abs(x).max())


@pytest.mark.parametrize("L", [4, 8, 16])
@pytest.mark.parametrize("padded", [0, 1])
def test_spd_and_bounds(L, padded):
    inst = _inst(L, padded)
    g = kernel_table(inst["ghat"])
    A = assemble_dense(g, inst["d"], padded)
    assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()
    w = np.linalg.eigvalsh(A)
    lo, hi = lambda_lb(inst["ghat"], inst["d"]), lambda_ub(inst["ghat"], inst["d"])
    assert w.min() > 0
    assert w.min() >= lo * (1 - 1e-12)
    assert w.max() <= hi * (1 + 1e-12)


@pytest.mark.parametrize("L", [4, 8, 32])
def test_periodic_plane_waves(L):
    eps = 1e-2
    gh = spectrum(L, eps)
    g = kernel_table(gh)
    dval = 0.7
    d = np.full((L, L), dval)
    i1, i2 = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    for (m, n) in [(0, 0), (1, 0), (0, 1), (1, 2), (L // 2, L // 2), (L - 1, 3 % L)]:
        ph = 2 * np.pi * ((m * i1 + n * i2) % L) / L
        for v in (np.cos(ph), np.sin(ph)):
            if np.abs(v).max() < 0.5:
                continue
            lam = dval + gh[m, n]
            np.testing.assert_allclose(apply_direct(g, d, v, 0), lam * v, rtol=0,
                                       atol=2e-14 * lam * L)


@pytest.mark.parametrize("L", [2, 4])
def test_padded_is_compressed_circulant(L):
    inst = _inst(L, 1)
    M = 2 * L
    gh = inst["ghat"]
    F1 = np.exp(-2j * np.pi * np.outer(np.arange(M), np.arange(M)) / M)
    F = np.kron(F1, F1)                     # 2-D DFT on row-major M x M
    Circ = (F.conj().T @ np.diag(gh.ravel()) @ F) / (M * M)
    assert np.abs(Circ.imag).max() < 1e-13
    keep = (np.arange(M)[:, None] * M + np.arange(M)[None, :])[:L, :L].ravel()
    A_ref = Circ.real[np.ix_(keep, keep)] + np.diag(inst["d"].ravel())
    A = assemble_dense(kernel_table(gh), inst["d"], 1)
    np.testing.assert_allclose(A, A_ref, rtol=0, atol=1e-13 * gh.max())


@pytest.mark.parametrize("L,padded", [(8, 0), (32, 0), (64, 0), (8, 1), (32, 1), (64, 1)])
def test_fft_route_equals_direct(L, padded):
    inst = _inst(L, padded)
    g = kernel_table(inst["ghat"])
    x = np.random.default_rng(5).standard_normal((L, L))
    yd = apply_direct(g, inst["d"], x, padded)
    yf = apply_fft(inst["ghat"], inst["d"], x, padded)
    np.testing.assert_allclose(yf, yd, rtol=0, atol=1e-13 * np.abs(yd).max())


@pytest.mark.parametrize("seed", [0, 1])
def test_fft_route_equals_direct_L512(seed):
    """The FFT route at padded L = 512 (M = 1024: the served M = 1024 class,
    the load-stepped sequences and the L = 512 FP64 workload lean on it)
    against the direct real-space sum, on random vectors and a diagonal with
    zeros; also at one worker thread (same result up to rounding)."""
    L = 512
    inst = padded_instance(L, [91, seed], eps=1e-3)
    g = kernel_table(inst["ghat"])
    x = np.random.default_rng([92, seed]).standard_normal((L, L))
    yd = apply_direct(g, inst["d"], x, 1)
    yf = apply_fft(inst["ghat"], inst["d"], x, 1)
    np.testing.assert_allclose(yf, yd, rtol=0, atol=1e-13 * np.abs(yd).max())
    y1 = apply_fft(inst["ghat"], inst["d"], x, 1, workers=1)
    np.testing.assert_allclose(y1, yd, rtol=0, atol=1e-13 * np.abs(yd).max())


@pytest.mark.parametrize("padded", [0, 1])
def test_sampled_outputs(padded):
    L = 16
    inst = _inst(L, padded)
    g = kernel_table(inst["ghat"])
    x = np.random.default_rng(6).standard_normal((L, L))
    y = apply_direct(g, inst["d"], x, padded)
    rows = [0, 3, 15, 7, 15]
    cols = [0, 9, 15, 0, 2]
    np.testing.assert_allclose(apply_direct_at(g, inst["d"], x, padded, rows, cols),
                               y[rows, cols], rtol=1e-13)


def test_planted_index_mistake_is_caught(monkeypatch):
    """A convolution that uses (i + j) instead of (i - j) for the column
    separation fails the plane-wave pin (the sine wave in particular)."""
    L = 8
    gh = spectrum(L, 1e-2)
    g = kernel_table(gh)
    d = np.full((L, L), 0.5)

    def wrong(g, x, padded):
        M = g.shape[0]
        y = np.zeros((L, L))
        col = (np.arange(L)[None, :] + np.arange(L)[:, None]) % M
        for delta in range(L):
            y += np.roll(x, delta, axis=0) @ g[delta][col]
        return y

    i1, i2 = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    v = np.sin(2 * np.pi * ((1 * i1 + 2 * i2) % L) / L)
    good = apply_direct(g, d, v, 0)
    assert np.allclose(good, (0.5 + gh[1, 2]) * v, atol=1e-13)
    monkeypatch.setattr(op_mod, "conv_direct", wrong)
    bad = op_mod.apply_direct(g, d, v, 0)
    assert not np.allclose(bad, (0.5 + gh[1, 2]) * v, atol=1e-6)


def test_shape_errors():
    g = np.zeros((8, 8))
    with pytest.raises(ValueError):
        conv_direct(g, np.zeros((8, 8)), True)
    with pytest.raises(ValueError):
        conv_direct(g, np.zeros((4, 4)), False)


def test_conv_direct_offsets_partition():
    """Partial sums over a partition of the row separations add up to the
    whole direct sum (the timing sample of the CPU baseline uses them)."""
    from oracle import conv_direct, kernel_table
    from workloads import spectrum
    L = 12
    g = kernel_table(spectrum(2 * L, 1e-3))
    x = np.random.default_rng([91, 0]).standard_normal((L, L))
    full = conv_direct(g, x, True)
    offs = list(range(-(L - 1), L))
    parts = conv_direct(g, x, True, offsets=offs[::2]) + conv_direct(g, x, True, offsets=offs[1::2])
    np.testing.assert_allclose(parts, full, rtol=0, atol=1e-13 * np.abs(full).max())
