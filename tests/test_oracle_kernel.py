"""Pins of the oracle's kernel table g_M (inverse DFT of the multiplier).

Each check is fixed by the mathematics, not by re-running the oracle's own
formula: the DC sum, the value at the origin, Parseval, evenness, a term-by-term
complex DFT (sine terms included) and numpy's inverse FFT.
"""

import numpy as np
import pytest

from workloads import spectrum
from oracle import kernel_table, kernel_table_bruteforce


@pytest.mark.parametrize("M,eps", [(2, 0.5), (4, 1e-2), (8, 1e-3), (64, 1e-2), (256, 1e-4)])
def test_dc_sum_and_origin(M, eps):
    gh = spectrum(M, eps)
    g = kernel_table(gh)
    # sum over all separations = multiplier at k = 0
    assert np.sum(g) == pytest.approx(gh[0, 0], rel=1e-13)
    assert gh[0, 0] == pytest.approx(1 / np.sqrt(eps), rel=1e-15)
    # value at zero separation = mean of the multiplier
    assert g[0, 0] == pytest.approx(np.mean(gh), rel=1e-13)


@pytest.mark.parametrize("M", [4, 16, 128])
def test_parseval_and_evenness(M):
    gh = spectrum(M, 1e-3)
    g = kernel_table(gh)
    assert np.sum(g * g) == pytest.approx(np.sum(gh * gh) / M**2, rel=1e-12)
    idx = (-np.arange(M)) % M
    np.testing.assert_allclose(g, g[idx, :], rtol=0, atol=1e-14 * np.abs(g).max())
    np.testing.assert_allclose(g, g[:, idx], rtol=0, atol=1e-14 * np.abs(g).max())
    np.testing.assert_allclose(g, g.T, rtol=0, atol=1e-14 * np.abs(g).max())


@pytest.mark.parametrize("M", [2, 4, 8, 16])
def test_bruteforce_complex_dft(M):
    gh = spectrum(M, 1e-2)
    np.testing.assert_allclose(kernel_table(gh), kernel_table_bruteforce(gh),
                               rtol=0, atol=1e-13 * gh.max())


@pytest.mark.parametrize("M", [8, 64, 512])
def test_matches_numpy_ifft2(M):
    gh = spectrum(M, 1e-3)
    ref = np.fft.ifft2(gh)
    assert np.abs(ref.imag).max() < 1e-14 * gh.max()
    np.testing.assert_allclose(kernel_table(gh), ref.real, rtol=0, atol=1e-14 * gh.max())


def test_nonseparable_spectrum():
    """A random spectrum that is even in each index but not separable."""
    rng = np.random.default_rng(7)
    M = 8
    a = rng.random((M, M)) + 0.5
    idx = (-np.arange(M)) % M
    a = (a + a[idx, :] + a[:, idx] + a[idx][:, idx]) / 4
    np.testing.assert_allclose(kernel_table(a), kernel_table_bruteforce(a), atol=1e-14)
    np.testing.assert_allclose(kernel_table(a), np.fft.ifft2(a).real, atol=1e-14)


def test_planted_mistake_is_caught():
    """A kernel table missing the 1/M^2 normalisation, or built with a
    transposed multiplier on a non-symmetric spectrum, fails the pins."""
    rng = np.random.default_rng(3)
    M = 8
    a = rng.random((M, M)) + 0.5
    idx = (-np.arange(M)) % M
    a = (a + a[idx, :] + a[:, idx] + a[idx][:, idx]) / 4   # even, not symmetric
    good = kernel_table(a)
    bad_norm = good * M * M
    bad_transpose = kernel_table(a.T)
    bf = kernel_table_bruteforce(a)
    assert not np.allclose(bad_norm, bf, atol=1e-10)
    assert not np.allclose(bad_transpose, bf, atol=1e-10)
    assert np.allclose(good, bf, atol=1e-14)
