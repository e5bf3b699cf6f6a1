"""Pins of the oracle's Green's function of eq. (1c) and its spectrum.

* the plaquette integral of 1/r: the self term has the closed value
  4 ln(1 + sqrt 2); other separations agree with adaptive 2-D quadrature
  (scipy dblquad); far away it tends to the point value 1/|Delta| with an
  O(|Delta|^-3) correction; a planted sign mistake in the primitive fails;
* the table is even in each index, and its spectrum (cosine-matrix DFT)
  agrees with numpy's FFT (an independent library route), is real, even and
  strictly positive (so diag(d) + C is SPD for any d >= 0).
"""

import numpy as np
import pytest
from scipy import integrate

from oracle import plaquette_integral, green_table, green_spectrum
from oracle.greens import _xlog


def test_self_term_closed_value():
    assert plaquette_integral(0.0, 0.0) == pytest.approx(4.0 * np.log(1.0 + np.sqrt(2.0)), rel=1e-15)


@pytest.mark.parametrize("dx,dy", [(1.0, 0.0), (0.0, 2.0), (2.0, 3.0), (-3.0, 1.0), (5.0, 5.0)])
def test_against_quadrature(dx, dy):
    v, _ = integrate.dblquad(lambda y, x: 1.0 / np.hypot(dx - x, dy - y), -0.5, 0.5, -0.5, 0.5,
                             epsabs=1e-13, epsrel=1e-13)
    assert plaquette_integral(dx, dy) == pytest.approx(v, rel=1e-11)


def test_far_field():
    for dx, dy in [(30.0, 0.0), (20.0, 25.0), (0.0, 60.0)]:
        r = np.hypot(dx, dy)
        assert abs(plaquette_integral(dx, dy) - 1.0 / r) <= 0.1 / r**3


def test_planted_sign_mistake_fails():
    def wrong(dx, dy):
        def prim(x, y):
            r = np.hypot(x, y)
            return _xlog(x, y + r) - _xlog(y, x + r)  # sign error
        x0, x1, y0, y1 = dx - 0.5, dx + 0.5, dy - 0.5, dy + 0.5
        return prim(x1, y1) - prim(x0, y1) - prim(x1, y0) + prim(x0, y0)
    v, _ = integrate.dblquad(lambda y, x: 1.0 / np.hypot(2.0 - x, 3.0 - y), -0.5, 0.5, -0.5, 0.5)
    assert abs(wrong(2.0, 3.0) - v) > 1e-3


@pytest.mark.parametrize("M", [8, 16, 64])
def test_spectrum(M):
    nu, E, a = 0.3, 2.0, 0.5
    g = green_table(M, nu, E, a)
    assert np.array_equal(g, g[(-np.arange(M)) % M][:, (-np.arange(M)) % M])
    gh = green_spectrum(M, nu, E, a)
    F = np.fft.fft2(g)
    assert np.max(np.abs(F.imag)) <= 1e-12 * np.max(np.abs(F.real))
    assert np.max(np.abs(gh - F.real)) <= 1e-12 * np.max(np.abs(gh))
    assert np.allclose(gh, gh.T, rtol=0, atol=1e-12 * np.abs(gh).max())
    assert gh.min() > 0.0
    pref = (1 - nu * nu) / (np.pi * E * a)
    assert gh.min() == pytest.approx(1.8243 * pref, rel=2e-3)  # the lattice kernel's smallest eigenvalue


def test_far_field_series_to_rounding():
    """Far away, P = 1/r + 1/(24 r^3) + O(r^-5) (monopole plus the square's
    quadrupole): the extended-precision corner sum reaches it to ~1e-13."""
    for dx, dy in [(2000.0, 1000.0), (4095.0, 0.0), (1500.0, 1500.0)]:
        r = np.hypot(dx, dy)
        ref = 1.0 / r + 1.0 / (24.0 * r**3)
        assert plaquette_integral(dx, dy) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("L,padded", [(4, 1), (16, 0), (32, 1), (64, 1)])
def test_library_spectrum_matches_oracle(L, padded):
    """fftcg_greens_spectrum (host code of the library: plan-time set-up, no
    GPU) against the oracle's cosine-matrix DFT of the same table."""
    from paper_1305_3625_amd import binding
    nu, E, a = 0.25, 3.0, 1.5
    M = 2 * L if padded else L
    lib = binding.greens_spectrum(L, padded, nu, E, a)
    ref = green_spectrum(M, nu, E, a)
    assert np.max(np.abs(lib - ref)) <= 1e-13 * np.max(np.abs(ref))
    m = np.arange(M)
    assert np.array_equal(lib, lib[(-m) % M]) and np.array_equal(lib, lib[:, (-m) % M])


def test_library_spectrum_errors():
    from paper_1305_3625_amd import binding
    for args in [(3, 1, 0.3, 1.0, 1.0), (16, 1, 1.0, 1.0, 1.0), (16, 1, 0.3, 0.0, 1.0), (16, 1, 0.3, 1.0, -1.0),
                 (8192, 1, 0.3, 1.0, 1.0), (16, 2, 0.3, 1.0, 1.0)]:
        with pytest.raises(binding.FftcgError):
            binding.greens_spectrum(*args)
