"""The physical Green's function of Sec. 2, eq. (1c), and its spectrum.

Eq. (1c) couples fibre i to fibre j through the 1/r kernel of an elastic
half-space averaged over the square plaquette (side a) of fibre j:

    G(Delta) = (1 - nu^2) / (pi E a^2) * integral over the plaquette centred
               at Delta a of dx' dy' / |r'|.

With lengths in units of a the integral is a * P(Delta), where P is the
integral of 1/r over the unit square centred at Delta; P has the closed form
of the four-corner sum of the antiderivative x ln(y + r) + y ln(x + r) of
1/r (a standard primitive, checked against numerical quadrature in the
tests).  So G(Delta) = (1 - nu^2)/(pi E a) * P(Delta).

On the M x M FFT grid the kernel table takes each index a in [0, M) to the
separation a (a <= M/2) or a - M (a > M/2), whose magnitude min(a, M - a)
is what enters P (even in each argument); the spectrum is its DFT,
real and even because the table is; computed here by cosine-matrix products
(the plain DFT definition, no FFT).  The paper gives no values of nu, E, a.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import numpy as np


def _xlog(x, u):
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(x != 0, x * np.log(np.where(u > 0, u, 1)), 0)


def _primitive(x, y):
    """x ln(y + r) + y ln(x + r), r = |(x, y)|: d^2/dx dy of it is 1/r."""
    r = np.hypot(x, y)
    return _xlog(x, y + r) + _xlog(y, x + r)


def plaquette_integral(dx, dy):
    """Integral of 1/r over the unit square centred at (dx, dy).  The
    four-corner sum cancels O(r log r) terms down to O(1/r), so it is formed
    in extended precision (numpy longdouble) and rounded once."""
    dx = np.asarray(dx, dtype=np.longdouble)
    dy = np.asarray(dy, dtype=np.longdouble)
    h = np.longdouble(0.5)
    x0, x1, y0, y1 = dx - h, dx + h, dy - h, dy + h
    v = _primitive(x1, y1) - _primitive(x0, y1) - _primitive(x1, y0) + _primitive(x0, y0)
    return np.asarray(v, dtype=np.float64)


def green_table(M, nu, E, a):
    """G on the M x M grid (minimal-image separations), eq. (1c)."""
    idx = np.arange(M)
    # |separation| (P is even in each argument), so the table is exactly even
    sep = np.minimum(idx, M - idx).astype(np.float64)
    pref = (1.0 - nu * nu) / (np.pi * E * a)
    return pref * plaquette_integral(sep[:, None], sep[None, :])


def green_spectrum(M, nu, E, a):
    """DFT of green_table: ghat(m, n) = sum_ab G(a, b) cos(2 pi m a/M) cos(2 pi n b/M)
    (the sine terms cancel: G is even in each index)."""
    g = green_table(M, nu, E, a)
    k = np.arange(M)
    C = np.cos(2.0 * np.pi * ((np.outer(k, k)) % M) / M)
    return C @ g @ C.T
