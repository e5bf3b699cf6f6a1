"""The operator A = diag(d) + C on the L x L grid.

Sec. 2, eq. (1b): the displacement at site i is the sum over all sites j of
the Green's function of their separation times the force at j; eq. (2) gathers
this into one linear system.  In the SPD form used here

    (A x)(i) = d_i x_i + sum_{j in [0,L)^2} g_M((i - j) mod M) x_j ,

with g_M from ``kernel_table``.  Periodic grid: M = L.  Zero-padded grid:
M = 2L; separations lie in (-L, L)^2 where ``mod M`` is injective, so C is
the linear (Toeplitz-block-Toeplitz) convolution, i.e. "embed in M x M zeros,
convolve circularly, crop".

Routes (each pinned against the others and against closed forms):

* ``conv_direct``   the real-space sum organised by row separation: for each
  row offset delta, rows i1 of the output receive x[i1 - delta, :] @ T_delta
  where T_delta[j2, i2] = g_M(delta mod M, (i2 - j2) mod M).  Exactly L^4
  multiply-adds; no FFT.
* ``assemble_dense`` the L^2 x L^2 matrix entry by entry (small L).
* ``apply_direct_at`` single output entries, O(L^2) each, for sampling large
  grids.
* ``apply_fft``     eq. (3) literally: F^{-1}(ghat * F(pad x)), cropped, with
  scipy's 2-D FFT of real input as a library step (a real input has a
  Hermitian spectrum and ghat is real and even, so the product keeps that
  symmetry and the half spectrum n in [0, M/2] determines the result).  Used
  for grids where the direct sum is too slow; pinned against ``conv_direct``.
"""

from __future__ import annotations

import os

import numpy as np
import scipy.fft


def _check(g, x, padded):
    M = g.shape[0]
    L = x.shape[0]
    if x.shape != (L, L) or g.shape != (M, M):
        raise ValueError("shape mismatch")
    if (padded and M != 2 * L) or (not padded and M != L):
        raise ValueError("M must be 2L (padded) or L (periodic)")
    return L, M


def conv_direct(g: np.ndarray, x: np.ndarray, padded: bool, offsets=None) -> np.ndarray:
    """(C x)(i) = sum_j g_M((i-j) mod M) x_j by the direct real-space sum.

    ``offsets`` (padded grid only; default all of -(L-1)..L-1) restricts the
    sum to those row separations: a partial sum, used only to time a sample
    of the full sum's terms on large grids."""
    L, M = _check(g, x, padded)
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros((L, L))
    col = (np.arange(L)[None, :] - np.arange(L)[:, None]) % M  # [j2, i2] -> (i2 - j2) mod M
    if padded:
        for delta in (range(-(L - 1), L) if offsets is None else offsets):
            T = g[delta % M][col]
            if delta >= 0:
                y[delta:, :] += x[:L - delta, :] @ T
            else:
                y[:L + delta, :] += x[-delta:, :] @ T
    else:
        for delta in range(L):
            T = g[delta][col]
            # row i1 of the output takes row (i1 - delta) mod L of x
            y += np.roll(x, delta, axis=0) @ T
    return y


def apply_direct(g, d, x, padded):
    """(A x) = d * x + C x with the direct real-space convolution."""
    return np.asarray(d) * np.asarray(x) + conv_direct(g, x, padded)


def apply_direct_at(g, d, x, padded, rows, cols):
    """(A x)(i) for the listed sites i = (rows[k], cols[k]); O(L^2) each."""
    L, M = _check(g, x, padded)
    x = np.asarray(x, dtype=np.float64)
    j1 = np.arange(L)[:, None]
    j2 = np.arange(L)[None, :]
    out = np.empty(len(rows))
    for k, (i1, i2) in enumerate(zip(rows, cols)):
        w = g[(i1 - j1) % M, (i2 - j2) % M]
        out[k] = d[i1, i2] * x[i1, i2] + float(np.sum(w * x))
    return out


def assemble_dense(g, d, padded):
    """A as an explicit L^2 x L^2 matrix; site (i1, i2) is row i1*L + i2."""
    M = g.shape[0]
    L = M // 2 if padded else M
    i1, i2 = np.divmod(np.arange(L * L), L)
    A = g[(i1[:, None] - i1[None, :]) % M, (i2[:, None] - i2[None, :]) % M].copy()
    A[np.arange(L * L), np.arange(L * L)] += np.asarray(d, dtype=np.float64).ravel()
    return A


def host_workers():
    """Host threads this process may run on (the FFT library's worker count)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def apply_fft(ghat, d, x, padded, workers=None):
    """Eq. (3): d * x + crop(F^{-1}(ghat * F(embed x))) with scipy's FFT of
    real input, FP64, on ``workers`` host threads (default: all of them)."""
    M = ghat.shape[0]
    L = x.shape[0]
    if (padded and M != 2 * L) or (not padded and M != L):
        raise ValueError("M must be 2L (padded) or L (periodic)")
    w = host_workers() if workers is None else int(workers)
    xp = np.zeros((M, M))
    xp[:L, :L] = x
    X = scipy.fft.rfft2(xp, workers=w)
    y = scipy.fft.irfft2(ghat[:, :M // 2 + 1] * X, s=(M, M), workers=w)[:L, :L]
    return np.asarray(d) * x + y
