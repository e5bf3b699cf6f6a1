"""Real-space kernel table g_M from the DFT multiplier ghat.

Sec. 3: the Green's function depends only on the separation of two sites, so
the coupling matrix is a convolution, and eq. (3) states that it is diagonal
in Fourier space.  For an M x M multiplier ghat that is real and even in each
index, the real-space kernel is its inverse DFT

    g_M(a) = (1/M^2) sum_k ghat(k) exp(+2 pi i k.a / M)
           = (1/M^2) sum_k ghat(k) cos(2 pi k1 a1 / M) cos(2 pi k2 a2 / M),

because the sine terms are odd in k1 or k2 and cancel.  The normalisation
1/M^2 is the one Listing 3 applies after the inverse transform.
"""

from __future__ import annotations

import cmath
import math

import numpy as np


def _cos_matrix(M: int) -> np.ndarray:
    """Cos[a, k] = cos(2 pi ((a k) mod M) / M); the product is reduced exactly
    in integers before the library cosine."""
    a = np.arange(M, dtype=np.int64)
    return np.cos(2.0 * np.pi * ((np.outer(a, a) % M) / M))


def kernel_table(ghat: np.ndarray) -> np.ndarray:
    """g_M = (1/M^2) Cos @ ghat @ Cos^T, two FP64 matrix products, no FFT.

    Requires ghat real and even in each index (checked by the caller's pins).
    """
    ghat = np.asarray(ghat, dtype=np.float64)
    M = ghat.shape[0]
    if ghat.shape != (M, M):
        raise ValueError("ghat must be square")
    C = _cos_matrix(M)
    return (C @ ghat @ C.T) / float(M * M)


def kernel_table_bruteforce(ghat) -> np.ndarray:
    """The complex inverse DFT summed term by term in pure Python (sine terms
    included).  For tiny M only; it pins ``kernel_table``."""
    ghat = np.asarray(ghat, dtype=np.float64)
    M = ghat.shape[0]
    out = np.zeros((M, M))
    for a1 in range(M):
        for a2 in range(M):
            s = 0j
            for k1 in range(M):
                for k2 in range(M):
                    s += ghat[k1, k2] * cmath.exp(2j * math.pi * (k1 * a1 + k2 * a2) / M)
            out[a1, a2] = (s / (M * M)).real
    return out
