"""Dense Cholesky solve of the assembled system (small grids only).

Sec. 3 states that the matrix problem is symmetric positive definite; the
Cholesky factorisation of the explicit L^2 x L^2 matrix (``assemble_dense``)
gives the exact solution up to rounding, independent of CG and of the FFT.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from .operator import assemble_dense


def solve_dense(g, d, b, padded):
    """x = A^{-1} b by Cholesky (scipy.linalg.cho_factor / cho_solve)."""
    A = assemble_dense(g, d, padded)
    c = scipy.linalg.cho_factor(A, lower=True)
    L = b.shape[0]
    return scipy.linalg.cho_solve(c, np.asarray(b, dtype=np.float64).ravel()).reshape(L, L)
