"""Reference solves: FP64 CG run to stagnation, then certified.

The reference solution of A x = b is computed by the oracle's CG (Sec. 3) with
the direct real-space matvec (small and medium grids) or with the eq. (3)
FFT matvec (grids where the direct sum is too slow), driven to stagnation
(||r||/||b|| <= 1e-13 or no decrease over 20 iterations).  The true residual
is then recomputed and turned into a certified relative-error bound
(``bounds.error_bound``).  Errors of other solvers are measured against this
solution, never against one stopped at the same tolerance.
"""

from __future__ import annotations

import numpy as np

from .kernel_table import kernel_table
from .operator import apply_direct, apply_fft
from .cg import cg
from .bounds import lambda_lb, error_bound


def reference_solve(ghat, d, b, padded, x0=None, route="auto", tol=1e-13,
                    maxit=20000, g=None):
    """Returns (x, info) with info['bound'] the certified relative error."""
    M = ghat.shape[0]
    L = b.shape[0]
    if route == "auto":
        route = "direct" if L <= 256 else "fft"
    if route == "direct":
        if g is None:
            g = kernel_table(ghat)
        mv = lambda v: apply_direct(g, d, v, padded)  # noqa: E731
    elif route == "fft":
        mv = lambda v: apply_fft(ghat, d, v, padded)  # noqa: E731
    else:
        raise ValueError(route)
    x, info = cg(mv, b, x0=x0, tol=tol, maxit=maxit, stagnation=20)
    r = b - mv(x)
    rn = float(np.sqrt(np.sum(r * r)))
    xn = float(np.sqrt(np.sum(x * x)))
    lam = lambda_lb(ghat, d)
    info.update(route=route, true_res=rn, xnorm=xn, lambda_lb=lam,
                bound=error_bound(rn, xn, lam) if xn > 0 else 0.0,
                relres=rn / info["bnorm"] if info["bnorm"] > 0 else 0.0, M=M)
    return x, info
