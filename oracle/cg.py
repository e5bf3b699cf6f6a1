"""Unpreconditioned conjugate gradient (Hestenes-Stiefel), FP64.

Sec. 3 solves the symmetric positive definite system by the conjugate
gradient method, without a preconditioner (Sec. 4).  The iteration is the
textbook one, from the mathematics: the step length alpha minimises the
A-norm of the error along the search direction p, alpha = (r.r)/(p.Ap); the
residual follows by r <- r - alpha Ap; the next direction is made
A-conjugate to p by beta = (r.r)_new/(r.r)_old, p <- r + beta p.
"""

from __future__ import annotations

import numpy as np


def cg(matvec, b, x0=None, tol=1e-10, maxit=10000, stagnation=20,
       record=False, x_true=None, matvec_true=None):
    """Solve A x = b by Hestenes-Stiefel CG.

    Stops when ||r||/||b|| <= tol (recursive residual), when the residual has
    not decreased for ``stagnation`` iterations, or after ``maxit``.
    Returns (x, info).  With ``record`` the per-iteration history of the
    recursive residual (and, if given, the error against ``x_true`` in the
    A-norm and the true residual via ``matvec_true``) is kept in ``info``.
    """
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.sqrt(np.sum(b * b)))
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = np.array(x0, dtype=np.float64)
        r = b - matvec(x)
    info = dict(iterations=0, bnorm=bnorm, converged=False, history=[])
    if bnorm == 0.0:
        info["converged"] = True
        return np.zeros_like(b), info
    p = r.copy()
    rho = float(np.sum(r * r))
    best = rho
    since_best = 0
    resids = [np.sqrt(rho)]
    if record:
        info["residuals"] = [r.copy()]
    for k in range(1, maxit + 1):
        q = matvec(p)
        pq = float(np.sum(p * q))
        if not (pq > 0.0) or not np.isfinite(pq):
            info["breakdown"] = True
            break
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        rho_new = float(np.sum(r * r))
        beta = rho_new / rho
        p = r + beta * p
        rho = rho_new
        info["iterations"] = k
        resids.append(np.sqrt(rho))
        if record:
            info["residuals"].append(r.copy())
            h = dict(k=k, rec=np.sqrt(rho))
            if x_true is not None and matvec_true is not None:
                e = x - x_true
                h["err_A"] = float(np.sqrt(np.sum(e * matvec_true(e))))
                h["true_res"] = float(np.sqrt(np.sum((b - matvec_true(x)) ** 2)))
            info["history"].append(h)
        if np.sqrt(rho) <= tol * bnorm:
            info["converged"] = True
            break
        if rho < best:
            best = rho
            since_best = 0
        else:
            since_best += 1
            if since_best >= stagnation:
                break
    info["rec_residuals"] = resids
    return x, info
