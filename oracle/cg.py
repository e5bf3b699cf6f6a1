"""Unpreconditioned conjugate gradient in the order of Sec. 3, Listing 2.

Listing 2 lists, per iteration: the product of the matrix with the search
direction, the search length (a dot product), the new solution and the new
residual (two vector additions), the residual length (a dot product), the
update of the search direction (a vector addition) and a convergence check.
The paper uses no preconditioner (Sec. 4).  Everything is FP64.
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
        q = matvec(p)                       # product with the search direction
        pq = float(np.sum(p * q))           # search length ...
        if not (pq > 0.0) or not np.isfinite(pq):
            info["breakdown"] = True
            break
        alpha = rho / pq                    # ... alpha = rho / (p.q)
        x += alpha * p                      # new x
        r -= alpha * q                      # new residual
        rho_new = float(np.sum(r * r))      # residual length
        beta = rho_new / rho
        p = r + beta * p                    # update of the search direction
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
        if np.sqrt(rho) <= tol * bnorm:     # convergence check
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
