"""Conjugate gradient with a Fourier-space (circulant) preconditioner.

An extension beyond the paper: Sec. 4 reports that the solver ran without a
preconditioner.  The operator's long-range part is a convolution, diagonal in
Fourier space (Sec. 3, eq. (3)); its diagonal part diag(d) is approximated
by its mean, the best multiple of the identity in the Frobenius norm (the
optimal circulant approximation of a diagonal matrix).  The preconditioner is
therefore the inverse of the M-periodic circulant

    S = dbar I + C_M,    dbar = mean(d),

applied to the zero-padded vector and cropped:  P^{-1} r = crop(S^{-1} pad(r)).
On a periodic grid (M = L) with uniform d it is exactly A^{-1}.  It is
symmetric positive definite for any grid (crop = pad^T and S is SPD since
ghat > 0, dbar >= 0).

The iteration is the textbook preconditioned CG: with z = P^{-1} r,
alpha = (r.z)/(p.Ap), x += alpha p, r -= alpha Ap, z = P^{-1} r,
beta = (r.z)_new/(r.z)_old, p = z + beta p.  Everything is FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import numpy as np
import scipy.fft

from .operator import host_workers


def circulant_precond(ghat, d, padded):
    """Returns z = P^{-1} r as a function of r (L x L arrays).  scipy's FFT of
    real input is a library step for S^{-1} = F^{-1} diag(1/(dbar + ghat)) F
    (1/(dbar + ghat) is real and even, so the half spectrum suffices)."""
    ghat = np.asarray(ghat, dtype=np.float64)
    M = ghat.shape[0]
    L = M // 2 if padded else M
    dbar = float(np.mean(d))
    inv = 1.0 / (dbar + ghat[:, :M // 2 + 1])
    w = host_workers()

    def apply(r):
        r = np.asarray(r, dtype=np.float64)
        z = np.zeros((M, M))
        z[:L, :L] = r
        y = scipy.fft.irfft2(scipy.fft.rfft2(z, workers=w) * inv, s=(M, M), workers=w)
        return y[:L, :L].copy()

    return apply


def pcg(matvec, precond, b, x0=None, tol=1e-10, maxit=10000, stagnation=20, record=False):
    """Solve A x = b by preconditioned CG.  Stops when ||r||/||b|| <= tol on
    the recursive residual, after ``stagnation`` iterations without decrease,
    or after ``maxit``.  Returns (x, info); ``record`` keeps the residuals and
    the preconditioned residuals of every iteration."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.sqrt(np.sum(b * b)))
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = np.array(x0, dtype=np.float64)
        r = b - matvec(x)
    info = dict(iterations=0, bnorm=bnorm, converged=False)
    if bnorm == 0.0:
        info["converged"] = True
        return np.zeros_like(b), info
    z = precond(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    rr = float(np.sum(r * r))
    best, since_best = rr, 0
    if record:
        info["residuals"] = [r.copy()]
        info["zs"] = [z.copy()]
    if np.sqrt(rr) <= tol * bnorm:
        info["converged"] = True
        return x, info
    for k in range(1, maxit + 1):
        q = matvec(p)
        pq = float(np.sum(p * q))
        if not (pq > 0.0) or not np.isfinite(pq):
            info["breakdown"] = True
            break
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        z = precond(r)
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        rr = float(np.sum(r * r))
        info["iterations"] = k
        if record:
            info["residuals"].append(r.copy())
            info["zs"].append(z.copy())
        if np.sqrt(rr) <= tol * bnorm:
            info["converged"] = True
            break
        if rr < best:
            best, since_best = rr, 0
        else:
            since_best += 1
            if since_best >= stagnation:
                break
    info["relres"] = float(np.sqrt(rr)) / bnorm
    return x, info
