"""Closed-form spectrum bounds of A = diag(d) + C and the certified stop rule.

The circular convolution on the M x M grid has eigenvalues ghat(k) (eq. (3):
C is diagonal in Fourier space).  The L x L operator is that circulant (M = L)
or a principal compression of it (zero-padded, M = 2L), so by Cauchy
interlacing its eigenvalues lie in [min ghat, max ghat]; Weyl's inequality then
bounds the eigenvalues of A by [min d + min ghat, max d + max ghat].

For any approximate solution x with residual r = b - A x,
    ||x - x*|| <= ||r|| / lambda_lb,   ||x*|| >= ||x|| - ||x - x*||,
so  ||x - x*|| / ||x*|| <= tau  holds whenever
    ||r|| <= tau * lambda_lb * ||x|| / (1 + tau).
"""

from __future__ import annotations

import numpy as np


def lambda_lb(ghat, d):
    return float(np.min(d)) + float(np.min(ghat))


def lambda_ub(ghat, d):
    return float(np.max(d)) + float(np.max(ghat))


def kappa_ub(ghat, d):
    return lambda_ub(ghat, d) / lambda_lb(ghat, d)


def certified_ok(rnorm, xnorm, tau, lam_lb):
    """True when the residual certifies relative error <= tau."""
    return rnorm <= tau * lam_lb * xnorm / (1.0 + tau)


def error_bound(rnorm, xnorm, lam_lb):
    """Upper bound on ||x - x*|| / ||x*|| from the residual norm."""
    e = rnorm / lam_lb
    if xnorm <= e:
        return float("inf")
    return e / (xnorm - e)
