"""The quasi-static fracture driver of Sec. 2 (displacement control, uniform
fibre stiffness k, fibres breaking one at a time).

At unit displacement the intact fibres I carry f_I with

    (I/k + G)_II f_I = 1_I,

eq. (2) divided by k and restricted to the intact set: a broken fibre
carries no force (f_i = 0) and drops out of the system.  The forces scale
linearly with the displacement D, so the intact fibre with the largest
f_i / t_i breaks first, at D = t_i / f_i (ties to the smallest row-major
index); then the system is solved again without it.  The breaking rule
and the threshold distribution of the paper's references are not given;
this is the rule the paper's description implies.

``restricted_solve`` solves the restricted system by CG on the projected
operator P A P (P the 0/1 mask) with the right-hand side P 1: the iterates
stay in the intact subspace, where P A P is SPD.  ``fracture_sequence``
runs the driver, or replays a given sequence of broken fibres (to compare
against another implementation step by step where near-ties admit several
answers).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import numpy as np

from .cg import cg
from .operator import apply_fft


def restricted_solve(ghat, k, mask, padded, x0=None, tol=1e-13, maxit=20000):
    """f with (I/k + C)_II f_I = 1_I and f = 0 off I (mask: 1 intact, 0 broken)."""
    m = np.asarray(mask, dtype=np.float64)
    d = np.full(m.shape, 1.0 / k)
    mv = lambda v: m * apply_fft(ghat, d, m * v, padded)  # noqa: E731
    f, info = cg(mv, m.copy(), x0=None if x0 is None else m * x0, tol=tol, maxit=maxit)
    return m * f, info


def fracture_sequence(ghat, k, t, steps, padded, replay=None, tol=1e-13):
    """Returns (broken, dbreak, f, ratios): the fibre broken at each step, the
    displacement at which it breaks, the final forces, and each step's full
    f / t array (intact entries; -inf elsewhere) for validating choices."""
    L = t.shape[0]
    mask = np.ones((L, L))
    f = np.zeros((L, L))
    broken, dbreak, ratios = [], [], []
    for s in range(steps):
        f, _ = restricted_solve(ghat, k, mask, padded, x0=f, tol=tol)
        rho = np.where(mask > 0, f / t, -np.inf)
        ratios.append(rho)
        if replay is None:
            i = int(np.argmax(rho.ravel()))  # first maximum: ties to the smallest index
        else:
            i = int(replay[s])
        broken.append(i)
        v = rho.ravel()[i]
        dbreak.append(1.0 / v if v > 0 else np.inf)
        mask.ravel()[i] = 0.0
    return np.array(broken), np.array(dbreak), f, ratios
