"""Load-step rule of the load-stepped workload.

Sec. 2: at each simulation step the displacement is set, the forces are
solved for, and bonds whose local strain exceeds their random threshold break.
The synthetic rule used here: after each solve, among the entries not yet
broken (d_i != 0), the one with the largest ratio x_i / t_i breaks
(d_i <- 0); ties go to the smallest row-major index.
"""

from __future__ import annotations

import numpy as np


def loadstep_argmax(x, t, d):
    """Row-major index of argmax_{i: d_i != 0} x_i / t_i (first on ties)."""
    ratio = np.asarray(x, dtype=np.float64).ravel() / np.asarray(t, dtype=np.float64).ravel()
    live = np.asarray(d).ravel() != 0.0
    if not np.any(live):
        return -1
    ratio = np.where(live, ratio, -np.inf)
    return int(np.argmax(ratio))


def loadstep_valid(j, x_ref, t, d, e_inf):
    """Whether index j is an acceptable choice given the reference solution
    x_ref and a bound e_inf on the max-norm error of the solution that chose
    j (near-ties admit several correct answers)."""
    t = np.asarray(t, dtype=np.float64).ravel()
    xr = np.asarray(x_ref, dtype=np.float64).ravel()
    live = np.asarray(d).ravel() != 0.0
    if j < 0 or not live[j]:
        return False
    k = loadstep_argmax(x_ref, t, d)
    rho = xr / t
    return rho[j] >= rho[k] - e_inf * (1.0 / t[j] + 1.0 / t[k])
