"""Full-size pin of the oracle's FFT route (run with RUN_SLOW=1; minutes).

At padded L = 2048 (M = 4096) the reference solutions the mixed-precision
solves are compared with come from CG with the eq. (3) FFT product.  Here
that route's solution of the L = 2048 workload (seed 0) is certified by a
residual b - A x computed with the direct real-space sum (L^4 = 1.8e13
multiply-adds, no FFT), turned into the closed-form error bound: the FFT
route's x is within 1e-11 of the exact solution.
"""

import numpy as np
import pytest

from workloads import c3_instance
from oracle import kernel_table, apply_direct, reference_solve, lambda_lb, error_bound

pytestmark = pytest.mark.slow


def test_fft_route_solution_certified_by_direct_residual_L2048():
    inst = c3_instance(0)
    x, info = reference_solve(inst["ghat"], inst["d"], inst["b"], 1, route="fft")
    g = kernel_table(inst["ghat"])
    r = inst["b"] - apply_direct(g, inst["d"], x, 1)
    rn = float(np.linalg.norm(r))
    bound = error_bound(rn, float(np.linalg.norm(x)), lambda_lb(inst["ghat"], inst["d"]))
    print(f"L=2048: {info['iterations']} iterations, FFT-route bound {info['bound']:.3e}, "
          f"direct-residual bound {bound:.3e}")
    assert bound <= 1e-11
    # the two residuals agree to the rounding of the two products
    assert abs(rn - info["true_res"]) <= 1e-12 * float(np.linalg.norm(inst["b"]))
