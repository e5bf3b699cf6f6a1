"""The largest grids (M = 8192): zero-padded L = 4096 and periodic L = 8192.

* one operator product, FP64 and FP32 operator, at 40 sampled outputs against
  the oracle's direct O(L^2) sum per output;
* a mixed-precision solve at L = 4096 (padded, eps = 1e-4, 30% zeros in d,
  b ~ N(0,1)): its error is certified from the oracle's FP64 residual
  (numpy-FFT product), a property that holds at any size; with and without
  the circulant preconditioner.
"""

import numpy as np
import pytest

from paper_1305_3625_amd import binding
from workloads import spectrum, padded_instance
from oracle import kernel_table, apply_direct_at, apply_fft, lambda_lb, error_bound
from gpu_util import dev, host, banner

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,padded", [(4096, 1), (8192, 0)])
def test_apply_sampled_M8192(L, padded):
    M = 2 * L if padded else L
    gh = spectrum(M, 1e-4)
    g = kernel_table(gh)
    rng = np.random.default_rng([96, L, padded])
    d = rng.uniform(0.0, 1.5, (L, L))
    x = rng.standard_normal((L, L))
    plan = binding.Plan(L, padded, gh)
    banner("apply-M8192", L, padded)
    rows = list(rng.integers(0, L, 34)) + [0, L - 1, 0, L - 1, L // 2, 1]
    cols = list(rng.integers(0, L, 34)) + [0, L - 1, L - 1, 0, L // 2, L - 2]
    ref = apply_direct_at(g, d, x, padded, rows, cols)
    scale = np.abs(x).max() * np.abs(g).sum()
    for prec, tol in ((binding.FP64, 1e-13), (binding.MIXED, 1e-6)):
        y = dev(np.zeros((L, L)))
        plan.apply(dev(d), dev(x), y, precision=prec)
        yh = host(y)
        e = np.max(np.abs(yh[rows, cols] - ref)) / scale
        print(f"apply M8192 L {L} pad {padded} prec {prec}: max sampled error / (max|x| sum|g|) {e:.3e}")
        assert e <= tol, prec
        del y
    plan.close()


@pytest.mark.parametrize("precond", [binding.PRECOND_NONE, binding.PRECOND_CIRCULANT])
def test_solve_L4096_mixed_certified(precond):
    import torch
    L = 4096
    inst = padded_instance(L, [97, 0], eps=1e-4, normal_b=True)
    plan = binding.Plan(L, 1, inst["ghat"])
    plan.set_precond(precond)
    banner("solve-L4096", precond)
    x = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, tol=1e-8, precision=binding.MIXED)
    xh = host(x)
    del x
    assert info["status"] == binding.OK
    r = inst["b"] - apply_fft(inst["ghat"], inst["d"], xh, 1)
    bound = error_bound(float(np.linalg.norm(r)), float(np.linalg.norm(xh)), lambda_lb(inst["ghat"], inst["d"]))
    print(f"L4096 precond {precond}: iters {info['iterations']} checks {info['checks']} certified {bound:.3e} "
          f"ms {info['device_ms']:.1f}")
    assert bound <= 1e-8
    plan.close()
