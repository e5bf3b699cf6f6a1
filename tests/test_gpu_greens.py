"""Solves with the physical Green's function of eq. (1c) on the GPU against
the oracle: the library builds the spectrum (fftcg_greens_spectrum), the
oracle builds its own (closed-form plaquette integrals, cosine-matrix DFT)
and solves to stagnation; uniform fibre stiffness k (d = 1/k), loads b."""

import numpy as np
import pytest

from paper_1305_3625_amd import binding
from oracle import green_spectrum, reference_solve
from gpu_util import dev, host, relerr, banner

pytestmark = pytest.mark.gpu

MODES = [(binding.FP64, 1e-10, 1e-10), (binding.MIXED, 1e-8, 1e-8)]


@pytest.mark.parametrize("L,padded", [(64, 0), (64, 1), (512, 1)])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("precond", [binding.PRECOND_NONE, binding.PRECOND_CIRCULANT])
def test_greens_solve(L, padded, mode, precond):
    import torch
    prec, tol, bar = mode
    nu, E, a, k = 0.3, 1.0, 1.0, 2.0
    M = 2 * L if padded else L
    rng = np.random.default_rng([95, L, padded])
    d = np.full((L, L), 1.0 / k)
    b = rng.uniform(0.0, 1.0, (L, L))
    gh_ref = green_spectrum(M, nu, E, a)
    xr, rinfo = reference_solve(gh_ref, d, b, padded, route="direct" if L <= 64 else "fft")
    assert rinfo["bound"] < 1e-12
    plan = binding.Plan(L, padded, binding.greens_spectrum(L, padded, nu, E, a))
    plan.set_precond(precond)
    banner("greens", L, padded, prec, precond)
    x = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    info = plan.solve(dev(d), dev(b), x, tol=tol, precision=prec)
    err = relerr(host(x), xr)
    print(f"greens L {L} pad {padded} prec {prec} pre {precond}: iters {info['iterations']} err {err:.2e}")
    assert info["status"] == binding.OK
    assert err <= bar
