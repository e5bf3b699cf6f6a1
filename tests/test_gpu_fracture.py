"""The fracture driver (fftcg_fracture) on the GPU against the oracle's
driver (Sec. 2): the oracle replays the GPU's sequence of broken fibres and
checks every choice is a valid argmax of f/t up to the solves' certified
error (near-ties admit several answers), the breaking displacements agree,
and the final forces agree within the error bar."""

import numpy as np
import pytest

from paper_1305_3625_amd import binding
from workloads import spectrum, fracture_instance
from oracle import fracture_sequence
from gpu_util import dev, host, relerr, banner

pytestmark = pytest.mark.gpu

MODES = [(binding.FP64, 1e-10), (binding.MIXED, 1e-8)]


@pytest.mark.parametrize("L", [16, 64])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("precond", [binding.PRECOND_NONE, binding.PRECOND_CIRCULANT])
def test_fracture_against_oracle(L, mode, precond):
    import torch
    prec, tol = mode
    steps = 30
    inst = fracture_instance(2, L=L)
    gh = spectrum(2 * L, 1e-3)
    plan = binding.Plan(L, 1, gh)
    plan.set_precond(precond)
    f = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    banner("fracture", L, prec, precond)
    st, broken, dbreak, iters = plan.fracture(inst["k"], dev(inst["t"]), f, steps, tol=tol, precision=prec)
    assert st == binding.OK
    fo_broken, fo_dbreak, fo_f, ratios = fracture_sequence(gh, inst["k"], inst["t"], steps, 1, replay=broken)
    t = inst["t"].ravel()
    for s in range(steps):
        rho = ratios[s].ravel()
        k = int(np.argmax(rho))
        j = int(broken[s])
        assert np.isfinite(rho[j]), (s, j)  # an intact fibre
        # per-entry error of f <= ||f - f*|| <= tol ||f|| (certified)
        einf = 2 * tol * np.linalg.norm(np.where(np.isfinite(rho), rho * t, 0.0))
        assert rho[j] >= rho[k] - einf * (1.0 / t[j] + 1.0 / t[k]), (s, j, k)
    np.testing.assert_allclose(dbreak, fo_dbreak, rtol=50 * tol)
    assert relerr(host(f), fo_f) <= 10 * tol
    print(f"L {L} prec {prec} pre {precond}: mean iters {iters.mean():.1f}, first D {dbreak[0]:.6f}, "
          f"last D {dbreak[-1]:.6f}")
    plan.close()


def test_fracture_errors():
    import torch
    plan = binding.Plan(16, 1, spectrum(32, 1e-3))
    f = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    t = dev(np.ones((16, 16)))
    for bad in [dict(k=0.0), dict(steps=0), dict(steps=257), dict(tol=0.0), dict(maxit=0)]:
        args = dict(k=1.0, steps=4, tol=1e-8, maxit=100)
        args.update(bad)
        st, *_ = plan.fracture(args["k"], t, f, args["steps"], tol=args["tol"], maxit=args["maxit"])
        assert st == binding.EINVAL, bad


def test_fracture_breaks_everything():
    """L = 4: all 16 fibres break, each exactly once, in an order the oracle
    accepts; the last step has a single intact fibre."""
    import torch
    L = 4
    inst = fracture_instance(3, L=L)
    gh = spectrum(2 * L, 1e-2)
    plan = binding.Plan(L, 1, gh)
    f = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    banner("fracture-all")
    st, broken, dbreak, iters = plan.fracture(inst["k"], dev(inst["t"]), f, L * L, tol=1e-10,
                                              precision=binding.FP64)
    assert st == binding.OK
    assert sorted(broken.tolist()) == list(range(L * L))
    _, fo_dbreak, _, _ = fracture_sequence(gh, inst["k"], inst["t"], L * L, 1, replay=broken)
    np.testing.assert_allclose(dbreak, fo_dbreak, rtol=1e-8)
    assert float(torch.abs(f).sum()) > 0.0  # the last intact fibre carried the load
