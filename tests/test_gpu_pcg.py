"""The Fourier-space (circulant) preconditioned CG on the GPU against the
oracle (an extension beyond the paper's unpreconditioned solver).

* periodic grid with uniform d: the preconditioner is the exact inverse, so
  the solve needs one or two iterations;
* padded and periodic grids in both modes against the oracle's reference
  solution (run to stagnation): error <= 1e-10 (FP64) / 1e-8 (mixed), and at
  most about as many iterations as the oracle's own preconditioned CG and far
  fewer than plain CG;
* padded L = 2048 mixed: error certified from the oracle's FP64 residual;
* the server with a preconditioned plan: bitwise equal alone and in a mix,
  within the error bar of the oracle;
* error paths of fftcg_plan_set_precond.
"""

import time

import numpy as np
import pytest

from paper_1305_3625_amd import binding
from workloads import spectrum, periodic_instance, padded_instance, c2_instance, c3_instance, c4_request
from oracle import (reference_solve, apply_fft, pcg, circulant_precond, lambda_lb, error_bound)
from gpu_util import dev, host, relerr, banner

pytestmark = pytest.mark.gpu

MODES = [(binding.FP64, 1e-10, 1e-10), (binding.MIXED, 1e-8, 1e-8)]


def _solve(plan, inst, prec, tol, maxit=20000):
    import torch
    L = inst["L"]
    x = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, tol=tol, maxit=maxit, precision=prec,
                      raise_on_error=False)
    return host(x), info


def test_pcg_periodic_uniform_exact():
    L = 64
    gh = spectrum(L, 1e-2)
    d = np.full((L, L), 0.8)
    b = np.random.default_rng(90).uniform(0, 1, (L, L))
    xr = circulant_precond(gh, d, 0)(b)  # exact inverse here (pinned in the oracle tests)
    plan = binding.Plan(L, 0, gh)
    plan.set_precond(binding.PRECOND_CIRCULANT)
    inst = dict(L=L, d=d, b=b)
    for prec, tol, bar in MODES:
        banner("pcg-exact", prec)
        x, info = _solve(plan, inst, prec, tol)
        assert info["status"] == binding.OK, info
        assert info["iterations"] <= 2, info
        assert relerr(x, xr) <= bar


_REFS = {}


def _reference(L, padded):
    if (L, padded) not in _REFS:
        if (L, padded) == (512, 1):
            inst = c2_instance(0)
        elif padded:
            inst = padded_instance(L, [91, L], eps=1e-3)
        else:
            inst = periodic_instance(L, [92, L], eps=1e-2)
        xr, rinfo = reference_solve(inst["ghat"], inst["d"], inst["b"], padded,
                                    route="direct" if L <= 128 else "fft")
        assert rinfo["bound"] < 1e-12
        mv = lambda v: apply_fft(inst["ghat"], inst["d"], v, padded)  # noqa: E731
        _, pinfo = pcg(mv, circulant_precond(inst["ghat"], inst["d"], padded), inst["b"], tol=1e-10)
        _REFS[(L, padded)] = (inst, xr, pinfo["iterations"])
    return _REFS[(L, padded)]


@pytest.mark.parametrize("L,padded", [(16, 1), (64, 1), (128, 1), (512, 1), (64, 0)])
@pytest.mark.parametrize("mode", MODES)
def test_pcg_against_oracle(L, padded, mode):
    prec, tol, bar = mode
    inst, xr, oracle_iters = _reference(L, padded)
    plan = binding.Plan(L, padded, inst["ghat"])
    x0, info0 = _solve(plan, inst, prec, tol)  # plain CG on the same plan
    plan.set_precond(binding.PRECOND_CIRCULANT)
    banner("pcg", L, padded, prec)
    x, info = _solve(plan, inst, prec, tol)
    assert info["status"] == binding.OK, info
    err = relerr(x, xr)
    print(f"L {L} pad {padded} prec {prec}: pcg iters {info['iterations']} (oracle pcg {oracle_iters}, "
          f"cg {info0['iterations']}) checks {info['checks']} err {err:.3e} bound {info['error_bound']:.3e} "
          f"ms {info['device_ms']:.3f} (cg {info0['device_ms']:.3f})")
    assert err <= bar
    assert info["error_bound"] <= bar
    assert info["iterations"] <= oracle_iters + 4
    if padded and L >= 64:
        assert 2 * info["iterations"] <= info0["iterations"]


def test_pcg_L2048_mixed_certified():
    inst = c3_instance(0)
    plan = binding.Plan(2048, 1, inst["ghat"])
    plan.set_precond(binding.PRECOND_CIRCULANT)
    banner("pcg-L2048-mixed")
    x, info = _solve(plan, inst, binding.MIXED, inst["tol"])
    assert info["status"] == binding.OK, info
    r = inst["b"] - apply_fft(inst["ghat"], inst["d"], x, 1)
    bound = error_bound(float(np.linalg.norm(r)), float(np.linalg.norm(x)), lambda_lb(inst["ghat"], inst["d"]))
    print(f"L2048 pcg mixed: iters {info['iterations']} checks {info['checks']} certified {bound:.3e} "
          f"ms {info['device_ms']:.2f}")
    assert bound <= 1e-8
    assert info["iterations"] <= 60


def _wait(srv, tickets, L, timeout=120.0):
    out, t0 = {}, time.time()
    while len(out) < len(tickets):
        for tk in srv.completed():
            out[tk] = srv.poll(tk, L)
        if time.time() - t0 > timeout:
            raise TimeoutError("requests still pending")
        time.sleep(0.001)
    return out


def test_pcg_server_alone_equals_mix():
    M = 256
    plan = binding.Plan(M // 2, 1, spectrum(M, 1e-3))
    plan.set_precond(binding.PRECOND_CIRCULANT)
    reqs = [c4_request(500 + k, M) for k in range(5)]
    srv = binding.Server(memory_budget=1 << 30)
    banner("pcg-serve")
    alone = []
    for r in reqs:
        st, tk = srv.submit(plan, r["d"], r["b"], tol=1e-8)
        assert st == binding.OK
        res = _wait(srv, [tk], M // 2)[tk]
        assert res.status == binding.OK, res.info
        alone.append(res.x)
    tks = []
    for r in reqs:
        st, tk = srv.submit(plan, r["d"], r["b"], tol=1e-8)
        assert st == binding.OK
        tks.append(tk)
    res = _wait(srv, tks, M // 2)
    for tk, xa in zip(tks, alone):
        assert res[tk].status == binding.OK
        assert np.array_equal(res[tk].x, xa)
    srv.close()
    gh = spectrum(M, 1e-3)
    xr, _ = reference_solve(gh, reqs[0]["d"], reqs[0]["b"], 1)
    assert relerr(alone[0], xr) <= 1e-8


def test_set_precond_errors():
    plan = binding.Plan(16, 1, spectrum(32, 1e-3))
    with pytest.raises(binding.FftcgError):
        plan.set_precond(7)
    plan.set_precond(binding.PRECOND_CIRCULANT)
    plan.set_precond(binding.PRECOND_NONE)


def test_set_precond_refused_while_served():
    M = 1024
    plan = binding.Plan(M // 2, 1, spectrum(M, 1e-3))
    r = c4_request(600, M)
    srv = binding.Server(memory_budget=1 << 30)
    banner("pcg-in-use")
    st, tk = srv.submit(plan, r["d"], r["b"], tol=1e-8)
    assert st == binding.OK
    with pytest.raises(binding.FftcgError):
        plan.set_precond(binding.PRECOND_CIRCULANT)  # the request holds the plan
    res = _wait(srv, [tk], M // 2)[tk]
    assert res.status == binding.OK
    plan.set_precond(binding.PRECOND_CIRCULANT)
    srv.close()


def test_pcg_warm_start_and_zero_rhs():
    import torch
    L = 128
    inst, xr, _ = _reference(128, 1)
    plan = binding.Plan(L, 1, inst["ghat"])
    plan.set_precond(binding.PRECOND_CIRCULANT)
    banner("pcg-warm")
    x = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    cold = plan.solve(dev(inst["d"]), dev(inst["b"]), x, tol=1e-10, precision=binding.FP64)
    x0 = dev(xr * (1.0 + 1e-3))  # near the solution: 3 fewer orders of magnitude to go
    info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, x0=x0, tol=1e-10, precision=binding.FP64)
    assert info["status"] == binding.OK and info["iterations"] < cold["iterations"]
    assert relerr(host(x), xr) <= 1e-10
    z = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    info = plan.solve(dev(inst["d"]), z, x, tol=1e-10, precision=binding.MIXED)
    assert info["status"] == binding.OK and info["iterations"] == 0
    assert float(torch.abs(x).max()) == 0.0


def test_pcg_server_small_class():
    """L = 32 (a fused-engine class without a preconditioner) runs on the
    multi-pass engine once the plan is preconditioned."""
    M = 64
    gh = spectrum(M, 1e-3)
    plan = binding.Plan(M // 2, 1, gh)
    plan.set_precond(binding.PRECOND_CIRCULANT)
    reqs = [c4_request(700 + k, M) for k in range(3)]
    srv = binding.Server(memory_budget=1 << 28)
    banner("pcg-serve-small")
    tks = [srv.submit(plan, r["d"], r["b"], tol=1e-8)[1] for r in reqs]
    res = _wait(srv, tks, M // 2)
    for r, tk in zip(reqs, tks):
        assert res[tk].status == binding.OK
        xr, _ = reference_solve(gh, r["d"], r["b"], 1)
        assert relerr(res[tk].x, xr) <= 1e-8
    srv.close()
