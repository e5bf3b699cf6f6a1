"""Parity of fftcg_solve on the GPU against the oracle.

* closed form (periodic, uniform d, constant b);
* dense Cholesky on grids up to 16 x 16, periodic and padded, both modes;
* periodic L = 64 instances (eps 1e-2) against the oracle's direct-route CG
  run to stagnation: relative error <= 1e-10 (FP64);
* the serving grids on both engines: padded L = 32, 64, 128 (M <= 256) and
  periodic L = 128, 256, against the oracle's direct-route CG, both modes;
* padded L = 512 (eps 1e-3, 30% zeros in d) against the oracle's FFT-route
  reference: <= 1e-10 (FP64) and <= 1e-8 (mixed);
* padded L = 2048 (eps 1e-4, b ~ N(0,1)) in mixed precision: the error is
  certified from the oracle's FP64 residual of the GPU solution (a property
  that holds at any size), <= 1e-8;
* edge cases: b = 0, maxit = 1, warm start at the solution, invalid d;
* results do not depend on how the host splits a solve into launched
  chunks (bitwise, padded L = 512, both modes).
"""

import numpy as np
import pytest

from paper_1305_3625_amd import binding
from workloads import spectrum, periodic_instance, padded_instance, c1_instance, c2_instance, c3_instance
from oracle import (kernel_table, solve_dense, reference_solve, apply_fft, lambda_lb, error_bound)
from gpu_util import dev, host, relerr, banner

pytestmark = pytest.mark.gpu

MODES = [(binding.FP64, 1e-10, 1e-10), (binding.MIXED, 1e-8, 1e-8)]


def _solve(plan, inst, prec, tol, x0=None, maxit=20000):
    import torch
    L = inst["L"]
    x = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, x0=x0, tol=tol, maxit=maxit, precision=prec,
                      raise_on_error=False)
    return host(x), info


def test_closed_form():
    L = 64
    gh = spectrum(L, 1e-2)
    plan = binding.Plan(L, 0, gh)
    inst = dict(L=L, d=np.full((L, L), 0.8), b=np.full((L, L), 0.37))
    for prec, tol, _ in MODES:
        banner("closed-form", prec)
        x, info = _solve(plan, inst, prec, tol)
        assert info["status"] == binding.OK
        np.testing.assert_allclose(x, 0.37 / (0.8 + 10.0), rtol=1e-12 if prec == binding.FP64 else 1e-8)
        assert info["iterations"] <= 2


@pytest.mark.parametrize("L", [2, 4, 8, 16])
@pytest.mark.parametrize("padded", [0, 1])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("engine", [binding.ENGINE_MULTIPASS, binding.ENGINE_FUSED])
def test_cholesky(L, padded, mode, engine):
    prec, tol, bar = mode
    inst = padded_instance(L, [60, L], eps=1e-3) if padded else periodic_instance(L, [61, L], eps=1e-2)
    g = kernel_table(inst["ghat"])
    xs = solve_dense(g, inst["d"], inst["b"], padded)
    plan = binding.Plan(L, padded, inst["ghat"])
    plan.set_engine(engine)
    banner("cholesky", L, padded, prec, engine)
    x, info = _solve(plan, inst, prec, tol)
    assert info["status"] == binding.OK, info
    err = relerr(x, xs)
    assert err <= bar, (err, info)
    assert info["error_bound"] <= bar


@pytest.mark.parametrize("s", [0, 1, 2, 3])
@pytest.mark.parametrize("engine", [binding.ENGINE_MULTIPASS, binding.ENGINE_FUSED])
def test_periodic_L64(s, engine):
    inst = c1_instance(s)
    xr, rinfo = reference_solve(inst["ghat"], inst["d"], inst["b"], 0)
    assert rinfo["bound"] < 1e-12
    plan = binding.Plan(64, 0, inst["ghat"])
    plan.set_engine(engine)
    banner("periodic-L64", s, engine)
    x, info = _solve(plan, inst, binding.FP64, inst["tol"])
    assert info["status"] == binding.OK
    err = relerr(x, xr)
    print(f"seed {s} engine {engine}: iters {info['iterations']} err {err:.3e} bound {info['error_bound']:.3e} "
          f"ms {info['device_ms']:.3f}")
    assert err <= 1e-10
    assert info["error_bound"] <= 1e-10


_REFS = {}


def _serving_reference(L, padded):
    if (L, padded) not in _REFS:
        inst = padded_instance(L, [63, L], eps=1e-3) if padded else periodic_instance(L, [64, L], eps=1e-2)
        xr, rinfo = reference_solve(inst["ghat"], inst["d"], inst["b"], padded, route="direct" if L <= 128 else "fft")
        assert rinfo["bound"] < 1e-12
        _REFS[(L, padded)] = (inst, xr)
    return _REFS[(L, padded)]


@pytest.mark.parametrize("L,padded", [(32, 1), (64, 1), (128, 1), (128, 0), (256, 0), (256, 1)])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("engine", [binding.ENGINE_MULTIPASS, binding.ENGINE_FUSED])
def test_serving_grids(L, padded, mode, engine):
    if engine == binding.ENGINE_FUSED and (2 * L if padded else L) > 256:
        pytest.skip("the fused engine serves M <= 256")
    prec, tol, bar = mode
    inst, xr = _serving_reference(L, padded)
    plan = binding.Plan(L, padded, inst["ghat"])
    plan.set_engine(engine)
    banner("serving-grid", L, padded, prec, engine)
    x, info = _solve(plan, inst, prec, tol)
    assert info["status"] == binding.OK, info
    err = relerr(x, xr)
    print(f"L {L} pad {padded} prec {prec} engine {engine}: iters {info['iterations']} checks {info['checks']} "
          f"err {err:.3e} bound {info['error_bound']:.3e} ms {info['device_ms']:.3f}")
    assert err <= bar
    assert info["error_bound"] <= bar


@pytest.fixture(scope="module")
def padded512():
    inst = c2_instance(0)
    xr, rinfo = reference_solve(inst["ghat"], inst["d"], inst["b"], 1, route="fft")
    assert rinfo["bound"] < 1e-12
    return inst, xr


@pytest.mark.parametrize("mode", MODES)
def test_padded_L512(padded512, mode):
    prec, tol, bar = mode
    inst, xr = padded512
    plan = binding.Plan(512, 1, inst["ghat"])
    banner("padded-L512", prec)
    x, info = _solve(plan, inst, prec, tol)
    assert info["status"] == binding.OK
    err = relerr(x, xr)
    print(f"mode {prec}: iters {info['iterations']} checks {info['checks']} err {err:.3e} "
          f"bound {info['error_bound']:.3e} ms {info['device_ms']:.2f}")
    assert err <= bar


@pytest.mark.parametrize("mode", MODES)
def test_results_independent_of_launch_chunking(padded512, mode):
    """The host only chooses how many iterations each launched chunk holds,
    from the check intervals seen so far in the solve and, in mixed
    precision, in the previous solve on the same plan; every check and stop
    decision is taken on the device, and every reduction has a fixed order.
    So a solve gives bitwise the same x, iteration and check counts on a
    fresh plan, after a solve of another instance, and after itself."""
    prec, tol, _ = mode
    inst, _ = padded512
    other = c2_instance(1)
    banner("chunking-independence", prec)
    fresh = binding.Plan(512, 1, inst["ghat"])
    x_a, info_a = _solve(fresh, inst, prec, tol)
    used = binding.Plan(512, 1, inst["ghat"])
    _, info_o = _solve(used, other, prec, tol)
    x_b, info_b = _solve(used, inst, prec, tol)
    x_c, info_c = _solve(used, inst, prec, tol)
    print(f"mode {prec}: iters {info_a['iterations']} / other {info_o['iterations']} / "
          f"{info_b['iterations']} / {info_c['iterations']}, checks {info_a['checks']}")
    for x, info in ((x_b, info_b), (x_c, info_c)):
        assert info["status"] == binding.OK
        assert (info["iterations"], info["checks"]) == (info_a["iterations"], info_a["checks"])
        assert np.array_equal(x, x_a)


def test_padded_L2048_mixed_certified():
    inst = c3_instance(0)
    plan = binding.Plan(2048, 1, inst["ghat"])
    banner("padded-L2048-mixed")
    x, info = _solve(plan, inst, binding.MIXED, inst["tol"])
    assert info["status"] == binding.OK
    r = inst["b"] - apply_fft(inst["ghat"], inst["d"], x, 1)
    rn, xn = np.linalg.norm(r), np.linalg.norm(x)
    bound = error_bound(rn, xn, lambda_lb(inst["ghat"], inst["d"]))
    print(f"L2048 mixed: iters {info['iterations']} checks {info['checks']} oracle-certified bound {bound:.3e} "
          f"relres {rn / np.linalg.norm(inst['b']):.3e} ms {info['device_ms']:.1f}")
    assert bound <= 1e-8
    assert rn / np.linalg.norm(inst["b"]) <= inst["tol"]


def test_zero_rhs():
    L = 32
    inst = padded_instance(L, [62, 0])
    inst["b"] = np.zeros((L, L))
    plan = binding.Plan(L, 1, inst["ghat"])
    import torch
    x0 = dev(np.ones((L, L)))
    for prec, tol, _ in MODES:
        x = torch.full((L, L), 7.0, dtype=torch.float64, device="cuda")
        info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, x0=x0, tol=tol, precision=prec)
        assert info["status"] == binding.OK and info["iterations"] == 0
        assert np.all(host(x) == 0.0)


def test_maxit_one_returns_last_iterate():
    L = 64
    inst = padded_instance(L, [63, 0])
    plan = binding.Plan(L, 1, inst["ghat"])
    for prec, tol, _ in MODES:
        x, info = _solve(plan, inst, prec, tol, maxit=1)
        assert info["status"] == binding.ENOCONV
        assert info["iterations"] == 1
        # one CG step from zero: x = alpha b with alpha = b.b / b.Ab
        from oracle import apply_direct
        g = kernel_table(inst["ghat"])
        Ab = apply_direct(g, inst["d"], inst["b"], 1)
        alpha = np.sum(inst["b"] ** 2) / np.sum(inst["b"] * Ab)
        assert relerr(x, alpha * inst["b"]) <= (1e-12 if prec == binding.FP64 else 1e-6)


def test_warm_start_at_solution():
    L = 32
    inst = padded_instance(L, [64, 0])
    g = kernel_table(inst["ghat"])
    xs = solve_dense(g, inst["d"], inst["b"], 1)
    plan = binding.Plan(L, 1, inst["ghat"])
    import torch
    x = dev(xs)
    info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, x0=x, tol=1e-10, precision=binding.FP64)
    assert info["status"] == binding.OK
    assert info["iterations"] <= 1
    assert relerr(host(x), xs) <= 1e-12


@pytest.mark.parametrize("bad", ["nan_d", "neg_d", "inf_b"])
def test_invalid_data(bad):
    L = 16
    inst = padded_instance(L, [65, 0])
    if bad == "nan_d":
        inst["d"][3, 4] = np.nan
    elif bad == "neg_d":
        inst["d"][0, 0] = -0.5
    else:
        inst["b"][5, 5] = np.inf
    plan = binding.Plan(L, 1, inst["ghat"])
    for prec, tol, _ in MODES:
        x, info = _solve(plan, inst, prec, tol)
        assert info["status"] == binding.EINVAL


@pytest.mark.parametrize("engine", [binding.ENGINE_MULTIPASS, binding.ENGINE_FUSED])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_breakdown_on_non_finite_start(engine, bad):
    """A non-finite start vector makes the first true residual non-finite:
    the solve ends with EBREAKDOWN (both precisions), and the next solve on
    the same plan is unaffected."""
    import torch
    L = 32
    inst = padded_instance(L, [65, 0])
    plan = binding.Plan(L, 1, inst["ghat"])
    plan.set_engine(engine)
    x0 = np.zeros((L, L))
    x0[3, 7] = bad
    for prec, tol, _ in MODES:
        banner("breakdown", engine, bad, prec)
        x = torch.zeros((L, L), dtype=torch.float64, device="cuda")
        info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, x0=dev(x0), tol=tol, precision=prec,
                          raise_on_error=False)
        assert info["status"] == binding.EBREAKDOWN, info
        x2, info2 = _solve(plan, inst, prec, tol)
        assert info2["status"] == binding.OK
    plan.close()


def test_error_target_option():
    """fftcg_plan_set_error_target: by default the certified target is the
    residual tolerance; fixed per precision it holds whatever tol is."""
    inst = c2_instance(2)
    xr, rinfo = reference_solve(inst["ghat"], inst["d"], inst["b"], 1, route="fft")
    plan = binding.Plan(512, 1, inst["ghat"])
    banner("error-target")
    x_a, info_a = _solve(plan, inst, binding.FP64, 1e-6)
    assert info_a["status"] == binding.OK and info_a["error_bound"] <= 1e-6
    assert relerr(x_a, xr) <= 1e-6
    plan.set_error_target(binding.FP64, 1e-10)
    plan.set_error_target(binding.MIXED, 1e-8)
    x_b, info_b = _solve(plan, inst, binding.FP64, 1e-6)
    x_c, info_c = _solve(plan, inst, binding.MIXED, 1e-6)
    print(f"tol 1e-6: tau = tol {info_a['iterations']} iterations (error {relerr(x_a, xr):.2e}); "
          f"tau 1e-10 {info_b['iterations']} (error {relerr(x_b, xr):.2e}); "
          f"mixed tau 1e-8 {info_c['iterations']} (error {relerr(x_c, xr):.2e})")
    assert info_b["status"] == binding.OK and info_b["error_bound"] <= 1e-10
    assert relerr(x_b, xr) <= 1e-10
    assert info_b["iterations"] > info_a["iterations"]
    assert info_c["status"] == binding.OK and info_c["error_bound"] <= 1e-8
    assert relerr(x_c, xr) <= 1e-8
    for bad in [(binding.FP64, -1.0), (binding.FP64, 1.0), (2, 1e-8)]:
        with pytest.raises(binding.FftcgError):
            plan.set_error_target(*bad)
    plan.set_error_target(binding.FP64, 0.0)
    x_d, info_d = _solve(plan, inst, binding.FP64, 1e-6)
    assert info_d["iterations"] == info_a["iterations"]
    plan.close()
