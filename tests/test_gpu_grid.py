"""The CG update folded into the row-inverse pass behind a grid-wide barrier
(fftcg_plan_set_grid_sync), against the separate update kernel and the
oracle.

Sec. 3 (the update r <- r - alpha q of the CG iteration, Listing 2): the
folded form computes the same alpha from the same p.q partials in the same
order and the same r update; only the r.r partial sums are grouped
differently, so solutions agree to within the solves' tolerance, not bitwise.

* which grids and precisions take it;
* FP64 solves folded and separate against the oracle;
* full-size C3 instance, folded and separate, both against the oracle's
  stored solution samples;
* L = 256 against the oracle's solution run to stagnation;
* the fallback: a barrier that gives up (wait limit forced to zero from the
  host, every workgroup still exits) makes the host repeat the solve with the
  separate kernel; the result is bitwise the separate kernel's, also for a
  warm start given in place (x0 == x);
* the masked operator of the fracture driver (Sec. 2) through the folded
  path at L = 512, breaks replayed by the oracle;
* repeatability, a busy device, and the iteration timing aid;
* the turn pass (the row-inverse pass going on into the next iteration's
  forward row pass, mode 1 where it fits) against the folded update alone
  (mode 3): the same arithmetic in the same order, so bitwise the same.
"""

import json
import os

import numpy as np
import pytest

from paper_1305_3625_amd import binding
from workloads import spectrum, c3_instance, padded_instance, fracture_instance
from oracle import reference_solve, fracture_sequence
from gpu_util import dev, host, relerr, banner

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ON = (binding.GRID_ON, binding.GRID_ON_TURN)  # the folded update, with or without the turn pass


def _solve(plan, inst, mode, x0=None, tol=1e-8):
    import torch
    L = inst["L"]
    plan.set_grid_sync(mode)
    x = torch.zeros((L, L), dtype=torch.float64, device="cuda") if x0 is None else x0
    info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, x0=None if x0 is None else x, tol=tol,
                      precision=binding.MIXED, raise_on_error=False)
    return host(x), info


def test_grid_sync_states():
    L = 2048
    plan = binding.Plan(L, 1, spectrum(2 * L, 1e-4))
    banner("grid-states", L)
    # the turn pass fits in 128 VGPRs: four workgroups per CU, the whole grid
    assert plan.grid_sync(binding.MIXED) == binding.GRID_ON_TURN
    # FP64 at M = 4096: 2 workgroups of the pass per CU, fewer than it has
    assert plan.grid_sync(binding.FP64) in (binding.GRID_UNSUPPORTED,) + ON
    plan.set_grid_sync(0)
    assert plan.grid_sync(binding.MIXED) == binding.GRID_OFF
    plan.set_grid_sync(3)
    assert plan.grid_sync(binding.MIXED) == binding.GRID_ON
    plan.set_grid_sync(1)
    assert plan.grid_sync(binding.MIXED) == binding.GRID_ON_TURN
    for bad in (-1, 4):
        with pytest.raises(binding.FftcgError):
            plan.set_grid_sync(bad)
    plan.close()


@pytest.mark.parametrize("s", [0])
def test_grid_full_size_against_oracle_samples(s):
    with open(os.path.join(GOLD, f"padded_L2048_seed{s}_samples.json")) as fh:
        g = json.load(fh)
    inst = c3_instance(s)
    plan = binding.Plan(2048, 1, inst["ghat"])
    banner("grid-L2048", s)
    pos = np.array(g["pos"])
    xs = {}
    for mode in (1, 0):
        x, info = _solve(plan, inst, mode)
        assert info["status"] == binding.OK and info["error_bound"] <= 1e-8, (mode, info)
        gap = np.max(np.abs(x.ravel()[pos] - np.array(g["x"])))
        print(f"mode {mode}: iters {info['iterations']} bound {info['error_bound']:.3e} "
              f"max sampled gap {gap / g['xnorm']:.3e}")
        assert gap <= (1e-8 + g["bound"]) * g["xnorm"], (mode, gap)
        xs[mode] = (x, info)
        # mode 1 ran folded throughout (no barrier gave up)
        assert plan.grid_sync(binding.MIXED) == (binding.GRID_ON_TURN if mode == 1 else binding.GRID_OFF)
    assert abs(xs[1][1]["iterations"] - xs[0][1]["iterations"]) <= 2
    assert relerr(xs[1][0], xs[0][0]) <= 2e-8
    plan.close()


def test_grid_L256_against_oracle():
    L = 256
    inst = padded_instance(L, [3, 7], eps=1e-4, normal_b=True)
    xr, rinfo = reference_solve(inst["ghat"], inst["d"], inst["b"], 1)
    plan = binding.Plan(L, 1, inst["ghat"])
    banner("grid-L256", L)
    assert plan.grid_sync(binding.MIXED) in ON
    for mode in (1, 0):
        x, info = _solve(plan, inst, mode)
        err = relerr(x, xr)
        print(f"mode {mode}: iters {info['iterations']} error {err:.3e} (oracle bound {rinfo['bound']:.1e})")
        assert info["status"] == binding.OK
        assert err <= 1e-8 + rinfo["bound"]
    plan.close()


@pytest.mark.parametrize("L", [256, 512])
def test_grid_fp64_against_oracle(L):
    """FP64 solves (the periodic and padded FP64 workloads' precision) with
    the folded update and with the separate kernel, against the oracle."""
    import torch
    inst = padded_instance(L, [3, 12, L], eps=1e-3)
    xr, rinfo = reference_solve(inst["ghat"], inst["d"], inst["b"], 1)
    plan = binding.Plan(L, 1, inst["ghat"])
    banner("grid-fp64", L)
    assert plan.grid_sync(binding.FP64) in ON
    for mode in (1, 0):
        plan.set_grid_sync(mode)
        x = torch.zeros((L, L), dtype=torch.float64, device="cuda")
        info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, tol=1e-10, precision=binding.FP64)
        err = relerr(host(x), xr)
        print(f"mode {mode}: iters {info['iterations']} error {err:.3e}")
        assert info["status"] == binding.OK and err <= 1e-10 + rinfo["bound"]
    ms, folded = plan.profile_iteration(dev(inst["d"]), dev(inst["b"]), torch.empty_like(x), reps=8,
                                        precision=binding.FP64)
    assert not folded  # mode 0 was set last
    plan.set_grid_sync(1)
    ms, folded = plan.profile_iteration(dev(inst["d"]), dev(inst["b"]), torch.empty_like(x), reps=8,
                                        precision=binding.FP64)
    assert folded and ms[3] == 0.0 and all(v > 0 for v in ms[:3])
    assert (ms[4] > 0) == (folded == 2)
    plan.close()


def test_grid_fallback_repeats_solve():
    L = 512
    inst = padded_instance(L, [3, 8], eps=1e-4, normal_b=True)
    plan = binding.Plan(L, 1, inst["ghat"])
    banner("grid-fallback", L)
    x0, info0 = _solve(plan, inst, 0)
    x2, info2 = _solve(plan, inst, 2)
    assert info2["status"] == binding.OK
    assert plan.grid_sync(binding.MIXED) == binding.GRID_FELL_BACK
    # the repeated solve is the separate kernel's, bitwise
    assert np.array_equal(x2, x0) and info2["iterations"] == info0["iterations"]
    # setting a mode again takes the folded path up again
    plan.set_grid_sync(1)
    assert plan.grid_sync(binding.MIXED) in ON
    x1, info1 = _solve(plan, inst, 1)
    assert info1["status"] == binding.OK and relerr(x1, x0) <= 2e-8
    plan.close()


def test_grid_fallback_warm_start_in_place():
    """x0 == x: the abandoned attempt overwrote x, the repeat starts from
    the caller's x0 again (kept aside while the folded path runs)."""
    import torch
    L = 512
    inst = padded_instance(L, [3, 9], eps=1e-4, normal_b=True)
    rng = np.random.default_rng([3, 9, 1])
    w = rng.standard_normal((L, L)) * 0.1
    plan = binding.Plan(L, 1, inst["ghat"])
    banner("grid-fallback-in-place", L)
    xa = dev(w)
    xa_h, info_a = _solve(plan, inst, 0, x0=xa)
    xb = dev(w)
    xb_h, info_b = _solve(plan, inst, 2, x0=xb)
    assert info_a["status"] == binding.OK and info_b["status"] == binding.OK
    assert plan.grid_sync(binding.MIXED) == binding.GRID_FELL_BACK
    assert np.array_equal(xa_h, xb_h) and info_a["iterations"] == info_b["iterations"]
    torch.cuda.synchronize()
    plan.close()


def test_grid_fracture_masked_L512():
    """The fracture driver's projected (masked) operator through the folded
    update, plain CG in mixed precision; every break is a valid choice for
    the oracle's replay and the forces match."""
    import torch
    L, steps, tol = 512, 6, 1e-8
    inst = fracture_instance(0, L=L)
    gh = spectrum(2 * L, 1e-3)
    plan = binding.Plan(L, 1, gh)
    assert plan.grid_sync(binding.MIXED) in ON
    f = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    banner("grid-fracture-L512", steps)
    st, broken, dbreak, iters = plan.fracture(inst["k"], dev(inst["t"]), f, steps, tol=tol,
                                              precision=binding.MIXED)
    assert st == binding.OK
    assert plan.grid_sync(binding.MIXED) in ON
    _, fo_dbreak, fo_f, ratios = fracture_sequence(gh, inst["k"], inst["t"], steps, 1, replay=broken)
    t = inst["t"].ravel()
    for s in range(steps):
        rho = ratios[s].ravel()
        k = int(np.argmax(rho))
        j = int(broken[s])
        assert np.isfinite(rho[j]), (s, j)
        einf = 2 * tol * np.linalg.norm(np.where(np.isfinite(rho), rho * t, 0.0))
        assert rho[j] >= rho[k] - einf * (1.0 / t[j] + 1.0 / t[k]), (s, j, k)
    np.testing.assert_allclose(dbreak, fo_dbreak, rtol=50 * tol)
    err = relerr(host(f), fo_f)
    print(f"mean iters {iters.mean():.1f}, force error {err:.3e}")
    assert err <= 10 * tol
    plan.close()


def test_grid_repeatable():
    """Two folded solves of the same system agree bitwise (alpha and the
    r.r partials are summed in a fixed order; the barrier adds no order)."""
    L = 1024
    inst = padded_instance(L, [3, 10], eps=1e-4, normal_b=True)
    plan = binding.Plan(L, 1, inst["ghat"])
    banner("grid-repeatable", L)
    xa, ia = _solve(plan, inst, 1)
    xb, ib = _solve(plan, inst, 1)
    assert ia["status"] == binding.OK and ib["status"] == binding.OK
    assert plan.grid_sync(binding.MIXED) in ON
    assert np.array_equal(xa, xb) and ia["iterations"] == ib["iterations"]
    plan.close()


def test_grid_with_other_stream_busy():
    """A solve while another stream keeps the device busy (FP32 matrix
    products, about 0.2 s): whether the barrier completes or gives up and
    the solve is repeated with the separate kernel, the result is the
    separate kernel's to within the tolerance."""
    import torch
    L = 2048
    inst = c3_instance(1)
    plan = binding.Plan(L, 1, inst["ghat"])
    banner("grid-busy-device", L)
    x0, i0 = _solve(plan, inst, 0)
    plan.set_grid_sync(1)
    a = torch.randn(8192, 8192, device="cuda")
    bm = torch.randn(8192, 8192, device="cuda")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for _ in range(20):
            c = torch.mm(a, bm)
    x = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, tol=1e-8, precision=binding.MIXED, raise_on_error=False)
    torch.cuda.synchronize()
    state = plan.grid_sync(binding.MIXED)
    print(f"state {state}, iters {info['iterations']} (separate {i0['iterations']}), "
          f"bound {info['error_bound']:.3e}, checksum {float(c[0, 0]):.3e}")
    assert info["status"] == binding.OK and info["error_bound"] <= 1e-8
    assert state in ON + (binding.GRID_FELL_BACK,)
    assert relerr(host(x), x0) <= 2e-8
    plan.close()


@pytest.mark.parametrize("L", [256, 2048])
def test_profile_iteration(L):
    """The iteration timing aid: positive pass times, the folded update
    reported as such (no separate update pass), the separate kernel timed
    when the plan uses it; b = 0 stops at once and is refused."""
    import torch
    inst = padded_instance(L, [3, 11], eps=1e-4, normal_b=True)
    plan = binding.Plan(L, 1, inst["ghat"])
    banner("profile-iteration", L)
    d, b = dev(inst["d"]), dev(inst["b"])
    x = torch.empty((L, L), dtype=torch.float64, device="cuda")
    ms, folded = plan.profile_iteration(d, b, x, reps=40)
    print(f"folded: {folded}, ms {[round(v, 4) for v in ms]}")
    assert folded and all(v > 0 for v in ms[:3]) and ms[3] == 0.0
    assert (folded == 2) == (plan.grid_sync(binding.MIXED) == binding.GRID_ON_TURN) == (ms[4] > 0)
    if folded == 2:
        with pytest.raises(binding.FftcgError):  # the turn pass needs two iterations
            plan.profile_iteration(d, b, x, reps=1)
    plan.set_grid_sync(3)
    ms3, folded3 = plan.profile_iteration(d, b, x, reps=40)
    print(f"folded, no turn: ms {[round(v, 4) for v in ms3]}")
    assert folded3 == 1 and all(v > 0 for v in ms3[:3]) and ms3[3] == 0.0 and ms3[4] == 0.0
    plan.set_grid_sync(0)
    ms0, folded0 = plan.profile_iteration(d, b, x, reps=40)
    print(f"separate: ms {[round(v, 4) for v in ms0]}")
    assert not folded0 and all(v > 0 for v in ms0[:4]) and ms0[4] == 0.0
    ms64, _ = plan.profile_iteration(d, b, x, reps=4, precision=binding.FP64)
    assert all(v > 0 for v in ms64[:4])
    with pytest.raises(binding.FftcgError):
        plan.profile_iteration(d, torch.zeros_like(b), x, reps=4)
    with pytest.raises(binding.FftcgError):
        plan.profile_iteration(d, b, x, reps=0)
    plan.close()


def test_grid_two_solves_concurrently():
    """Two host threads solve with one plan at once, each on its own stream
    (two workspaces): two folded row-inverse passes may then compete for
    the device.  Whether their barriers complete or give up (the solve then
    repeats with the separate kernel), both results match the separate
    kernel's to within the tolerance."""
    import threading
    import torch
    L = 2048
    insts = [c3_instance(s) for s in (0, 1)]
    plan = binding.Plan(L, 1, insts[0]["ghat"])
    banner("grid-two-streams", L)
    ref = [_solve(plan, inst, 0)[0] for inst in insts]
    plan.set_grid_sync(1)
    D = [dev(i["d"]) for i in insts]
    B = [dev(i["b"]) for i in insts]
    X = [torch.zeros((L, L), dtype=torch.float64, device="cuda") for _ in insts]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    infos = [None, None]
    torch.cuda.synchronize()

    def run(k):
        infos[k] = plan.solve(D[k], B[k], X[k], tol=1e-8, precision=binding.MIXED, stream=streams[k],
                              raise_on_error=False)

    th = [threading.Thread(target=run, args=(k,)) for k in (0, 1)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    state = plan.grid_sync(binding.MIXED)
    print(f"state {state}, iters {[i['iterations'] for i in infos]}")
    assert state in ON + (binding.GRID_FELL_BACK,)
    for k in (0, 1):
        assert infos[k]["status"] == binding.OK and infos[k]["error_bound"] <= 1e-8
        assert relerr(host(X[k]), ref[k]) <= 2e-8
    plan.close()


@pytest.mark.parametrize("L,precision,tol", [(2048, binding.MIXED, 1e-8), (256, binding.MIXED, 1e-8),
                                             (512, binding.FP64, 1e-10)])
def test_turn_pass_bitwise_as_folded(L, precision, tol):
    """Mode 1 (the turn pass, where it fits) against mode 3 (the folded
    update and the forward row pass as separate launches): beta from the
    same r.r partials in the same order, p <- r + beta p and the x update
    with the same operations, so the solutions, iteration counts and error
    bounds are bitwise equal."""
    import torch
    inst = c3_instance(0) if L == 2048 else padded_instance(L, [3, 13, L], eps=1e-4, normal_b=True)
    plan = binding.Plan(L, 1, inst["ghat"])
    banner("turn-vs-folded", L, precision)
    out = {}
    for mode in (3, 1):
        plan.set_grid_sync(mode)
        state = plan.grid_sync(precision)
        x = torch.zeros((L, L), dtype=torch.float64, device="cuda")
        info = plan.solve(dev(inst["d"]), dev(inst["b"]), x, tol=tol, precision=precision)
        out[mode] = (host(x), info, state)
        print(f"mode {mode}: state {state} iters {info['iterations']} bound {info['error_bound']:.3e}")
    assert out[3][2] == binding.GRID_ON
    if L == 2048:
        assert out[1][2] == binding.GRID_ON_TURN
    assert out[1][2] in ON
    assert out[1][1]["iterations"] == out[3][1]["iterations"]
    assert out[1][1]["error_bound"] == out[3][1]["error_bound"]
    assert np.array_equal(out[1][0], out[3][0])
    plan.close()
