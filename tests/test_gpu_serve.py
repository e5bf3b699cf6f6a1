"""The continuous-batching server on the GPU.

* every request's x is bitwise the same alone and in a mix of sizes, and
  within 1e-8 of the oracle;
* admission under a tight memory budget (requests wait for slots) and the
  error paths: ENOMEM, EAGAIN, ENOTFOUND;
* a request that fails (maxit reached) retires alone while the others in its
  batch are unchanged;
* a load-stepped sequence: each broken index is a valid choice for the
  oracle's solution of that step (near-ties admit several answers), the
  oracle replays the GPU's choices, and the final x matches it.
"""

import time

import numpy as np
import pytest

from paper_1305_3625_amd import binding
from workloads import spectrum, padded_instance, c4_request, c5_sequence
from oracle import (kernel_table, reference_solve, apply_direct, loadstep_argmax, loadstep_valid,
                    lambda_lb)
from gpu_util import banner, relerr

pytestmark = pytest.mark.gpu

EPS = 1e-3


def _wait(srv, tickets, L, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for tk in tickets:
            if tk in out:
                continue
            r = srv.poll(tk, L[tk] if isinstance(L, dict) else L)
            if r.status != binding.PENDING:
                out[tk] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(tickets) - len(out)} requests still pending")
        time.sleep(0.001)
    return out


@pytest.fixture(scope="module")
def plans():
    return {M: binding.Plan(M // 2, 1, spectrum(M, EPS)) for M in (32, 64, 128, 256, 512)}


def test_alone_equals_mix(plans):
    banner("serve-alone-vs-mix")
    # M <= 256: fused classes (one workgroup per slot); M = 512: multi-pass
    reqs = [c4_request(k, M) for k, M in enumerate([64, 128, 64, 256, 32, 128, 512, 64, 256, 512])]
    srv = binding.Server(memory_budget=1 << 30)
    alone = []
    for r in reqs:
        st, tk = srv.submit(plans[r["M"]], r["d"], r["b"], tol=1e-8)
        assert st == binding.OK
        res = _wait(srv, [tk], r["L"])[tk]
        assert res.status == binding.OK, res.info
        alone.append(res.x)
    # all at once, twice (the second batch sees slots reused)
    for _ in range(2):
        tks = []
        Ls = {}
        for r in reqs:
            st, tk = srv.submit(plans[r["M"]], r["d"], r["b"], tol=1e-8)
            assert st == binding.OK
            tks.append(tk)
            Ls[tk] = r["L"]
        res = _wait(srv, tks, Ls)
        for r, tk, xa in zip(reqs, tks, alone):
            assert res[tk].status == binding.OK
            assert np.array_equal(res[tk].x, xa)
    stats = srv.stats()
    assert stats["completed"] == 3 * len(reqs) and stats["failed"] == 0
    # every ticket reported as completed exactly once
    seen = srv.completed(cap=7) + srv.completed(cap=100)
    assert len(seen) == 3 * len(reqs) and len(set(seen)) == len(seen)
    assert set(tks) <= set(seen)
    assert srv.completed() == []
    srv.close()
    # accuracy against the oracle
    for r, xa in zip(reqs[:4], alone[:4]):
        xr, info = reference_solve(spectrum(r["M"], EPS), r["d"], r["b"], 1)
        assert relerr(xa, xr) <= 1e-8


def test_tight_budget_admission(plans):
    banner("serve-tight-budget")
    probe = binding.Server(memory_budget=1 << 30)
    r = c4_request(100, 256)
    st, tk = probe.submit(plans[256], r["d"], r["b"])
    _wait(probe, [tk], 128)
    one = probe.stats()["bytes_in_use"]
    probe.close()
    assert one > 0
    srv = binding.Server(memory_budget=int(2.5 * one))
    reqs = [c4_request(200 + k, 256) for k in range(6)]
    tks = []
    for r in reqs:
        st, tk = srv.submit(plans[256], r["d"], r["b"])
        assert st == binding.OK
        tks.append(tk)
    peak = 0
    t0 = time.time()
    done = {}
    while len(done) < len(tks) and time.time() - t0 < 120:
        peak = max(peak, srv.stats()["in_flight"])
        assert srv.stats()["bytes_in_use"] <= int(2.5 * one)
        for tk in tks:
            if tk not in done:
                res = srv.poll(tk, 128)
                if res.status != binding.PENDING:
                    done[tk] = res
        time.sleep(0.0005)
    assert len(done) == len(tks)
    assert all(v.status == binding.OK for v in done.values())
    assert peak <= 2
    srv.close()


def test_pageable_inputs(plans):
    """Past the pinned-staging cap (a quarter of the budget, at least 1 MiB)
    queued inputs wait in pageable memory and reach the device through the
    slot's staging buffer: results bitwise equal to pinned submissions."""
    banner("serve-pageable")
    reqs = [c4_request(400 + k, 128) for k in range(20)]  # 64 KiB of inputs each
    ref = binding.Server(memory_budget=1 << 30)
    want = []
    for r in reqs:
        st, tk = ref.submit(plans[128], r["d"], r["b"], tol=1e-8)
        assert st == binding.OK
        want.append(_wait(ref, [tk], 64)[tk].x)
    ref.close()
    srv = binding.Server(memory_budget=4 << 20, max_slots=2)
    tks = []
    for r in reqs:
        st, tk = srv.submit(plans[128], r["d"], r["b"], tol=1e-8)
        assert st == binding.OK
        tks.append(tk)
    res = _wait(srv, tks, 64)
    for tk, w in zip(tks, want):
        assert res[tk].status == binding.OK
        assert np.array_equal(res[tk].x, w)
    srv.close()


def test_error_paths(plans):
    banner("serve-errors")
    r = c4_request(300, 256)
    srv = binding.Server(memory_budget=1 << 20)   # less than one slot of M=256
    st, _ = srv.submit(plans[256], r["d"], r["b"])
    assert st == binding.ENOMEM
    bad = r["b"].copy()
    bad[0, 0] = np.nan
    st, _ = srv.submit(plans[32], np.ones((16, 16)), bad[:16, :16])
    assert st == binding.EINVAL
    res = srv.poll(123456, 16)
    assert res.status == binding.ENOTFOUND
    srv.close()
    # queue cap: with one slot and a queue of one, a burst gets EAGAIN
    srv = binding.Server(memory_budget=1 << 30, max_slots=1, queue_cap=1)
    r = c4_request(301, 256)
    sts, tks = [], []
    for _ in range(40):
        st, tk = srv.submit(plans[256], r["d"], r["b"])
        sts.append(st)
        if st == binding.OK:
            tks.append(tk)
    assert binding.EAGAIN in sts
    res = _wait(srv, tks, 128)
    assert all(v.status == binding.OK for v in res.values())
    tk = tks[0]
    assert srv.poll(tk, 128).status == binding.ENOTFOUND
    srv.close()


def test_failed_request_is_isolated(plans):
    banner("serve-isolation")
    reqs = [c4_request(400 + k, 128) for k in range(4)]
    srv = binding.Server(memory_budget=1 << 30)
    alone = []
    for r in reqs:
        st, tk = srv.submit(plans[128], r["d"], r["b"])
        alone.append(_wait(srv, [tk], 64)[tk].x)
    tks = []
    for i, r in enumerate(reqs):
        st, tk = srv.submit(plans[128], r["d"], r["b"], maxit=(2 if i == 1 else 10000))
        tks.append(tk)
    res = _wait(srv, tks, 64)
    assert res[tks[1]].status == binding.ENOCONV
    assert res[tks[1]].info["iterations"] == 2
    for i in (0, 2, 3):
        assert res[tks[i]].status == binding.OK
        assert np.array_equal(res[tks[i]].x, alone[i])
    srv.close()


def test_loadstep_sequence_replay():
    L, steps = 32, 24
    M = 2 * L
    seq = c5_sequence(7, L=L)
    gh = spectrum(M, EPS)
    g = kernel_table(gh)
    plan = binding.Plan(L, 1, gh)
    srv = binding.Server(memory_budget=1 << 30)
    banner("serve-sequence", L, steps)
    st, tk = srv.submit_sequence(plan, seq["d"], seq["b"], seq["t"], steps, tol=1e-8)
    assert st == binding.OK
    t0 = time.time()
    while True:
        r = srv.poll_sequence(tk, L, steps, bounds=True)
        if r.status != binding.PENDING:
            break
        assert time.time() - t0 < 120
        time.sleep(0.002)
    assert r.status == binding.OK, r.info
    x_gpu, broken, iters, step_bounds = r.x
    # every step's solve was certified to the target
    assert np.all(step_bounds > 0.0) and np.all(step_bounds <= 1e-8)
    assert len(set(broken.tolist())) == steps and np.all(broken >= 0)
    # replay: the oracle solves each step with the GPU's sequence of breaks
    d = seq["d"].copy()
    x_ref = None
    for s in range(steps):
        x_ref, info = reference_solve(gh, d, seq["b"], 1, g=g)
        # the GPU's solution of this step has certified error <= 1e-8 (relative,
        # 2-norm), which bounds its max-norm error
        e_inf = 1e-8 * np.linalg.norm(x_ref) / (1 - 1e-8) + info["bound"] * np.linalg.norm(x_ref)
        j = int(broken[s])
        assert loadstep_valid(j, x_ref, seq["t"], d, e_inf), (s, j, loadstep_argmax(x_ref, seq["t"], d))
        d.ravel()[j] = 0.0
    # the returned x is the last step's solution (before its own break)
    assert relerr(x_gpu, x_ref) <= 1e-8
    srv.close()


@pytest.mark.parametrize("M", [128, 512])   # a fused class and a multi-pass class
def test_refresh_period_option(plans, M):
    """The server's refresh_period sets the mixed solves' FP64 check period:
    a short period adds checks, and the results stay within 1e-8 of the
    oracle either way."""
    banner("serve-refresh-period", M)
    r = c4_request(600 + M, M)
    xr, _ = reference_solve(spectrum(M, EPS), r["d"], r["b"], 1, route="fft")
    checks = {}
    for period in (0, 4):
        srv = binding.Server(memory_budget=1 << 30, refresh_period=period)
        st, tk = srv.submit(plans[M], r["d"], r["b"], tol=1e-8)
        assert st == binding.OK
        res = _wait(srv, [tk], r["L"])[tk]
        srv.close()
        assert res.status == binding.OK, res.info
        assert relerr(res.x, xr) <= 1e-8
        checks[period] = res.info["checks"]
        # with a period of 4 no two checks are more than 4 iterations apart
        if period == 4:
            assert res.info["checks"] >= res.info["iterations"] // 4
    print(f"M {M}: checks with the default period {checks[0]}, with period 4 {checks[4]}")
    assert checks[4] > checks[0]


def test_shutdown_cancels_unfinished(plans):
    """fftcg_server_shutdown: a finished request stays pollable with its
    result; requests running (they cannot converge: tol 1e-300) and queued
    end ECANCELED, the running ones with the iterations they ran; they are
    counted; later submissions are refused with ECANCELED; the plan is free
    again."""
    banner("serve-shutdown")
    srv = binding.Server(memory_budget=1 << 30, max_slots=4)
    r0 = c4_request(700, 512)
    st, tk0 = srv.submit(plans[512], r0["d"], r0["b"], tol=1e-8)
    assert st == binding.OK
    t0 = time.time()
    while srv.stats()["completed"] < 1:
        assert time.time() - t0 < 60
        time.sleep(0.001)
    reqs = [c4_request(701 + k, 512) for k in range(8)]
    tks = []
    for r in reqs:
        st, tk = srv.submit(plans[512], r["d"], r["b"], tol=1e-300, maxit=10 ** 8)
        assert st == binding.OK
        tks.append(tk)
    t0 = time.time()
    while srv.stats()["in_flight"] < 4:
        assert time.time() - t0 < 60
        time.sleep(0.001)
    time.sleep(0.05)
    srv.shutdown()
    srv.shutdown()  # a second call does nothing
    st, _ = srv.submit(plans[512], r0["d"], r0["b"])
    assert st == binding.ECANCELED
    first = srv.poll(tk0, 256)
    assert first.status == binding.OK
    xr, _ = reference_solve(spectrum(512, EPS), r0["d"], r0["b"], 1, route="fft")
    assert relerr(first.x, xr) <= 1e-8
    res = [srv.poll(tk, 256) for tk in tks]
    assert all(v.status == binding.ECANCELED for v in res)
    ran = [v.info["iterations"] for v in res]
    assert sum(1 for k in ran if k > 0) == 4   # the four that held slots had run
    stats = srv.stats()
    assert stats["canceled"] == 8 and stats["completed"] == 1
    assert stats["in_flight"] == 0 and stats["queued"] == 0 and stats["bytes_in_use"] == 0
    srv.close()
    # no request holds the plan any more
    plans[512].set_precond(binding.PRECOND_NONE)


def test_graph_replay_equals_direct_launches(plans):
    """Multi-pass chunks replayed from captured HIP graphs give bitwise the
    same solutions, iteration and check counts as the same chunks launched
    kernel by kernel, over several rounds of a changing mix (graph shapes
    are reused across rounds with different slot contents)."""
    banner("serve-graphs")
    p1024 = binding.Plan(512, 1, spectrum(1024, EPS))
    pl = {**plans, 1024: p1024}
    reqs = [c4_request(800 + k, M) for k, M in enumerate([256, 512, 1024, 512, 256, 1024, 512, 256])]
    out = {}
    for graphs in (False, True):
        srv = binding.Server(memory_budget=2 << 30, graphs=graphs)
        res = []
        for rnd in range(3):
            batch = reqs[rnd:] + reqs[:rnd]  # a different order, so slots hold different requests
            tks = []
            Ls = {}
            for r in batch:
                st, tk = srv.submit(pl[r["M"]], r["d"], r["b"], tol=1e-8)
                assert st == binding.OK
                tks.append(tk)
                Ls[tk] = r["L"]
            got = _wait(srv, tks, Ls)
            for r, tk in zip(batch, tks):
                assert got[tk].status == binding.OK, got[tk].info
                res.append((id(r), got[tk].x, got[tk].info["iterations"], got[tk].info["checks"]))
        srv.close()
        out[graphs] = res
    for (ia, xa, ita, ca), (ib, xb, itb, cb) in zip(out[False], out[True]):
        assert ia == ib and ita == itb and ca == cb
        assert np.array_equal(xa, xb)
    p1024.close()


def test_reserve_then_serve():
    """Capacity reservation: the reserved slots and pinned buffers exist
    before any request (device bytes in use), requests of the reserved
    classes give bitwise the results of a server without reservation, the
    plan cannot be destroyed while the server holds it, and limits are
    checked."""
    banner("serve-reserve")
    p512 = binding.Plan(256, 1, spectrum(512, EPS))
    p1024 = binding.Plan(512, 1, spectrum(1024, EPS))
    pl = {512: p512, 1024: p1024}
    reqs = [c4_request(900 + k, M) for k, M in enumerate([512, 1024, 512, 1024, 512, 512])]
    out = {}
    for reserve in (False, True):
        srv = binding.Server(memory_budget=2 << 30, max_slots=16)
        if reserve:
            assert srv.class_slots(p512) == 0
            srv.reserve(p512, 4)
            srv.reserve(p1024, 2)
            assert srv.class_slots(p512) == 4 and srv.class_slots(p1024) == 2
            assert srv.class_slots(p512, binding.FP64) == 0
            used = srv.stats()["bytes_in_use"]
            assert used > 0
            srv.reserve(p1024, 1)  # never shrinks
            assert srv.stats()["bytes_in_use"] == used
            with pytest.raises(binding.FftcgError):
                srv.reserve(p512, 17)  # above max_slots
            with pytest.raises(binding.FftcgError):
                p1024.close()  # the server holds the plan
        tks, Ls = [], {}
        for r in reqs:
            st, tk = srv.submit(pl[r["M"]], r["d"], r["b"], tol=1e-8)
            assert st == binding.OK
            tks.append(tk)
            Ls[tk] = r["L"]
        got = _wait(srv, tks, Ls)
        out[reserve] = [(got[tk].x, got[tk].info["iterations"]) for tk in tks]
        assert all(got[tk].status == binding.OK for tk in tks)
        srv.close()
    for (xa, ia), (xb, ib) in zip(out[False], out[True]):
        assert ia == ib and np.array_equal(xa, xb)
    p512.close()
    p1024.close()  # released with the server
