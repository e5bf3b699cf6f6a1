"""Pins of the oracle's CG (Sec. 3) and reference solves.

* closed form: periodic grid, uniform d, constant b => x = b / (d + ghat(0,0)),
  reached in one iteration (the constant vector is the k = 0 plane wave);
* dense Cholesky agreement on grids up to 16 x 16, periodic and padded;
* finite termination: periodic L = 4 with uniform d has 5 distinct
  eigenvalues, so CG converges in at most 5 iterations;
* CG invariants: recursive vs true residual, A-norm error monotone, residual
  orthogonality;
* the certified error bound holds against the Cholesky solution;
* the FFT-route reference agrees with the direct-route reference.
"""

import numpy as np
import pytest

from workloads import spectrum, periodic_instance, padded_instance
from oracle import (kernel_table, apply_direct, cg, solve_dense, reference_solve,
                    lambda_lb, error_bound, certified_ok, loadstep_argmax,
                    loadstep_valid)


def test_closed_form_periodic_uniform():
    L, eps, dval, bval = 64, 1e-2, 0.8, 0.37
    gh = spectrum(L, eps)
    g = kernel_table(gh)
    d = np.full((L, L), dval)
    b = np.full((L, L), bval)
    x, info = cg(lambda v: apply_direct(g, d, v, 0), b, tol=1e-13)
    assert gh[0, 0] == pytest.approx(10.0, rel=1e-15)
    np.testing.assert_allclose(x, bval / (dval + 10.0), rtol=1e-14)
    assert info["iterations"] == 1


@pytest.mark.parametrize("L", [2, 4, 8, 16])
@pytest.mark.parametrize("padded", [0, 1])
def test_cholesky_agreement(L, padded):
    if padded:
        inst = padded_instance(L, [80, L], eps=1e-3)
    else:
        inst = periodic_instance(L, [81, L], eps=1e-2)
    g = kernel_table(inst["ghat"])
    xd = solve_dense(g, inst["d"], inst["b"], padded)
    x, info = reference_solve(inst["ghat"], inst["d"], inst["b"], padded, g=g)
    err = np.linalg.norm(x - xd) / np.linalg.norm(xd)
    # CG stops at ||r||/||b|| <= 1e-13, so the error is at most kappa * 1e-13
    # (kappa <= 13.5 here) plus the Cholesky solution's own rounding error.
    assert err <= 2e-12
    assert info["bound"] + 1e-14 >= err


def test_finite_termination_L4():
    L = 4
    gh = spectrum(L, 0.3)
    g = kernel_table(gh)
    d = np.full((L, L), 0.6)
    b = np.random.default_rng(2).uniform(0, 1, (L, L))
    x, info = cg(lambda v: apply_direct(g, d, v, 0), b, tol=0.0, maxit=5)
    xd = solve_dense(g, d, b, 0)
    assert np.linalg.norm(x - xd) <= 1e-13 * np.linalg.norm(xd)
    # at most 5 distinct eigenvalues (up to rounding of ghat)
    vals = np.unique(np.round(gh.ravel(), 12))
    assert len(vals) == 5


def test_cg_invariants():
    L = 16
    inst = padded_instance(L, [82, 0], eps=1e-3)
    g = kernel_table(inst["ghat"])
    mv = lambda v: apply_direct(g, inst["d"], v, 1)  # noqa: E731
    xs = solve_dense(g, inst["d"], inst["b"], 1)
    x, info = cg(mv, inst["b"], tol=1e-12, record=True, x_true=xs, matvec_true=mv)
    hist = info["history"]
    bn = info["bnorm"]
    errA = [h["err_A"] for h in hist]
    assert all(errA[i + 1] <= errA[i] * (1 + 1e-10) + 1e-15 for i in range(len(errA) - 1))
    for k, h in enumerate(hist):
        assert abs(h["rec"] - h["true_res"]) <= 1e-13 * (k + 1) * bn
    rs = info["residuals"]
    for i in range(min(6, len(rs))):
        for j in range(i):
            c = np.sum(rs[i] * rs[j]) / (np.linalg.norm(rs[i]) * np.linalg.norm(rs[j]))
            assert abs(c) < 1e-8


def test_certified_bound_holds():
    L = 12
    inst = padded_instance(L, [83, 0], eps=1e-3)
    g = kernel_table(inst["ghat"])
    xs = solve_dense(g, inst["d"], inst["b"], 1)
    mv = lambda v: apply_direct(g, inst["d"], v, 1)  # noqa: E731
    lam = lambda_lb(inst["ghat"], inst["d"])
    for tol in (1e-2, 1e-4, 1e-6, 1e-8):
        x, _ = cg(mv, inst["b"], tol=tol)
        r = inst["b"] - mv(x)
        rn, xn = np.linalg.norm(r), np.linalg.norm(x)
        err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
        assert err <= error_bound(rn, xn, lam) * (1 + 1e-12)
        if certified_ok(rn, xn, 1e-6, lam):
            assert err <= 1e-6


def test_fft_reference_matches_direct_reference():
    L = 48
    inst = padded_instance(L, [84, 0], eps=1e-3)
    xd, _ = reference_solve(inst["ghat"], inst["d"], inst["b"], 1, route="direct")
    xf, infof = reference_solve(inst["ghat"], inst["d"], inst["b"], 1, route="fft")
    assert np.linalg.norm(xf - xd) / np.linalg.norm(xd) < 1e-12
    assert infof["bound"] < 1e-11


def test_zero_rhs():
    L = 8
    inst = periodic_instance(L, [85, 0])
    g = kernel_table(inst["ghat"])
    x, info = cg(lambda v: apply_direct(g, inst["d"], v, 0), np.zeros((L, L)))
    assert np.all(x == 0) and info["iterations"] == 0


def test_loadstep_rule():
    x = np.array([[1.0, 2.0], [2.0, 0.5]])
    t = np.array([[1.0, 1.0], [1.0, 0.1]])
    d = np.ones((2, 2))
    assert loadstep_argmax(x, t, d) == 3           # 0.5/0.1 = 5
    d[1, 1] = 0
    assert loadstep_argmax(x, t, d) == 1           # tie 2.0 at 1 and 2 -> first
    d[:] = 0
    assert loadstep_argmax(x, t, d) == -1
    d[:] = 1
    assert loadstep_valid(3, x, t, d, 0.0)
    assert not loadstep_valid(1, x, t, d, 0.0)
    assert loadstep_valid(1, x, t, d, 1.0)         # within the error band
