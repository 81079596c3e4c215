"""Pins of the RK34 locally adaptive pseudo-stepping oracle (oracle/rk34.py):
the order conditions of the pair, its fourth-order local error on a nonlinear
residual against the C oracle's RK4 with many substeps, the closed-form
factor on a uniform state (stability polynomial from the Butcher matrix, step
growth and cap of the controller), the step bounds, and convergence of the
dual step with fewer pseudo-steps than fixed-step RK4."""
import numpy as np
import pytest

import oracle
from oracle import pmg, rk34
from paper_2107_14027_amd import inputs

ZETA, NU = 4.0, 1.0 / 1600.0
T_CFG = (1.0 / (2.0 * np.pi)) ** 2 / NU


def test_order_conditions():
    A = rk34.butcher()
    c = A.sum(1)
    b, bh = rk34.B, rk34.BHAT
    for w in (b, bh):
        assert w.sum() == pytest.approx(1.0, abs=1e-15)
        assert w @ c == pytest.approx(0.5, abs=1e-15)
    assert b @ c ** 2 == pytest.approx(1 / 3, abs=1e-15)
    assert b @ (A @ c) == pytest.approx(1 / 6, abs=1e-15)
    # the embedded solution is second order only
    assert abs(bh @ c ** 2 - 1 / 3) > 1e-2 or abs(bh @ (A @ c) - 1 / 6) > 1e-2
    # two-register structure: row i repeats the weights b_j below the sub-diagonal
    for i in range(2, 4):
        assert np.array_equal(A[i, :i - 1], b[:i - 1])


def test_fourth_order_local_error():
    """One step on y1' = -y1^2, y2' = y1 y2 (exact: y1 = 1/(1+t), y2 = y2(0)(1+t)):
    the local error falls 16x per halving of the step.  (The FR residual is only
    Lipschitz -- the Rusanov speed has kinks -- so a smooth system pins the order.)"""
    f = lambda y: np.array([-y[0] ** 2, y[0] * y[1]])
    y0 = np.array([1.0, 0.5])
    errs = []
    for h in (0.1, 0.05, 0.025):
        y, _ = rk34.step(f, y0, np.full(2, h), h, 1e30)
        errs.append(np.linalg.norm(y - np.array([1.0 / (1.0 + h), 0.5 * (1.0 + h)])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 14.0 < r1 < 20.0 and 14.0 < r2 < 20.0, errs


def stability_poly(z):
    A = rk34.butcher()
    c = A.sum(1)
    g = rk34.B @ A @ A @ c
    return 1 + z + z * z / 2 + z ** 3 / 6 + g * z ** 4


@pytest.mark.parametrize("atol,fac", [(1e30, rk34.FAC_MAX), (1e-300, rk34.FAC_MIN)])
def test_uniform_closed_form(atol, fac):
    """At rest (V = 0, so every derivative is exactly zero) except for the
    auxiliary relaxation -q/T: each value follows q -> q R(-h_k / T) with the
    step h_k = clamp(h0 fac^k, h0/3, 3 h0) (the error ratio is pinned to one
    side of the clamp by atol)."""
    p, n, T = 2, (2, 1, 1), 0.05
    q0 = np.linspace(0.01, 0.09, 9)
    U = inputs.uniform(p, n, np.concatenate([[0.9, 0.0, 0.0, 0.0], q0]))
    lv = pmg.Level(p, n, ZETA, NU, T, None)
    h0, K = 1e-3, 150
    V, h = lv.rk34_steps(U, 0.0, np.zeros((U.shape[0], 3, U.shape[2])), None, np.full(U.shape, h0),
                         h0, atol, K)
    hk = [min(max(h0 * fac ** k, h0 / rk34.MULT), h0 * rk34.MULT) for k in range(K)]
    fq = np.prod([stability_poly(-x / T) for x in hk])
    # the residual of a uniform state is zero only to round-off (the derivative
    # of a constant, ~4e-16 in the momentum); over 150 steps that feeds back at
    # ~1e-12 of q, which has decayed to ~2e-3 of its start
    assert np.allclose(V[:, 4:], (q0 * fq)[None, :, None], rtol=1e-10, atol=0)
    assert np.allclose(V[:, :4], U[:, :4], rtol=0, atol=1e-15)
    hend = min(max(h0 * fac ** K, h0 / rk34.MULT), h0 * rk34.MULT)
    assert np.allclose(h[:, 4:], hend, rtol=1e-12)
    if fac > 1:
        # at-rest values (error estimate zero or round-off) grow to the cap too
        assert np.allclose(h[:, :4], h0 * rk34.MULT, rtol=1e-12)


def test_local_dual_step_converges_faster():
    P, n = 3, (2, 2, 2)
    Unm1 = inputs.tgv(P, n, noise=1e-4, seed=2)
    Un = oracle.rk4(P, n, Unm1, ZETA, NU, T_CFG, 2.5e-3, 4)
    G = 2 * Un - Unm1
    dt, dtau, tol = 1e-2, 1e-3, 1.2e-3
    U, it, res, rc, h = pmg.dual_step_local(P, n, G, Un, Unm1, ZETA, NU, T_CFG, dt, dtau, tol, 2000)
    Uo, ito, reso, rco = oracle.dual_step(P, n, G, Un, Unm1, ZETA, NU, T_CFG, dt, dtau, tol, 2000)
    assert rc == 0 and rco == 0 and res < tol
    assert it < ito
    assert np.all(h >= dtau / rk34.MULT * (1 - 1e-12)) and np.all(h <= dtau * rk34.MULT * (1 + 1e-12))
    # the reported norm is that of the returned state
    a, B = pmg.bdf_terms(pmg.Level(P, n, ZETA, NU, T_CFG, None), Un, Unm1, dt)
    Rs = pmg.Level(P, n, ZETA, NU, T_CFG, None).pseudo_residual(U.reshape(-1, 13, 64), a, B, None)
    assert pmg.velocity_rms(Rs) == pytest.approx(res, rel=1e-12)


def test_controller_is_deadbeat_for_an_h3_error(monkeypatch):
    """With the clamps opened, the controller exponent -1/3 matches the
    embedded estimate's h^3 scaling: from any starting step it lands in one
    step on the step whose error is SAFETY^3 atol, which it then keeps (two
    independent scalar equations, since the steps are per value)."""
    monkeypatch.setattr(rk34, "FAC_MIN", 0.0)
    monkeypatch.setattr(rk34, "FAC_MAX", 1e9)
    monkeypatch.setattr(rk34, "MULT", 1e9)
    f = lambda y: np.array([-y[0] ** 2, -y[1] ** 3])
    y0 = np.array([1.0, 0.5])
    atol = 1e-7
    land = []
    for h1 in (2e-3, 8e-3):
        _, h2 = rk34.step(f, y0, np.full(2, h1), h1, atol)
        _, h3 = rk34.step(f, y0, h2, h1, atol)
        land.append(h2)
        assert np.allclose(h3, h2, rtol=0.03)
    assert np.allclose(land[0], land[1], rtol=0.03)
