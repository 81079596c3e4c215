"""Pins of the oracle's time integration: classical RK4 (closed form on the
linear auxiliary relaxation mode, fourth-order convergence on a nonlinear
state), BDF dual time stepping (Sec. 5; closed-form pseudo-iteration on a
uniform state) and polynomial extrapolation (exact on quadratics)."""
import math

import numpy as np
import pytest

import oracle
from paper_2107_14027_amd import inputs

ZETA, NU = 4.0, 1.0 / 1600.0


def taylor4(z):
    return 1 - z + z * z / 2 - z ** 3 / 6 + z ** 4 / 24


def uniform_mode(p, n, P0, V0, q0):
    vals = np.concatenate([[P0], V0, q0])
    return inputs.uniform(p, n, vals)


@pytest.mark.parametrize("T,dt,steps", [(5e-3, 1e-3, 7), (40.528, 1e-3, 10)])
def test_rk4_linear_relaxation_closed_form(T, dt, steps):
    """Uniform state: only the aux source -q/T acts, so RK4 multiplies q by the
    degree-4 Taylor polynomial of exp(-dt/T) every step; P and V stay fixed."""
    p, n = 2, (2, 2, 2)
    rng = np.random.default_rng(0)
    q0 = rng.standard_normal(9)
    U = uniform_mode(p, n, 0.7, [0.2, -0.1, 0.4], q0)
    U1 = oracle.rk4(p, n, U, ZETA, NU, T, dt, steps)
    expect = q0 * taylor4(dt / T) ** steps
    assert np.allclose(U1[:, 4:], expect[None, :, None], rtol=1e-13, atol=1e-15)
    assert np.allclose(U1[:, :4], U[:, :4], rtol=0, atol=1e-14)


def test_rk4_fourth_order_on_nonlinear_state():
    p, n, T = 2, (2, 2, 2), 0.5
    U0 = inputs.tgv(p, n, noise=0.02, seed=3)
    tend = 0.08
    sols = [oracle.rk4(p, n, U0, ZETA, NU, T, tend / k, k) for k in (2, 4, 8, 16)]
    e = [np.max(np.abs(sols[i] - sols[-1])) for i in range(3)]
    rate = math.log2(e[0] / e[1])  # between dt and dt/2, against the finest solution
    assert rate > 3.6, (e, rate)


@pytest.mark.parametrize("order", [1, 2])
def test_dual_step_uniform_closed_form(order):
    """Uniform state: R(U) = source only, so each pseudo-step maps
    V - V* -> (V - V*) taylor4(c dtau/dt) with V* the BDF solution and
    c = 3/2 (BDF2) or 1 (BDF1); q -> q taylor4(dtau/T)."""
    p, n, T = 1, (2, 1, 2), 40.528
    dt, dtau, tol = 1e-2, 1e-3, 1e-6
    Vn, Vm1 = np.array([0.3, -0.2, 0.1]), np.array([0.28, -0.25, 0.12])
    q0 = np.full(9, 0.05)
    Un = uniform_mode(p, n, 0.9, Vn, q0)
    Um1 = uniform_mode(p, n, 0.9, Vm1, q0)
    G = uniform_mode(p, n, 0.9, 2 * Vn - Vm1, q0)
    U, it, res, rc = oracle.dual_step(p, n, G, Un, Um1, ZETA, NU, T, dt, dtau, tol, 500,
                                      order=order)
    assert rc == 0
    if order == 2:
        Vs, c = (4 * Vn - Vm1) / 3, 1.5
    else:
        Vs, c = Vn, 1.0
    rho = taylor4(c * dtau / dt)
    err0 = (2 * Vn - Vm1) - Vs
    # first k with rms(c/dt * err0 * rho^k) < tol
    k = 0
    while c / dt * math.sqrt(np.mean((err0 * rho ** k) ** 2)) >= tol:
        k += 1
    assert it == k
    assert np.allclose(U[:, 1:4], (Vs + err0 * rho ** k)[None, :, None], rtol=0, atol=1e-14)
    assert np.allclose(U[:, 4:], q0[0] * taylor4(dtau / T) ** k, rtol=1e-12)
    assert abs(res - c / dt * math.sqrt(np.mean((err0 * rho ** k) ** 2))) < 1e-12


def test_dual_step_failure_codes():
    p, n, T = 1, (2, 2, 1), 40.528
    Un = inputs.tgv(p, n)
    U, it, res, rc = oracle.dual_step(p, n, Un * 1.01, Un, Un, ZETA, NU, T, 1e-2, 1e-3, 1e-12, 3)
    assert rc == -5 and it == 3
    bad = Un.copy()
    bad[0, 1, 0] = np.nan
    U, it, res, rc = oracle.dual_step(p, n, bad, Un, Un, ZETA, NU, T, 1e-2, 1e-3, 1e-6, 3)
    assert rc == -4


def test_extrapolation_exact_on_polynomials_in_time():
    rng = np.random.default_rng(5)
    a, b, c = rng.standard_normal((3, 50))
    f = lambda t: a + b * t + c * t * t
    g = lambda t: a + b * t
    assert np.allclose(oracle.extrap(f(2.0), f(1.0), f(0.0), 2), f(3.0), atol=1e-13)
    assert np.allclose(oracle.extrap(g(2.0), g(1.0), None, 1), g(3.0), atol=1e-13)
    assert not np.allclose(oracle.extrap(f(2.0), f(1.0), None, 1), f(3.0), atol=1e-3)


def test_extrapolation_keeping_the_pressure():
    """keep_p: the pressure of every point is U^n's exactly; every other
    variable is the plain extrapolation (exact on quadratics in time)."""
    rng = np.random.default_rng(8)
    ne, ns = 3, 8
    a, b, c = (rng.standard_normal((ne, 13, ns)) for _ in range(3))
    f = lambda t: a + b * t + c * t * t
    G = oracle.extrap(f(2.0), f(1.0), f(0.0), 2, keep_p=True, ns=ns).reshape(ne, 13, ns)
    assert np.array_equal(G[:, 0], f(2.0)[:, 0])
    assert np.allclose(G[:, 1:], f(3.0)[:, 1:], rtol=0, atol=1e-12)
    G1 = oracle.extrap(f(2.0), f(1.0), None, 1, keep_p=True, ns=ns).reshape(ne, 13, ns)
    assert np.array_equal(G1[:, 0], f(2.0)[:, 0])
    assert np.allclose(G1[:, 1:], (2 * f(2.0) - f(1.0))[:, 1:], rtol=0, atol=1e-12)
