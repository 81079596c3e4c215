"""Pins of the P-multigrid oracle (oracle/pmg.py) against what the mathematics
fixes: projection and interpolation exactness of the transfer operators, the
closed-form factor of a whole cycle on uniform states (checks the per-level
pseudo-step growth, the step counts and the direction of the coarse
correction), the FAS fixed point (checks the sign of the coarse defect), and
the reduction to the C oracle's RK4 dual step when the coarse levels take no
steps."""
import numpy as np
import pytest

import oracle
from oracle import pmg
from paper_2107_14027_amd import inputs

ZETA, NU = 4.0, 1.0 / 1600.0
T_CFG = (1.0 / (2.0 * np.pi)) ** 2 / NU


def taylor4(z):
    return 1 - z + z * z / 2 - z ** 3 / 6 + z ** 4 / 24


def test_default_cycle_matches_paper():
    assert pmg.default_cycle(4) == [(4, 1), (3, 1), (2, 1), (1, 4), (2, 1), (3, 1), (4, 7)]
    assert pmg.default_cycle(2) == [(2, 1), (1, 4), (2, 7)]
    with pytest.raises(ValueError):
        pmg.check_cycle(3, [(3, 1), (1, 4), (3, 7)])
    with pytest.raises(ValueError):
        pmg.check_cycle(3, [(3, 1), (2, 1)])


@pytest.mark.parametrize("ph", [2, 3, 4, 5, 6])
def test_transfer_operators(ph):
    pl = ph - 1
    I, Pm = pmg.operators_1d(ph, pl)
    xh, wh = oracle.gauss_legendre(ph + 1)
    xl, _ = oracle.gauss_legendre(pl + 1)
    rng = np.random.default_rng(ph)
    # exact on polynomials of degree <= pl: both directions
    c = rng.standard_normal(pl + 1)
    f = lambda x: np.polynomial.polynomial.polyval(x, c)
    assert np.allclose(I @ f(xh), f(xl), atol=1e-13)
    assert np.allclose(Pm @ f(xl), f(xh), atol=1e-13)
    assert np.allclose(I @ Pm, np.eye(pl + 1), atol=1e-13)
    # the degree-ph Legendre polynomial is orthogonal to everything coarser
    e = np.zeros(ph + 1)
    e[ph] = 1.0
    assert np.allclose(I @ np.polynomial.legendre.legval(xh, e), 0.0, atol=1e-13)
    # L2 projection: the fine-quadrature residual is orthogonal to degree pl
    g = rng.standard_normal(ph + 1)
    r = g - Pm @ (I @ g)
    for k in range(pl + 1):
        assert abs(np.sum(wh * r * xh ** k)) < 1e-13
    # 3D: tensor product exact on a trivariate polynomial of degree pl per direction
    C = rng.standard_normal((pl + 1, pl + 1, pl + 1))

    def nodal(x):
        m = len(x)
        V = np.zeros((m, m, m))
        for k in range(m):
            for j in range(m):
                for i in range(m):
                    V[k, j, i] = np.polynomial.polynomial.polyval3d(x[i], x[j], x[k], C)
        return V.reshape(-1)
    Xh = nodal(xh)[None, None, :]
    assert np.allclose(pmg.apply3(I, Xh, ph + 1)[0, 0], nodal(xl), atol=1e-12)
    assert np.allclose(pmg.apply3(Pm, nodal(xl)[None, None, :], pl + 1)[0, 0], Xh[0, 0], atol=1e-12)


@pytest.mark.parametrize("bdf2", [True, False])
def test_cycle_closed_form_uniform(bdf2):
    """Uniform states: every level sees the same point-wise linear map, the
    transfers are exact on constants and the FAS defect vanishes, so a cycle
    multiplies the velocity error by prod taylor4(a dtau_l)^n_l and the
    auxiliary variables by prod taylor4(dtau_l / T)^n_l."""
    P, n, T = 3, (2, 1, 2), 40.528
    dt, dtau, fac = 1e-2, 1e-3, 1.75
    Vn, Vm1 = np.array([0.3, -0.2, 0.1]), np.array([0.28, -0.25, 0.12])
    q0 = np.linspace(0.01, 0.09, 9)
    mk = lambda V: inputs.uniform(P, n, np.concatenate([[0.9], V, q0]))
    Vs, a = ((4 * Vn - Vm1) / 3, 1.5 / dt) if bdf2 else (Vn, 1.0 / dt)
    cyc = pmg.default_cycle(P)
    ncyc = 2
    U, cycles, res, rc = pmg.pmg_dual_step(P, n, mk(2 * Vn - Vm1), mk(Vn), mk(Vm1) if bdf2 else None,
                                           ZETA, NU, T, dt, dtau, 1e-30, ncyc, factor=fac)
    assert rc == -5 and cycles == ncyc
    fv = np.prod([taylor4(a * dtau * fac ** (P - p)) ** k for p, k in cyc]) ** ncyc
    fq = np.prod([taylor4(dtau * fac ** (P - p) / T) ** k for p, k in cyc]) ** ncyc
    U = U.reshape(-1, 13, (P + 1) ** 3)
    err0 = (2 * Vn - Vm1) - Vs
    assert np.allclose(U[:, 1:4], (Vs + err0 * fv)[None, :, None], rtol=0, atol=1e-13)
    assert np.allclose(U[:, 4:], (q0 * fq)[None, :, None], rtol=1e-12, atol=0)
    assert np.allclose(U[:, 0], 0.9, rtol=0, atol=1e-13)


def test_fas_fixed_point():
    """With a fine-level forcing that makes U* an exact fixed point, a whole
    cycle must leave U* in place: the coarse systems then start at their own
    equilibrium (a wrong sign of the defect moves them)."""
    P, n = 3, (2, 2, 1)
    U = inputs.tgv(P, n, noise=1e-2, seed=4).reshape(-1, 13, (P + 1) ** 3)
    Un = inputs.tgv(P, n, noise=1e-2, seed=5).reshape(U.shape)
    Um = inputs.tgv(P, n, noise=1e-2, seed=6).reshape(U.shape)
    dt = 1e-2
    a, B = 1.5 / dt, (Um[:, 1:4] - 4.0 * Un[:, 1:4]) / (2.0 * dt)
    F = -pmg.Level(P, n, ZETA, NU, T_CFG, None).pseudo_residual(U, a, B, None)
    V, cycles, res, rc = pmg.pmg_dual_step(P, n, U, Un, Um, ZETA, NU, T_CFG, dt, 1e-3, 0.0, 1,
                                           forcing=F)
    assert cycles == 1 and res < 1e-12
    scale = np.abs(U).max()
    assert np.abs(V.reshape(U.shape) - U).max() < 1e-12 * scale
    # control: the same cycle without the forcing moves the state
    W, _, _, _ = pmg.pmg_dual_step(P, n, U, Un, Um, ZETA, NU, T_CFG, dt, 1e-3, 0.0, 1)
    assert np.abs(W.reshape(U.shape) - U).max() > 1e-6


@pytest.mark.parametrize("bdf2", [True, False])
def test_reduces_to_rk4_dual_step(bdf2):
    """Coarse levels taking no steps: each cycle is (one + seven) fine RK4
    pseudo-steps, which the C oracle's dual step computes independently."""
    P, n = 2, (2, 3, 2)
    Unm1 = inputs.tgv(P, n, noise=1e-4, seed=1)
    Un = oracle.rk4(P, n, Unm1, ZETA, NU, T_CFG, 2.5e-3, 4)
    G = 2 * Un - Unm1
    dt, dtau, k = 1e-2, 1e-3, 3
    cyc = [(2, 1), (1, 0), (2, 7)]
    U, cycles, res, rc = pmg.pmg_dual_step(P, n, G, Un, Unm1 if bdf2 else None, ZETA, NU, T_CFG,
                                           dt, dtau, 1e-30, k, cycle=cyc)
    Uo, ito, reso, rco = oracle.dual_step(P, n, G, Un, Unm1 if bdf2 else None, ZETA, NU, T_CFG,
                                          dt, dtau, 1e-30, 8 * k, order=2 if bdf2 else 1)
    assert cycles == k and ito == 8 * k and rc == rco == -5
    assert np.linalg.norm(U - Uo.reshape(-1)) <= 1e-13 * np.linalg.norm(Uo)
    assert abs(res - reso) <= 1e-10 * reso


def test_pmg_converges_and_certifies():
    """A converged P-multigrid step satisfies the tolerance it reports, needs
    fewer fine-level pseudo-steps than the plain RK4 dual step, and both
    converged velocities agree to the size the tolerance allows: a velocity
    residual r moves V by about r / a (a = 3 / (2 dt) from the BDF term)."""
    P, n = 3, (2, 2, 2)
    Unm1 = inputs.tgv(P, n, noise=1e-4, seed=2)
    Un = oracle.rk4(P, n, Unm1, ZETA, NU, T_CFG, 2.5e-3, 4)
    G = 2 * Un - Unm1
    dt, dtau, tol = 1e-2, 1e-3, 1.2e-3
    U, cycles, res, rc = pmg.pmg_dual_step(P, n, G, Un, Unm1, ZETA, NU, T_CFG, dt, dtau, tol, 100)
    assert rc == 0 and res < tol
    sh = (-1, 13, 64)
    a, B = 1.5 / dt, (Unm1.reshape(sh)[:, 1:4] - 4.0 * Un.reshape(sh)[:, 1:4]) / (2 * dt)
    Rs = pmg.Level(P, n, ZETA, NU, T_CFG, None).pseudo_residual(U.reshape(sh), a, B, None)
    assert pmg.velocity_rms(Rs) == pytest.approx(res, rel=1e-12)
    Uo, ito, reso, rco = oracle.dual_step(P, n, G, Un, Unm1, ZETA, NU, T_CFG, dt, dtau, tol, 5000)
    assert rco == 0
    fine_steps = cycles * sum(k for p, k in pmg.default_cycle(P) if p == P)
    assert fine_steps < ito
    dv = U.reshape(sh)[:, 1:4] - Uo.reshape(sh)[:, 1:4]
    assert np.sqrt(np.mean(dv ** 2)) < 2 * tol / a
