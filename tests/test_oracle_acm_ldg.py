"""Pins of the standard-ACM / LDG oracle (oracle/acm_ldg.py) against facts
outside it: the ACM-HD C oracle (same inviscid system and Rusanov flux when
nu = 0), the exact residual of a smooth field, conservation, the LDG energy
identity (which fixes the sign and size of tau, the sides the common solution
and viscous flux are taken from, and the gradient), and the one-sided
dependence that beta = 1/2 implies."""
import numpy as np
import pytest

import oracle
from oracle import acm_ldg as A

ZETA = 4.0
SKEW = np.array([[0.8, 0.1, 0.05], [0.0, 0.7, -0.1], [0.05, 0.0, 0.9]])


def rand_state(p, n, seed, nvar=4):
    rng = np.random.default_rng(seed)
    ne = n[0] * n[1] * n[2]
    return rng.standard_normal((ne, nvar, (p + 1) ** 3))


@pytest.mark.parametrize("p,n,jac", [(1, (3, 2, 2), None), (3, (2, 3, 2), SKEW), (4, (2, 2, 3), None)])
def test_inviscid_part_is_acmhd(p, n, jac):
    """At nu = 0 the P and V equations of ACM-HD (eq. acmhd_nd) are those of ACM,
    and both use the same Rusanov flux, whatever the auxiliary variables."""
    U13 = rand_state(p, n, 1, 13) * 0.5
    R13 = oracle.residual(p, n, U13, ZETA, 0.0, 0.3, jac)
    R4 = A.residual(p, n, U13[:, :4], ZETA, 0.0, beta=0.5, tau=0.0, jac=jac)
    assert np.max(np.abs(R4 - R13[:, :4])) <= 1e-12 * np.max(np.abs(R13[:, :4]))


def exact_residual(x, y, z, nu, a):
    """P = a cos x, V = (sin y, sin z, sin x) (divergence free):
    R_P = 0, R_V = -(V.grad)V - grad P + nu lap V."""
    u, v, w = np.sin(y), np.sin(z), np.sin(x)
    return np.stack([0 * x,
                     -v * np.cos(y) + a * np.sin(x) - nu * np.sin(y),
                     -w * np.cos(z) - nu * np.sin(z),
                     -u * np.cos(x) - nu * np.sin(x)], axis=1)


def smooth_case(p, N, nu, beta=0.5, tau=0.1):
    m = p + 1
    xg, _ = oracle.gauss_legendre(m)
    h = 2 * np.pi / N
    e = np.arange(N ** 3)
    ex, ey, ez = e % N, (e // N) % N, e // (N * N)
    q = np.arange(m ** 3)
    i, j, k = q % m, (q // m) % m, q // (m * m)
    x = (ex[:, None] + 0.5 + 0.5 * xg[i][None, :]) * h
    y = (ey[:, None] + 0.5 + 0.5 * xg[j][None, :]) * h
    z = (ez[:, None] + 0.5 + 0.5 * xg[k][None, :]) * h
    a = 0.3
    U = np.stack([a * np.cos(x), np.sin(y), np.sin(z), np.sin(x)], axis=1)
    R = A.residual(p, (N, N, N), U, ZETA, nu, beta, tau)
    Q = A.gradient(p, (N, N, N), U, beta).reshape(-1, 3, 3, m ** 3)
    Qx = np.zeros_like(Q)
    Qx[:, 0, 1], Qx[:, 1, 2], Qx[:, 2, 0] = np.cos(y), np.cos(z), np.cos(x)
    return np.max(np.abs(R - exact_residual(x, y, z, nu, a))), np.max(np.abs(Q - Qx))


@pytest.mark.parametrize("beta,tau", [(0.5, 0.1), (0.0, 0.3)])
def test_smooth_field_residual(beta, tau):
    """The residual of a smooth field converges to the exact -div F (a second
    derivative: order p - 1 with the LDG gradient, which converges at order p).
    nu = 0.05, so a wrong viscous term would leave an error of ~5e-2 at every
    resolution."""
    p, nu = 4, 0.05
    e1, g1 = smooth_case(p, 4, nu, beta, tau)
    e2, g2 = smooth_case(p, 8, nu, beta, tau)
    assert e2 < 1.5e-3 and g2 < 3e-4
    assert e1 / e2 > 2 ** (p - 1) * 0.9 and g1 / g2 > 2 ** p * 0.75


@pytest.mark.parametrize("jac", [None, SKEW])
def test_conservation(jac):
    """The common fluxes are single valued, so the quadrature of det J R over
    the periodic box vanishes for every variable."""
    p, n = 3, (3, 2, 3)
    U = rand_state(p, n, 2)
    R = A.residual(p, n, U, ZETA, 0.02, 0.5, 0.1, jac)
    _, w = oracle.gauss_legendre(p + 1)
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    tot = np.einsum("evq,q->v", R, W)
    assert np.max(np.abs(tot)) <= 1e-12 * np.einsum("evq,q->v", np.abs(R), W).max()


def face_jump_energy(p, n, U, jac):
    """sum over faces of |n_d| int |V_L - V_R|^2 (Gauss quadrature on the face)."""
    m = p + 1
    x, w = oracle.gauss_legendre(m)
    lm, lp = oracle.lagrange_eval(x, -1.0), oracle.lagrange_eval(x, 1.0)
    _, _, nmag = oracle.geometry(n[0], n[1], n[2], jac)
    X = U.reshape(n[2], n[1], n[0], 4, m, m, m)[:, :, :, 1:4]
    W2 = np.outer(w, w)
    tot = 0.0
    for d, (pax, eax) in enumerate(((-1, 2), (-2, 1), (-3, 0))):
        own_p = np.tensordot(X, lp, axes=([pax], [0]))
        nb_m = np.roll(np.tensordot(X, lm, axes=([pax], [0])), -1, axis=eax)
        tot += nmag[d] * np.sum((own_p - nb_m) ** 2 * W2)
    return tot


@pytest.mark.parametrize("beta,tau,jac", [(0.5, 0.1, None), (0.0, 0.7, SKEW), (-0.3, 0.1, SKEW)])
def test_ldg_energy_identity(beta, tau, jac):
    """For the viscous part alone (R(nu, tau) - R(0, 0)), with Gauss quadrature
    exact for the products: sum det J w V.R = -nu sum det J w |grad V|^2
    - tau sum_faces |n_d| int |[[V]]|^2, for any beta (the LDG identity)."""
    p, n, nu = 2, (3, 2, 2), 0.03
    U = rand_state(p, n, 3)
    Rv = (A.residual(p, n, U, ZETA, nu, beta, tau, jac) - A.residual(p, n, U, ZETA, 0.0, beta, 0.0, jac))
    Q = A.gradient(p, n, U, beta, jac)
    det, _, _ = oracle.geometry(n[0], n[1], n[2], jac)
    _, w = oracle.gauss_legendre(p + 1)
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    lhs = det * np.einsum("eiq,eiq,q->", U[:, 1:4], Rv[:, 1:4], W)
    rhs = -nu * det * np.einsum("ejq,ejq,q->", Q, Q, W) - tau * face_jump_energy(p, n, U, jac)
    assert abs(lhs - rhs) <= 1e-11 * abs(rhs)
    assert np.max(np.abs(Rv[:, 0])) == 0.0


def test_half_beta_takes_the_minus_side():
    """beta = 1/2: the common solution at a face is the minus-side element's
    trace, so an element's gradient does not depend on its plus-side
    neighbours, while a non-zero beta - 1/2 makes it depend on them."""
    p, n = 2, (4, 3, 3)
    U = rand_state(p, n, 4)
    Up = U.copy()
    Up[1, 1:4] += 0.5          # element ex = 1, ey = ez = 0
    for beta, same in ((0.5, True), (0.2, False)):
        Q0, Q1 = A.gradient(p, n, U, beta), A.gradient(p, n, Up, beta)
        scale = np.abs(Q0).max()
        # ex = 0: its plus-x neighbour changed (equal to round-off of the blend)
        assert (np.abs(Q0[0] - Q1[0]).max() <= 1e-14 * scale) == same
        # ex = 2: its minus-x neighbour changed
        assert np.abs(Q0[2] - Q1[2]).max() > 1e-3 * scale


@pytest.mark.parametrize("bdf2,tol,maxit", [(True, 1.2e-3, 400), (False, 1e-30, 6)])
def test_dual_step_reduces_to_acmhd(bdf2, tol, maxit):
    """At nu = 0 and tau = 0 the standard ACM dual step is the ACM-HD dual step
    (the C oracle) restricted to P and V: same states, norms and iteration counts."""
    from paper_2107_14027_amd import inputs
    p, n = 3, (2, 2, 2)
    Unm1 = inputs.tgv(p, n, noise=1e-4, seed=2)
    Un = oracle.rk4(p, n, Unm1, ZETA, 0.0, 0.3, 2.5e-3, 4)
    G = 2 * Un - Unm1
    Um = Unm1 if bdf2 else None
    Uo, ito, reso, rco = oracle.dual_step(p, n, G, Un, Um, ZETA, 0.0, 0.3, 1e-2, 1e-3, tol, maxit,
                                          order=2 if bdf2 else 1)
    sel = lambda X: np.asarray(X).reshape(-1, 13, (p + 1) ** 3)[:, :4]
    U, it, res, rc = A.dual_step(p, n, sel(G), sel(Un), None if Um is None else sel(Um), ZETA, 0.0,
                                 1e-2, 1e-3, tol, maxit, beta=0.5, tau=0.0)
    assert rc == rco and it == ito
    assert res == pytest.approx(reso, rel=1e-11)
    assert np.max(np.abs(U - sel(Uo))) <= 1e-12 * np.max(np.abs(sel(Uo)))
    if bdf2:
        assert rc == 0 and it > 1
