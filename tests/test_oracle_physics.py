"""Pins of the oracle's ACM-HD physics (paper Sec. 2.2, eq. acmhd_nd) and of the
common interface flux (Sec. 5) against the 2D component form, the flux
sparsity the paper counts, hyperbolicity, and an exact linear Riemann solution."""
import math
import os

import numpy as np
import pytest

import oracle

ZETA, NU, T = 4.0, 1.0 / 1600.0, 40.528


def golden():
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()[:2]
                vals[k] = float(v)
    return vals


def rand_state(rng, scale=1.0):
    return rng.standard_normal(13) * scale


def test_two_dimensional_reduction():
    """With w = 0 and no z-gradients the 3D system must equal the 2D component
    form eq. (acmhd_2d): fixes the orientation of S in the momentum flux."""
    rng = np.random.default_rng(1)
    for _ in range(10):
        P, u, v, qx, qy, rx, ry = rng.standard_normal(7)
        U = np.zeros(13)
        U[0], U[1], U[2] = P, u, v
        U[4], U[5], U[7], U[8] = qx, qy, rx, ry
        F = oracle.phys_flux(U, ZETA, NU, T)
        # eq. (acmhd_2d) ordering [P, u, v, q_x, q_y, r_x, r_y]
        fx = [ZETA * u, u * u + P - NU * qx, u * v - NU * rx, -u / T, 0.0, -v / T, 0.0]
        fy = [ZETA * v, u * v - NU * qy, v * v + P - NU * ry, 0.0, -u / T, 0.0, -v / T]
        sel = [0, 1, 2, 4, 5, 7, 8]
        assert np.allclose(F[0, sel], fx, atol=1e-15)
        assert np.allclose(F[1, sel], fy, atol=1e-15)
        src = oracle.source(U, T)
        assert np.allclose(src[sel], [0, 0, 0, -qx / T, -qy / T, -rx / T, -ry / T], atol=1e-16)
        # nothing is carried in z except the pressure in the (inactive) w equation
        assert np.allclose(F[2, [0, 1, 2]], [0.0, 0.0, 0.0], atol=1e-15)
        assert abs(F[2, 3] - P) < 1e-15


def test_flux_sparsity_matches_paper():
    """Sec. 3: a fraction s = 1 - (1+2d)/(1+d+d^2) of the flux entries vanish."""
    g = golden()
    rng = np.random.default_rng(2)
    U = rand_state(rng)
    F = oracle.phys_flux(U, ZETA, NU, T)
    d = 3
    zeros = np.sum(F == 0.0)
    assert zeros == 3 * 6
    s = zeros / F.size
    assert abs(s - (1 - (1 + 2 * d) / (1 + d + d * d))) < 1e-15
    assert abs(s - g["flux_sparsity_d3"]) < 5e-5


def numerical_jacobian(U, nhat, h=1e-6):
    J = np.zeros((13, 13))
    for c in range(13):
        e = np.zeros(13)
        e[c] = h
        fp = oracle.phys_flux(U + e, ZETA, NU, T).T @ nhat
        fm = oracle.phys_flux(U - e, ZETA, NU, T).T @ nhat
        J[:, c] = (fp - fm) / (2 * h)
    return J


@pytest.mark.parametrize("seed", range(6))
def test_hyperbolicity(seed):
    """Sec. 2.2: the flux Jacobian of ACM-HD has real eigenvalues."""
    rng = np.random.default_rng(10 + seed)
    U = rand_state(rng)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    A = numerical_jacobian(U, n)
    ev = np.linalg.eigvals(A)
    assert np.max(np.abs(ev.imag)) < 1e-6 * max(1.0, np.max(np.abs(ev.real)))
    # spectral radius of the ACM block: |V.n| + sqrt((V.n)^2 + zeta) (the Rusanov speed)
    vn = U[1:4] @ n
    assert abs(np.max(np.abs(ev.real)) - (abs(vn) + math.sqrt(vn * vn + ZETA))) < 1e-3


def test_common_flux_consistency_and_conservation():
    rng = np.random.default_rng(3)
    for _ in range(20):
        UL, UR = rand_state(rng), rand_state(rng)
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        # consistency: F^I(U, U) = F(U) . n
        assert np.allclose(oracle.common_flux(UL, UL, n, ZETA, NU, T),
                           oracle.phys_flux(UL, ZETA, NU, T).T @ n, atol=1e-14)
        # conservation: the flux leaving one side enters the other
        assert np.allclose(oracle.common_flux(UL, UR, n, ZETA, NU, T),
                           -oracle.common_flux(UR, UL, -n, ZETA, NU, T), atol=1e-14)
        # auxiliary equations: plain mean of the two normal fluxes (Sec. 5)
        fm = 0.5 * (oracle.phys_flux(UL, ZETA, NU, T) + oracle.phys_flux(UR, ZETA, NU, T)).T @ n
        assert np.allclose(oracle.common_flux(UL, UR, n, ZETA, NU, T)[4:], fm[4:], atol=1e-14)


def test_rusanov_equals_exact_linear_acoustic_riemann():
    """At rest the ACM part is linear acoustics (speeds +-sqrt(zeta)); the exact
    Godunov flux from the characteristic variables P +- c u must agree with the
    common flux up to the O(du^2) nonlinear momentum term."""
    c = math.sqrt(ZETA)
    rng = np.random.default_rng(4)
    eps = 1e-6
    for _ in range(10):
        UL = np.zeros(13)
        UR = np.zeros(13)
        UL[0], UR[0] = 1.0 + eps * rng.standard_normal(2)
        UL[1], UR[1] = eps * rng.standard_normal(2)
        n = np.array([1.0, 0.0, 0.0])
        wp = UL[0] + c * UL[1]          # right-going invariant from the left state
        wm = UR[0] - c * UR[1]          # left-going invariant from the right state
        Ps, us = 0.5 * (wp + wm), (wp - wm) / (2 * c)
        F = oracle.common_flux(UL, UR, n, ZETA, NU, T)
        assert abs(F[0] - ZETA * us) < 50 * eps * eps
        assert abs(F[1] - (Ps + us * us)) < 50 * eps * eps
