"""Pins of the oracle's flow diagnostics (oracle/diagnostics.py): the
Taylor-Green closed forms at t = 0 (kinetic energy 1/8, enstrophy 3 nu / 4),
single-mode fields that isolate each of the six gradient entries the curl
uses, an irrotational field (zero enstrophy; catches a wrong sign in the
curl), and uniform states."""
import numpy as np
import pytest

from oracle.diagnostics import diagnostics
from paper_2107_14027_amd import inputs

NU = 1.0 / 1600.0


def field(p, n, V, G):
    """State with velocity V[i](x, y, z) and aux G[i][k](x, y, z) closed forms."""
    X = inputs.point_coords(p, n)
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    P = np.zeros_like(x)
    return inputs._assemble(P, [f(x, y, z) for f in V], [[g(x, y, z) for g in row] for row in G])


Z = lambda x, y, z: 0.0 * x


@pytest.mark.parametrize("p,N,tol", [(3, 4, 2e-3), (3, 8, 2e-6), (5, 8, 1e-10)])
def test_taylor_green_t0(p, N, tol):
    ke, ens = diagnostics(p, (N, N, N), inputs.tgv(p, (N, N, N)), NU)
    assert abs(ke - 1.0 / 8.0) <= tol / 8.0
    assert abs(ens - 0.75 * NU) <= tol * 0.75 * NU


@pytest.mark.parametrize("comp,i,k", [(0, 0, 1), (0, 0, 2), (1, 1, 0), (1, 1, 2), (2, 2, 0), (2, 2, 1)])
def test_each_curl_entry(comp, i, k):
    """u_i = sin(x_k) (k != i): one gradient entry cos(x_k), |omega|^2 mean 1/2,
    kinetic energy 1/4."""
    p, n = 5, (4, 4, 4)
    V = [Z, Z, Z]
    G = [[Z, Z, Z], [Z, Z, Z], [Z, Z, Z]]
    V[i] = lambda x, y, z, k=k: np.sin((x, y, z)[k])
    G[i][k] = lambda x, y, z, k=k: np.cos((x, y, z)[k])
    ke, ens = diagnostics(p, n, field(p, n, V, G), NU)
    assert ke == pytest.approx(0.25, rel=1e-9)
    assert ens == pytest.approx(0.5 * NU, rel=1e-9)


def test_diagonal_gradient_has_no_vorticity():
    p, n = 4, (3, 3, 3)
    V = [lambda x, y, z: np.sin(x), lambda x, y, z: np.sin(y), lambda x, y, z: np.sin(z)]
    G = [[lambda x, y, z: np.cos(x), Z, Z], [Z, lambda x, y, z: np.cos(y), Z],
         [Z, Z, lambda x, y, z: np.cos(z)]]
    ke, ens = diagnostics(p, n, field(p, n, V, G), NU)
    assert ke == pytest.approx(0.75, rel=1e-9)
    assert abs(ens) < 1e-20


def test_irrotational_field():
    """V = grad phi, phi = sin(x + 2y) cos z: curl V = 0 although every
    off-diagonal gradient entry is non-zero (a sign error in the curl shows)."""
    p, n = 5, (4, 4, 4)
    a = lambda x, y, z: x + 2 * y
    V = [lambda x, y, z: np.cos(a(x, y, z)) * np.cos(z),
         lambda x, y, z: 2 * np.cos(a(x, y, z)) * np.cos(z),
         lambda x, y, z: -np.sin(a(x, y, z)) * np.sin(z)]
    H = [[lambda x, y, z: -np.sin(a(x, y, z)) * np.cos(z), lambda x, y, z: -2 * np.sin(a(x, y, z)) * np.cos(z),
          lambda x, y, z: -np.cos(a(x, y, z)) * np.sin(z)],
         [lambda x, y, z: -2 * np.sin(a(x, y, z)) * np.cos(z), lambda x, y, z: -4 * np.sin(a(x, y, z)) * np.cos(z),
          lambda x, y, z: -2 * np.cos(a(x, y, z)) * np.sin(z)],
         [lambda x, y, z: -np.cos(a(x, y, z)) * np.sin(z), lambda x, y, z: -2 * np.cos(a(x, y, z)) * np.sin(z),
          lambda x, y, z: -np.sin(a(x, y, z)) * np.cos(z)]]
    U = field(p, n, V, H)
    ke, ens = diagnostics(p, n, U, NU)
    assert abs(ens) < 1e-22
    assert ke > 0.1
    # flipping the sign of one entry of a pair makes it rotational
    U2 = U.copy()
    U2[:, 9] *= -1.0   # r_z
    assert diagnostics(p, n, U2, NU)[1] > 1e-4


def test_uniform_state():
    p, n = 2, (2, 3, 1)
    vals = np.concatenate([[0.3], [0.5, -0.25, 2.0], np.full(9, 0.7)])
    ke, ens = diagnostics(p, n, inputs.uniform(p, n, vals), NU)
    assert ke == pytest.approx(0.5 * (0.25 + 0.0625 + 4.0), rel=1e-14)
    # constant aux 0.7 everywhere: each curl component is a difference of equal values
    assert ens == 0.0
