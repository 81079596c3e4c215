"""Flow diagnostics of a state -- TEST INFRASTRUCTURE ONLY (part of the oracle).

Sec. 5 monitors the Taylor-Green run through the enstrophy
    eps(t) = (nu / |Omega|) int_Omega omega . omega dx,  omega = curl V,
which in the incompressible limit equals the kinetic-energy dissipation rate,
and through the kinetic energy (1 / |Omega|) int_Omega |V|^2 / 2 dx.
Readings taken where the paper is silent: the integrals are the Gauss quadrature
of the solution points (exact for the nodal polynomials' squares), and omega is
formed from the auxiliary variables, which hyperbolised diffusion drives to
the velocity gradient: omega = (s_y - r_z, q_z - s_x, r_x - q_y) with
q = grad u, r = grad v, s = grad w.
Pins: tests/test_oracle_diagnostics.py.
"""
import numpy as np

from . import NV, gauss_legendre


def diagnostics(p, n, U, nu):
    """(kinetic energy, enstrophy) of a state U[e][13][m^3] on an n lattice."""
    m = p + 1
    _, w = gauss_legendre(m)
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)         # point q = i + m (j + m k)
    U = np.asarray(U, dtype=np.float64).reshape(-1, NV, m ** 3)
    ne = U.shape[0]
    assert ne == n[0] * n[1] * n[2]
    u, v, wv = U[:, 1], U[:, 2], U[:, 3]
    qy, qz = U[:, 5], U[:, 6]
    rx, rz = U[:, 7], U[:, 9]
    sx, sy = U[:, 10], U[:, 11]
    om = (sy - rz, qz - sx, rx - qy)
    vol = 8.0 * ne        # reference volume of every element; det J cancels
    ke = float(np.sum(W[None, :] * 0.5 * (u * u + v * v + wv * wv))) / vol
    ens = nu * float(np.sum(W[None, :] * (om[0] ** 2 + om[1] ** 2 + om[2] ** 2))) / vol
    return ke, ens
