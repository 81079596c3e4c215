"""ACM-HD residual on linear hexahedra (non-constant Jacobian) -- TEST
INFRASTRUCTURE ONLY (part of the oracle).

The paper's future work (Sec. 6): elements whose Jacobian varies in space,
starting with linear hexahedra, where only the element corners are needed.
Each element is the trilinear image of [-1, 1]^3,
    x(xi) = sum_c N_c(xi) X_c,   N_c = prod_d (1 + s_cd xi_d) / 2,  s_cd = +-1,
with corners X_c, c = c0 + 2 c1 + 4 c2 (c_d = 0 at xi_d = -1).  With
a_d = dx/dxi_d, the metric terms at a point are the rows
    S_d = a_{d+1} x a_{d+2} = det(J) J^{-T} e_d,   det J = a_0 . S_0,
which for an affine element are the constant n_d of the paper's Sec. 2.1
mapping.  The FR residual of Table 1 then reads, per point,
    F_hat_d = sum_j S_dj F_j(U)                       (transformed flux)
    div     = sum_d [ d/dxi_d interpolant of F_hat_d
                      + h_l' (|S_d| F^I - F_hat_d^delta)(-1) + h_r' (...)(+1) ]
    R       = -div / det J + S(U)
with the common flux F^I (Rusanov on P, V; mean for the auxiliary equations,
Sec. 5) taken along the unit normal S_d / |S_d| at each face point.  The
flux on a face is evaluated once, from the metric of the element on its minus
side (the element on the plus side has the same face).  The physical flux is
eq. (acmhd_nd), written out here with numpy over whole lattices.

Arrays: U[e][13][m^3] (e = ex + nx (ey + ny ez), point q = i + m (j + m k)),
corners C[e][8][3].  Internally (nz, ny, nx, var, k, j, i).

Pins: tests/test_oracle_linear_hex.py (affine corners reproduce the
constant-Jacobian C oracle; free-stream preservation on distorted meshes;
conservation; convergence to the exact residual of a smooth field on
a smoothly distorted mesh).
"""
import numpy as np

from . import NV, correction_deriv, gauss_legendre, lagrange_deriv, lagrange_eval

PAX = (-1, -2, -3)
EAX = (2, 1, 0)
SIGNS = np.array([[2 * (c & 1) - 1, 2 * ((c >> 1) & 1) - 1, 2 * ((c >> 2) & 1) - 1] for c in range(8)],
                 dtype=np.float64)


def _apply(A, M, d):
    ax = PAX[d]
    return np.moveaxis(np.tensordot(A, M, axes=([ax], [1])), -1, ax)


def _face(A, vec, d):
    return np.tensordot(A, vec, axes=([PAX[d]], [0]))


def _spread(F, vec, d):
    ax = PAX[d]
    shape = [1] * (F.ndim + 1)
    shape[ax] = len(vec)
    return np.expand_dims(F, ax) * vec.reshape(shape)


def metric(C5, xi0, xi1, xi2):
    """Metric rows S[.., d, j, G] and det J[.., G] of the trilinear maps with
    corners C5[.., 8, 3] at the reference points (xi0, xi1, xi2) of a grid G."""
    G = np.broadcast(xi0, xi1, xi2).shape
    xi = [np.broadcast_to(x, G).ravel() for x in (xi0, xi1, xi2)]
    W = np.empty((8, 3, xi[0].size))
    for c in range(8):
        s = SIGNS[c]
        f = [0.5 * (1.0 + s[d] * xi[d]) for d in range(3)]
        for d in range(3):
            W[c, d] = 0.5 * s[d] * f[(d + 1) % 3] * f[(d + 2) % 3]
    a = np.einsum("...cj,cdg->...djg", C5, W)          # a[.., d, j, g] = dx_j/dxi_d
    S = np.stack([np.cross(a[..., (d + 1) % 3, :, :], a[..., (d + 2) % 3, :, :], axis=-2)
                  for d in range(3)], axis=-3)
    det = np.einsum("...jg,...jg->...g", a[..., 0, :, :], S[..., 0, :, :])
    return S.reshape(S.shape[:-1] + G), det.reshape(det.shape[:-1] + G)


def _flux_dot(X, nv, zeta, nu, T):
    """sum_j F_j(U) nv_j of eq. (acmhd_nd) for states X[z, y, x, 13, G] and
    vectors nv[z, y, x, 3, G]."""
    P = X[:, :, :, 0]
    V = [X[:, :, :, 1 + i] for i in range(3)]
    n = [nv[:, :, :, j] for j in range(3)]
    vn = V[0] * n[0] + V[1] * n[1] + V[2] * n[2]
    out = np.empty_like(X)
    out[:, :, :, 0] = zeta * vn
    for i in range(3):
        gn = sum(X[:, :, :, 4 + 3 * i + j] * n[j] for j in range(3))
        out[:, :, :, 1 + i] = V[i] * vn + P * n[i] - nu * gn
        for k in range(3):
            out[:, :, :, 4 + 3 * i + k] = -V[i] * n[k] / T
    return out


def common_flux(XL, XR, nh, zeta, nu, T):
    """F^I . n_hat between face states XL (minus side) and XR (Sec. 5)."""
    FL, FR = _flux_dot(XL, nh, zeta, nu, T), _flux_dot(XR, nh, zeta, nu, T)
    vnL = sum(XL[:, :, :, 1 + j] * nh[:, :, :, j] for j in range(3))
    vnR = sum(XR[:, :, :, 1 + j] * nh[:, :, :, j] for j in range(3))
    lam = np.maximum(np.abs(vnL) + np.sqrt(vnL * vnL + zeta), np.abs(vnR) + np.sqrt(vnR * vnR + zeta))
    F = 0.5 * (FL + FR)
    for v in range(4):
        F[:, :, :, v] -= 0.5 * lam * (XR[:, :, :, v] - XL[:, :, :, v])
    return F


def residual(p, n, U, C, zeta, nu, T):
    """R = -div F + S over the periodic lattice n of linear hexahedra with
    corners C[e][8][3]."""
    nx, ny, nz = n
    m = p + 1
    x, _ = gauss_legendre(m)
    D = lagrange_deriv(x)
    lm, lp = lagrange_eval(x, -1.0), lagrange_eval(x, 1.0)
    hl, hr = correction_deriv(p, x)
    X = np.asarray(U, dtype=np.float64).reshape(nz, ny, nx, NV, m, m, m)
    C5 = np.asarray(C, dtype=np.float64).reshape(nz, ny, nx, 8, 3)
    Sp, detp = metric(C5, x[None, None, :], x[None, :, None], x[:, None, None])   # grid (k, j, i)
    div = np.zeros_like(X)
    one = np.ones((1, 1))
    for d in range(3):
        Fh = _flux_dot(X, Sp[:, :, :, d], zeta, nu, T)
        div += _apply(Fh, D, d)
        # face grid (b, a): tangential nodes, xi_d = +1 on the plus face
        ta, tb = x[None, :], x[:, None]
        if d == 0:
            xis = [one, ta, tb]
        elif d == 1:
            xis = [ta, one, tb]
        else:
            xis = [ta, tb, one]
        Sf, _ = metric(C5, *xis)
        nvec = Sf[:, :, :, d]                                  # [.., 3, b, a]
        nmag = np.sqrt(np.sum(nvec * nvec, axis=3))
        nh = nvec / nmag[:, :, :, None]
        Xm, Xp = _face(X, lm, d), _face(X, lp, d)
        Xn = np.roll(Xm, -1, axis=EAX[d])                      # plus neighbour's minus face
        FIp = nmag[:, :, :, None] * common_flux(Xp, Xn, nh, zeta, nu, T)
        FIm = np.roll(FIp, 1, axis=EAX[d])
        div += _spread(FIm - _face(Fh, lm, d), hl, d)
        div += _spread(FIp - _face(Fh, lp, d), hr, d)
    R = -div / detp[:, :, :, None]
    R[:, :, :, 4:] -= X[:, :, :, 4:] / T
    return R.reshape(-1, NV, m ** 3)


def jacobian_det(p, C):
    """det J at every solution point, [e][m^3]."""
    m = p + 1
    x, _ = gauss_legendre(m)
    C5 = np.asarray(C, dtype=np.float64)[:, None, None]
    _, det = metric(C5, x[None, None, :], x[None, :, None], x[:, None, None])
    return det.reshape(-1, m ** 3)
