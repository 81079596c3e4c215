"""Standard ACM with LDG viscous fluxes -- TEST INFRASTRUCTURE ONLY (part of the oracle).

The paper's comparison system (Sec. 2.2, eq. (acm_2d), taken to three
dimensions; Sec. 5 runs it against ACM-HD): unknowns (P, u, v, w),

    dU/dtau + div F = 0,   F_j = [ zeta u_j ;  u_i u_j + P delta_ij - nu du_i/dx_j ].

The second-order term is formed by the FR route of Sec. 2.1 (the pair of
equations for a second-order PDE): first a corrected gradient of the velocity
with a common solution at the interfaces, then the FR divergence of the flux
evaluated with that gradient.  Interface treatment (Sec. 5): Rusanov on the
inviscid part (the same wave speed as for ACM-HD), LDG with parameters beta and
tau on the viscous part.  Readings taken where the paper gives only the two
numbers: at the interface between L (element on
the minus side of a face) and R (plus side), unit normal n along +xi_d,

    common solution        u^I = (u_L + u_R)/2 + beta (u_L - u_R)
    common viscous flux    F_v^I . n = (F_vL + F_vR).n / 2 - beta (F_vL - F_vR).n + tau (u_L - u_R)

with F_v = -nu grad u and the penalty on the velocity only; beta = 1/2 takes the
solution from L and the viscous flux from R.  The correction functions, points
and constant-Jacobian geometry are those of the ACM-HD oracle.

Arrays: U[e][4][m^3] with e = ex + nx (ey + ny ez) and point q = i + m (j + m k);
internally (nz, ny, nx, var, k, j, i).

Pins: tests/test_oracle_acm_ldg.py (reduction to the ACM-HD oracle at nu = 0,
closed-form smooth residual, conservation, the LDG energy identity for any
beta and tau, the side the common solution is taken from; the dual step's
reduction to the ACM-HD C oracle's dual step at nu = tau = 0).
"""
import numpy as np

from . import correction_deriv, gauss_legendre, geometry, lagrange_deriv, lagrange_eval

NA = 4
PAX = (-1, -2, -3)   # point axis of direction d (i, j, k)
EAX = (2, 1, 0)      # element axis of direction d (ex, ey, ez)


def operators(p):
    m = p + 1
    x, w = gauss_legendre(m)
    hl, hr = correction_deriv(p, x)
    return dict(w=w, D=lagrange_deriv(x), lm=lagrange_eval(x, -1.0), lp=lagrange_eval(x, 1.0),
                hl=hl, hr=hr)


def _apply(A, M, d):
    """out[.., i, ..] = sum_l M[i, l] A[.., l, ..] along the point axis of direction d."""
    ax = PAX[d]
    return np.moveaxis(np.tensordot(A, M, axes=([ax], [1])), -1, ax)


def _face(A, vec, d):
    """Value at a face of direction d: sum_l vec[l] A[.., l, ..] (that axis removed)."""
    return np.tensordot(A, vec, axes=([PAX[d]], [0]))


def _spread(F, vec, d):
    """Face array F times vec along the point axis of direction d."""
    ax = PAX[d]
    shape = [1] * (F.ndim + 1)
    shape[ax] = len(vec)
    return np.expand_dims(F, ax) * vec.reshape(shape)


def _lattice(p, n, U, nvar):
    nx, ny, nz = n
    m = p + 1
    return np.asarray(U, dtype=np.float64).reshape(nz, ny, nx, nvar, m, m, m)


def _neighbours(own_m, own_p, d):
    """Values across the faces: at e's minus face the plus-face value of e-1, at
    e's plus face the minus-face value of e+1 (periodic)."""
    return np.roll(own_p, 1, axis=EAX[d]), np.roll(own_m, -1, axis=EAX[d])


def _grad_lattice(p, n, X, beta, jac):
    """Corrected physical velocity gradient G[.., i, j, k, j, i] = du_i/dx_j
    (Sec. 2.1: derivative of the solution interpolant along each reference line
    plus (u^I - u^delta) h' at both ends, then dx/dxi applied)."""
    ops = operators(p)
    det, nvec, _ = geometry(n[0], n[1], n[2], jac)
    Jinv = nvec / det                        # (J^{-1})_{d j}
    V = X[:, :, :, 1:4]
    G = np.zeros(V.shape[:4] + (3,) + V.shape[4:])
    for d in range(3):
        om, op = _face(V, ops["lm"], d), _face(V, ops["lp"], d)
        nm, npl = _neighbours(om, op, d)
        # minus face: L = neighbour, R = own; plus face: L = own, R = neighbour
        ui_m = 0.5 * (nm + om) + beta * (nm - om)
        ui_p = 0.5 * (op + npl) + beta * (op - npl)
        gd = _apply(V, ops["D"], d) + _spread(ui_m - om, ops["hl"], d) + _spread(ui_p - op, ops["hr"], d)
        for j in range(3):
            G[:, :, :, :, j] += Jinv[d, j] * gd
    return G


def gradient(p, n, U, beta=0.5, jac=None):
    """Velocity gradient Q[e][3 i + j][m^3] = du_i/dx_j of a state U[e][4][m^3]."""
    X = _lattice(p, n, U, NA)
    G = _grad_lattice(p, n, X, beta, jac)
    m = p + 1
    return G.reshape(-1, 9, m ** 3)


def inviscid_normal_flux(Uf, nh):
    """[zeta V.n ; V (V.n) + P n] of face states Uf[.., 4, ..] (zeta applied by the caller)."""
    P, V = Uf[:, :, :, 0], Uf[:, :, :, 1:4]
    vn = nh[0] * V[:, :, :, 0] + nh[1] * V[:, :, :, 1] + nh[2] * V[:, :, :, 2]
    return vn, np.stack([V[:, :, :, i] * vn + P * nh[i] for i in range(3)], axis=3)


def common_flux(UL, UR, GL, GR, nh, zeta, nu, beta, tau):
    """Common normal flux (Sec. 5): Rusanov on the inviscid part, LDG on the viscous part."""
    vnL, mL = inviscid_normal_flux(UL, nh)
    vnR, mR = inviscid_normal_flux(UR, nh)
    lam = np.maximum(np.abs(vnL) + np.sqrt(vnL * vnL + zeta), np.abs(vnR) + np.sqrt(vnR * vnR + zeta))
    F = np.empty_like(UL)
    F[:, :, :, 0] = 0.5 * zeta * (vnL + vnR) - 0.5 * lam * (UR[:, :, :, 0] - UL[:, :, :, 0])
    for i in range(3):
        fvL = -nu * (GL[:, :, :, i, 0] * nh[0] + GL[:, :, :, i, 1] * nh[1] + GL[:, :, :, i, 2] * nh[2])
        fvR = -nu * (GR[:, :, :, i, 0] * nh[0] + GR[:, :, :, i, 1] * nh[1] + GR[:, :, :, i, 2] * nh[2])
        jump = UL[:, :, :, 1 + i] - UR[:, :, :, 1 + i]
        F[:, :, :, 1 + i] = (0.5 * (mL[:, :, :, i] + mR[:, :, :, i])
                             - 0.5 * lam * (UR[:, :, :, 1 + i] - UL[:, :, :, 1 + i])
                             + 0.5 * (fvL + fvR) - beta * (fvL - fvR) + tau * jump)
    return F


def residual(p, n, U, zeta, nu, beta=0.5, tau=0.1, jac=None):
    """R = -div F of a state U[e][4][m^3] over the periodic lattice n (Sec. 2.1, 2.2, 5)."""
    ops = operators(p)
    det, nvec, nmag = geometry(n[0], n[1], n[2], jac)
    X = _lattice(p, n, U, NA)
    G = _grad_lattice(p, n, X, beta, jac)
    P, V = X[:, :, :, 0], X[:, :, :, 1:4]
    # physical flux F[j] at the solution points
    F = np.empty((3,) + X.shape)
    for j in range(3):
        F[j][:, :, :, 0] = zeta * V[:, :, :, j]
        for i in range(3):
            F[j][:, :, :, 1 + i] = V[:, :, :, i] * V[:, :, :, j] + (P if i == j else 0.0) - nu * G[:, :, :, i, j]
    div = np.zeros_like(X)
    for d in range(3):
        Fh = nvec[d, 0] * F[0] + nvec[d, 1] * F[1] + nvec[d, 2] * F[2]
        div += _apply(Fh, ops["D"], d)
        nh = nvec[d] / nmag[d]
        Xm, Xp = _face(X, ops["lm"], d), _face(X, ops["lp"], d)
        Gm, Gp = _face(G, ops["lm"], d), _face(G, ops["lp"], d)
        _, Xn = _neighbours(Xm, Xp, d)
        _, Gn = _neighbours(Gm, Gp, d)
        FIp = common_flux(Xp, Xn, Gp, Gn, nh, zeta, nu, beta, tau)   # plus face: L = own
        FIm = np.roll(FIp, 1, axis=EAX[d])                           # minus face: e-1's plus face
        div += _spread(nmag[d] * FIm - _face(Fh, ops["lm"], d), ops["hl"], d)
        div += _spread(nmag[d] * FIp - _face(Fh, ops["lp"], d), ops["hr"], d)
    m = p + 1
    return (-div / det).reshape(-1, NA, m ** 3)


def pseudo_residual(p, n, U, Un, Unm1, dt, zeta, nu, beta, tau, jac):
    """R* = R(U) - M_V dU/dt with the BDF2 derivative (3U - 4Un + Unm1)/(2 dt),
    or BDF1 (U - Un)/dt when Unm1 is None; velocity only: the pressure has no
    physical time derivative (Sec. 2.2), as for ACM-HD."""
    Rs = residual(p, n, U, zeta, nu, beta, tau, jac)
    V, Vn = U[:, 1:4], Un[:, 1:4]
    dudt = (3.0 * V - 4.0 * Vn + Unm1[:, 1:4]) / (2.0 * dt) if Unm1 is not None else (V - Vn) / dt
    Rs[:, 1:4] -= dudt
    return Rs


def velocity_rms(Rs):
    """Root mean square of the three velocity components of R* over all points."""
    return float(np.sqrt(np.sum(Rs[:, 1:4] ** 2) / (3.0 * Rs.shape[0] * Rs.shape[2])))


def dual_step(p, n, U0, Un, Unm1, zeta, nu, dt, dtau, tol, max_iters, beta=0.5, tau=0.1, jac=None):
    """One BDF physical step of the standard ACM system by classical RK4
    pseudo-steps of size dtau on dU/dtau = R*(U) (Sec. 5's dual time stepping),
    until RMS(R*_V) < tol, tested on the first-stage residual of every
    pseudo-step.  Returns (U, iters, resid, rc): rc 0 converged, -5 max_iters
    reached, -4 non-finite norm."""
    m3 = (p + 1) ** 3
    U = np.array(U0, dtype=np.float64).reshape(-1, NA, m3)
    Un = np.asarray(Un, dtype=np.float64).reshape(-1, NA, m3)
    Unm1 = None if Unm1 is None else np.asarray(Unm1, dtype=np.float64).reshape(-1, NA, m3)
    c = (0.0, 0.5, 0.5, 1.0)
    b = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)
    it = 0
    while True:
        k = pseudo_residual(p, n, U, Un, Unm1, dt, zeta, nu, beta, tau, jac)
        res = velocity_rms(k)
        if not np.isfinite(res):
            return U, it, res, -4
        if res < tol:
            return U, it, res, 0
        if it >= max_iters:
            return U, it, res, -5
        acc = b[0] * k
        for s in range(1, 4):
            k = pseudo_residual(p, n, U + c[s] * dtau * k, Un, Unm1, dt, zeta, nu, beta, tau, jac)
            acc = acc + b[s] * k
        U = U + dtau * acc
        it += 1
