"""Pins of the oracle's full FR residual (paper Table 1 stages 1-6, Sec. 2.1-2.2):
free-stream preservation, discrete conservation on periodic lattices, an
independent weak-form nodal-DG brute force, exactness on piecewise polynomials,
design-order convergence on a manufactured solution, and symmetries."""
import math

import numpy as np
import numpy.polynomial.polynomial as npp
import pytest

import oracle
from paper_2107_14027_amd import inputs

ZETA, NU, T = 4.0, 1.0 / 1600.0, 40.528
SKEW = np.array([[0.30, 0.05, -0.02],
                 [0.01, 0.25, 0.04],
                 [-0.03, 0.02, 0.35]])   # a general constant Jacobian (det > 0)


def rand_U(p, n, seed, base=None):
    rng = np.random.default_rng(seed)
    ne = n[0] * n[1] * n[2]
    U = rng.standard_normal((ne, 13, (p + 1) ** 3)) * 0.3
    if base is not None:
        U += np.asarray(base)[None, :, None]
    return U


# --------------------------------------------------------------------------- free stream
@pytest.mark.parametrize("p", [1, 2, 3, 5])
@pytest.mark.parametrize("jac", [None, SKEW])
def test_free_stream(p, jac):
    vals = np.zeros(13)
    vals[:4] = [1.3, 0.4, -0.7, 0.2]
    U = inputs.uniform(p, (3, 2, 2), vals)
    R = oracle.residual(p, (3, 2, 2), U, ZETA, NU, T, jac)
    assert np.max(np.abs(R)) < 1e-12


# --------------------------------------------------------------------------- conservation
def weights3(p):
    _, w = np.polynomial.legendre.leggauss(p + 1)
    return np.einsum("k,j,i->kji", w, w, w).ravel()


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("jac", [None, SKEW])
def test_conservation(p, jac):
    n = (3, 2, 4)
    U = rand_U(p, n, seed=p, base=[1.0, 0.5, -0.3, 0.2] + [0.0] * 9)
    R = oracle.residual(p, n, U, ZETA, NU, T, jac)
    det = oracle.geometry(*n, jac)[0]
    W = weights3(p) * det
    tot = np.einsum("evq,q->v", R, W)
    scale = np.einsum("evq,q->v", np.abs(R), W)
    assert np.all(np.abs(tot[:4]) < 1e-13 * scale[:4])
    # the relaxation source of the auxiliary equations does not telescope
    tot_aux = np.einsum("evq,q->v", R[:, 4:] + U[:, 4:] / T, W)
    assert np.all(np.abs(tot_aux) < 1e-13 * (scale[4:] + 1.0))


# --------------------------------------------------------------------------- weak-form DG
def _lagrange_polys(x):
    out = []
    for k in range(len(x)):
        c = npp.polyfromroots(np.delete(x, k))
        out.append(c / npp.polyval(x[k], c))
    return out


def _flux_np(U, zeta, nu, T):
    """F[..., j, v] of eq. (acmhd_nd), written independently for the brute force."""
    P, V = U[..., 0], U[..., 1:4]
    S = U[..., 4:].reshape(U.shape[:-1] + (3, 3))      # S[i, k] = d u_i / d x_k
    F = np.zeros(U.shape[:-1] + (3, 13))
    for j in range(3):
        F[..., j, 0] = zeta * V[..., j]
        for i in range(3):
            F[..., j, 1 + i] = V[..., i] * V[..., j] + (P if i == j else 0.0) - nu * S[..., i, j]
            F[..., j, 4 + 3 * i + j] = -V[..., i] / T
    return F


def _numflux_np(Ui, Uo, nh, zeta, nu, T):
    """Outward common flux: Rusanov on (P, V), mean on the auxiliary variables."""
    fi = np.einsum("...jv,j->...v", _flux_np(Ui, zeta, nu, T), nh)
    fo = np.einsum("...jv,j->...v", _flux_np(Uo, zeta, nu, T), nh)
    vi, vo = Ui[..., 1:4] @ nh, Uo[..., 1:4] @ nh
    lam = np.maximum(np.abs(vi) + np.sqrt(vi ** 2 + zeta), np.abs(vo) + np.sqrt(vo ** 2 + zeta))
    F = 0.5 * (fi + fo)
    F[..., :4] -= 0.5 * lam[..., None] * (Uo[..., :4] - Ui[..., :4])
    return F


def weak_form_dg(p, n, U, zeta, nu, T, jac):
    """R from the weak form  int phi dU/dt = int grad(phi).F - oint phi F*.n_out + int phi S
    with the nodal Lagrange basis and Gauss quadrature on the same points."""
    nx, ny, nz = n
    m = p + 1
    x, w = np.polynomial.legendre.leggauss(m)
    polys = _lagrange_polys(x)
    L = np.array([[npp.polyval(xq, c) for xq in x] for c in polys])           # L[i, q]
    dL = np.array([[npp.polyval(xq, npp.polyder(c)) for xq in x] for c in polys])
    Lf = np.array([[npp.polyval(s, c) for s in (-1.0, 1.0)] for c in polys])  # Lf[i, side]
    J = inputs.box_jacobian(n) if jac is None else np.asarray(jac).reshape(3, 3)
    det = np.linalg.det(J)
    Ji = np.linalg.inv(J)
    # basis / gradient matrices over the tensor grid, index order (k, j, i) -> flat
    kron3 = lambda a, b, c: np.kron(np.kron(c, b), a)      # a acts on i, b on j, c on k
    G = [kron3(dL, L, L), kron3(L, dL, L), kron3(L, L, dL)]  # G[d][a, q] = dphi_a/dxi_d (x_q)
    W3 = np.kron(np.kron(w, w), w)
    ne = nx * ny * nz
    U4 = U.reshape(nz, ny, nx, 13, m ** 3)
    R = np.zeros_like(U4)
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                Ue = U4[ez, ey, ex].T                                       # [q, v]
                F = _flux_np(Ue, zeta, nu, T)                               # [q, j, v]
                Ft = np.einsum("dj,qjv->dqv", Ji, F)                        # reference flux
                vol = sum(G[d] @ (W3[:, None] * det * Ft[d]) for d in range(3))
                surf = np.zeros_like(vol)
                for d in range(3):
                    nd = det * Ji[d]                                       # n_d (Nanson)
                    area = np.linalg.norm(nd)
                    for side, sgn in ((0, -1.0), (1, 1.0)):
                        lf = Lf[:, side:side + 1]
                        lo = Lf[:, 1 - side:2 - side]
                        eye = np.eye(m)
                        mats = [eye, eye, eye]
                        mats[d] = lf
                        B = kron3(*mats)                                     # [a, face q]
                        mats[d] = lo
                        Bo = kron3(*mats)
                        off = [0, 0, 0]
                        off[d] = 1 if side else -1
                        nb = U4[(ez + off[2]) % nz, (ey + off[1]) % ny, (ex + off[0]) % nx].T
                        ui, uo = B.T @ Ue, Bo.T @ nb
                        Fs = _numflux_np(ui, uo, sgn * nd / area, zeta, nu, T)
                        wf = np.kron(*([w, w])) * area
                        surf += B @ (wf[:, None] * Fs)
                src = np.zeros_like(Ue)
                src[:, 4:] = -Ue[:, 4:] / T
                R[ez, ey, ex] = ((vol - surf) / (W3[:, None] * det) + src).T
    return R.reshape(ne, 13, m ** 3)


@pytest.mark.parametrize("p,n", [(1, (2, 1, 3)), (2, (2, 2, 2)), (3, (1, 2, 2)), (4, (2, 1, 1))])
@pytest.mark.parametrize("jac", [None, SKEW])
def test_matches_weak_form_dg(p, n, jac):
    U = rand_U(p, n, seed=7 + p, base=[1.0, 0.4, -0.2, 0.3] + [0.0] * 9)
    R = oracle.residual(p, n, U, ZETA, NU, T, jac)
    Rdg = weak_form_dg(p, n, U, ZETA, NU, T, jac)
    assert np.max(np.abs(R - Rdg)) < 1e-11 * np.max(np.abs(Rdg))


# --------------------------------------------------------------------------- polynomial exactness
@pytest.mark.parametrize("p", range(1, 7))
@pytest.mark.parametrize("jac", [None, SKEW])
def test_exact_on_continuous_piecewise_polynomials(p, jac):
    """g(t) = |t - 1|^p on a two-element periodic lattice is continuous, periodic
    and a degree-p polynomial inside each element; with continuous P and V the
    P and auxiliary residuals must equal the exact -zeta div V and
    (d_k u_i - S_ik)/T at every solution point."""
    n = (2, 2, 2)
    m = p + 1
    J = inputs.box_jacobian(n) if jac is None else np.asarray(jac)
    Ji = np.linalg.inv(J)
    X = inputs.point_coords(p, n, J)                          # [e][3][q]
    t = np.einsum("dj,ejq->edq", Ji, X) / 2.0                 # lattice coordinate in [0, 2]
    g = np.abs(t - 1.0) ** p
    dg = p * np.abs(t - 1.0) ** (p - 1) * np.sign(t - 1.0)     # dg/dt
    rng = np.random.default_rng(p)
    A = rng.standard_normal((4, 3))
    # field_c = A[c,0] g0 g1 + A[c,1] g1 g2 + A[c,2] g0 g2   (tensor degree <= p)
    terms = [(0, 1), (1, 2), (0, 2)]
    fields = np.zeros((4,) + g[:, 0].shape)
    grads = np.zeros((4, 3) + g[:, 0].shape)                   # d/dt_d
    for c in range(4):
        for a, (d1, d2) in enumerate(terms):
            fields[c] += A[c, a] * g[:, d1] * g[:, d2]
            grads[c, d1] += A[c, a] * dg[:, d1] * g[:, d2]
            grads[c, d2] += A[c, a] * g[:, d1] * dg[:, d2]
    # d/dx_j = sum_d (dt_d/dx_j) d/dt_d, dt_d/dx_j = Ji[d, j] / 2
    gx = np.einsum("dj,cdeq->cjeq", Ji / 2.0, grads)
    U = np.zeros((8, 13, m ** 3))
    U[:, 0] = fields[0]
    U[:, 1:4] = fields[1:4].transpose(1, 0, 2)
    U[:, 4:] = rng.standard_normal((8, 9, m ** 3))            # arbitrary auxiliary values
    R = oracle.residual(p, n, U, ZETA, NU, T, J)
    div = gx[1, 0] + gx[2, 1] + gx[3, 2]
    assert np.max(np.abs(R[:, 0] + ZETA * div)) < 1e-10 * np.max(np.abs(ZETA * div))
    for i in range(3):
        for k in range(3):
            exact = (gx[1 + i, k] - U[:, 4 + 3 * i + k]) / T
            assert np.max(np.abs(R[:, 4 + 3 * i + k] - exact)) < 1e-10 / T * (1 + np.max(np.abs(gx)))


# --------------------------------------------------------------------------- manufactured solution
def sines_exact_residual(p, n):
    """-div F + S for P = u = v = w = f = sin x sin y sin z, exact gradients.
    Closed form from sympy differentiation of the flux of eq. (acmhd_nd)."""
    import sympy as sp
    x, y, z = sp.symbols("x y z")
    X = (x, y, z)
    f = sp.sin(x) * sp.sin(y) * sp.sin(z)
    V = [f, f, f]
    P = f
    S = [[sp.diff(V[i], X[k]) for k in range(3)] for i in range(3)]
    flux = {}
    flux[0] = [ZETA * V[j] for j in range(3)]
    for i in range(3):
        flux[1 + i] = [V[i] * V[j] + (P if i == j else 0) - NU * S[i][j] for j in range(3)]
        for k in range(3):
            flux[4 + 3 * i + k] = [(-V[i] / T if j == k else 0) for j in range(3)]
    src = [0, 0, 0, 0] + [-S[i][k] / T for i in range(3) for k in range(3)]
    exprs = [-sum(sp.diff(flux[v][j], X[j]) for j in range(3)) + src[v] for v in range(13)]
    fns = [sp.lambdify(X, e, "numpy") for e in exprs]
    C = inputs.point_coords(p, n)
    out = np.zeros((C.shape[0], 13, C.shape[2]))
    for v in range(13):
        out[:, v] = np.broadcast_to(fns[v](C[:, 0], C[:, 1], C[:, 2]), out[:, v].shape)
    return out


@pytest.mark.parametrize("p", [1, 2, 3])
def test_manufactured_convergence(p):
    """Residual of the interpolated exact state converges to the exact operator
    at (at least) the design rate p in the max norm over solution points."""
    errs = []
    ns = [4, 8, 16] if p < 3 else [4, 8, 12]
    for nn in ns:
        n = (nn, nn, nn)
        U = inputs.sines(p, n)
        R = oracle.residual(p, n, U, ZETA, NU, T)
        E = sines_exact_residual(p, n)
        errs.append(np.max(np.abs(R[:, :4] - E[:, :4])))
    rates = [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(2)]
    assert rates[-1] > p - 0.2, (errs, rates)


# --------------------------------------------------------------------------- symmetries
def test_periodic_shift_equivariance():
    p, n = 2, (3, 2, 2)
    U = rand_U(p, n, seed=11, base=[1.0, 0.3, 0.1, -0.2] + [0.0] * 9)
    R = oracle.residual(p, n, U, ZETA, NU, T)
    U5 = U.reshape(n[2], n[1], n[0], 13, -1)
    Us = np.roll(U5, 1, axis=2).reshape(U.shape)
    Rs = oracle.residual(p, n, Us, ZETA, NU, T)
    assert np.array_equal(Rs, np.roll(R.reshape(U5.shape), 1, axis=2).reshape(U.shape))


def _swap_xy(U, p, n):
    """Exchange x and y: lattice axes, point axes i<->j, u<->v and the aux indices."""
    m = p + 1
    nx, ny, nz = n
    A = U.reshape(nz, ny, nx, 13, m, m, m)                   # [ez][ey][ex][v][k][j][i]
    A = A.transpose(0, 2, 1, 3, 4, 6, 5)                      # swap ex<->ey and i<->j
    perm = [0, 2, 1, 3]
    sig = [1, 0, 2]
    for i in range(3):
        for k in range(3):
            perm.append(4 + 3 * sig[i] + sig[k])
    return A[:, :, :, perm].reshape(U.shape)


def test_axis_swap_equivariance():
    p, n = 3, (2, 2, 3)
    U = rand_U(p, n, seed=12, base=[1.0, 0.3, 0.1, -0.2] + [0.0] * 9)
    R = oracle.residual(p, n, U, ZETA, NU, T)
    Rs = oracle.residual(p, n, _swap_xy(U, p, n), ZETA, NU, T)
    assert np.allclose(Rs, _swap_xy(R, p, n), atol=1e-13, rtol=0)


def test_mirror_equivariance():
    """x -> -x: reverse the x lattice and point order, flip u and the aux entries
    that pick up one sign (S_0k, S_i0 for i, k != 0)."""
    p, n = 2, (3, 2, 2)
    m = p + 1
    U = rand_U(p, n, seed=13, base=[1.0, 0.3, 0.1, -0.2] + [0.0] * 9)

    def mirror(A):
        B = A.reshape(n[2], n[1], n[0], 13, m, m, m)[:, :, ::-1, :, :, :, ::-1].copy()
        sgn = np.ones(13)
        sgn[1] = -1
        for i in range(3):
            for k in range(3):
                if (i == 0) != (k == 0):
                    sgn[4 + 3 * i + k] = -1
        return (B * sgn[None, None, None, :, None, None, None]).reshape(A.shape)

    R = oracle.residual(p, n, U, ZETA, NU, T)
    Rm = oracle.residual(p, n, mirror(U), ZETA, NU, T)
    assert np.allclose(Rm, mirror(R), atol=1e-13, rtol=0)


def test_compact_stencil_and_element_subset():
    p, n = 2, (5, 4, 4)
    U = rand_U(p, n, seed=14, base=[1.0, 0.2, 0.1, 0.0] + [0.0] * 9)
    R = oracle.residual(p, n, U, ZETA, NU, T)
    sel = np.array([0, 7, 33, 79])
    assert np.array_equal(oracle.residual_elems(p, n, U, sel, ZETA, NU, T), R[sel])
    # perturbing an element that is not a face neighbour leaves R of element 0 unchanged
    U2 = U.copy()
    far = 2 + 5 * (2 + 4 * 2)
    U2[far] += 1.0
    assert np.array_equal(oracle.residual_elems(p, n, U2, [0], ZETA, NU, T)[0], R[0])
    U2[1] += 1.0   # the +x neighbour
    assert not np.array_equal(oracle.residual_elems(p, n, U2, [0], ZETA, NU, T)[0], R[0])
