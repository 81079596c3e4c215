"""CPU oracle for the ACM-HD flux-reconstruction residual -- TEST INFRASTRUCTURE ONLY.

This package wraps ``fr_oracle.c`` (plain serial double precision C) with ctypes
and numpy.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product library never does, and the two share no
code.  Every function names the part of the paper it follows (Trojak, Watson,
Witherden, arXiv:2107.14027); the readings taken where the paper is silent are
listed in the C source header.

Pin status (tests/test_oracle_*.py):
  gauss_legendre, lagrange_*, correction_deriv   pinned (library + closed forms)
  phys_flux, common_flux                         pinned (2D eq., hyperbolicity,
                                                 consistency, sparsity count)
  residual, residual_elems                       pinned (free stream, conservation,
                                                 weak-form DG brute force, manufactured
                                                 solution convergence, equivariance)
  rk4                                            pinned (closed-form linear mode)
  dual_step                                      pinned (closed-form BDF recurrence)
  extrap                                         pinned (exact on quadratics)
  pmg.* (P-multigrid dual stepping, pmg.py)      pinned (projection/interpolation
                                                 exactness, closed-form cycle factors,
                                                 FAS fixed point, reduction to dual_step)
  rk34.step, pmg.dual_step_local (rk34.py)       pinned (order conditions, fourth-order local
                                                 error, closed-form uniform decay with the
                                                 controller's growth and cap, deadbeat
                                                 controller on an h^3 error, convergence)
  diagnostics.diagnostics (diagnostics.py)       pinned (Taylor-Green closed forms, single
                                                 modes per curl entry, irrotational field)
  mlp_*                                          pinned (finite differences, autograd; the
                                                 bfloat16 operand mode against autograd
                                                 through products with rounded operands and
                                                 torch's bfloat16 conversion)
  acm_ldg.residual, acm_ldg.gradient             pinned (reduction to the ACM-HD residual at
  (standard ACM with LDG, acm_ldg.py)            nu = 0, smooth-field convergence, conservation,
                                                 LDG energy identity for any beta and tau,
                                                 one-sided gradient at beta = 1/2)
  acm_ldg.dual_step                              pinned (equals the ACM-HD dual step on P, V
                                                 at nu = tau = 0: states, norms, iterations)
  linear_hex.residual (linear_hex.py)            pinned (affine corners = constant-Jacobian
                                                 residual, free stream on distorted meshes,
                                                 conservation, smooth-field convergence)
"""
import ctypes
import os
import subprocess

import numpy as np

NV = 13
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fr_oracle.c")
_SRC_MLP = os.path.join(_HERE, "mlp_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int)
_lib = None


def build(force=False):
    """Compile the oracle with gcc (serial, -O2, no fast-math)."""
    srcs = [_SRC, _SRC_MLP]
    if not force and os.path.exists(_LIB):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(_LIB) >= newest:
            return _LIB
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        I, D = ctypes.c_int, ctypes.c_double
        L.orc_gauss_legendre.argtypes = [I, _dp, _dp]
        L.orc_lagrange_eval.argtypes = [I, _dp, D, _dp]
        L.orc_lagrange_deriv.argtypes = [I, _dp, _dp]
        L.orc_correction_deriv.argtypes = [I, _dp, _dp, _dp]
        L.orc_phys_flux.argtypes = [_dp, D, D, D, _dp]
        L.orc_source.argtypes = [_dp, D, _dp]
        L.orc_common_flux.argtypes = [_dp, _dp, _dp, D, D, D, _dp]
        L.orc_residual.argtypes = [I, I, I, I, _dp, D, D, D, _dp, _dp]
        L.orc_residual_elems.argtypes = [I, I, I, I, _dp, D, D, D, _dp, ctypes.c_int64,
                                         _i64p, _dp]
        L.orc_geometry.argtypes = [I, I, I, _dp, _dp, _dp, _dp]
        L.orc_rk4.argtypes = [I, I, I, I, _dp, D, D, D, _dp, D, I]
        L.orc_dual_step.argtypes = [I, I, I, I, _dp, D, D, D, _dp, _dp, _dp, I, D, D, D, I,
                                    _ip, _dp]
        L.orc_extrap.argtypes = [ctypes.c_int64, _dp, _dp, _dp, I, _dp]
        L.orc_mlp_forward.argtypes = [ctypes.c_int64] + [_dp] * 9 + [ctypes.c_int]
        L.orc_bf16.argtypes = [ctypes.c_int64, _dp, _dp]
        L.orc_mlp_loss_grad.argtypes = [ctypes.c_int64] + [_dp] * 14 + [ctypes.c_int]
        L.orc_adam.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, D, D, D, D, I]
        for name in ("orc_gauss_legendre", "orc_residual", "orc_residual_elems",
                     "orc_geometry", "orc_rk4", "orc_dual_step", "orc_extrap"):
            getattr(L, name).restype = I
        L.orc_mlp_loss_grad.restype = D
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _jac(jac):
    if jac is None:
        return None, None
    j = _f64(jac).reshape(9)
    return j, _p(j)


# --------------------------------------------------------------------------- 1D operators
def gauss_legendre(m):
    """Gauss-Legendre nodes (ascending) and weights (Sec. 2.1: solution points)."""
    x = np.zeros(m)
    w = np.zeros(m)
    if lib().orc_gauss_legendre(m, _p(x), _p(w)):
        raise ValueError("bad m")
    return x, w


def lagrange_eval(x, t):
    """l_k(t) for the nodal basis on x (Sec. 2.1)."""
    x = _f64(x)
    out = np.zeros(len(x))
    lib().orc_lagrange_eval(len(x), _p(x), float(t), _p(out))
    return out


def lagrange_deriv(x):
    """D[i, k] = l_k'(x_i) (Sec. 2.1)."""
    x = _f64(x)
    D = np.zeros((len(x), len(x)))
    lib().orc_lagrange_deriv(len(x), _p(x), _p(D))
    return D


def correction_deriv(p, x):
    """h_l'(x_i), h_r'(x_i) for the DG (Radau) correction functions (Sec. 2.1)."""
    x = _f64(x)
    a = np.zeros(p + 1)
    b = np.zeros(p + 1)
    lib().orc_correction_deriv(p, _p(x), _p(a), _p(b))
    return a, b


# --------------------------------------------------------------------------- physics
def phys_flux(U, zeta, nu, T):
    """Physical flux F[j, v] of eq. (acmhd_nd) at one point."""
    U = _f64(U)
    F = np.zeros((3, NV))
    lib().orc_phys_flux(_p(U), zeta, nu, T, _p(F))
    return F


def source(U, T):
    U = _f64(U)
    S = np.zeros(NV)
    lib().orc_source(_p(U), T, _p(S))
    return S


def common_flux(UL, UR, nhat, zeta, nu, T):
    """Common normal flux at an interface (Sec. 5: Rusanov + mean)."""
    UL, UR, nh = _f64(UL), _f64(UR), _f64(nhat)
    F = np.zeros(NV)
    lib().orc_common_flux(_p(UL), _p(UR), _p(nh), zeta, nu, T, _p(F))
    return F


def geometry(nx, ny, nz, jac=None):
    """detJ, n_d (rows), |n_d| for the constant-Jacobian lattice."""
    j, jp = _jac(jac)
    det = ctypes.c_double()
    nvec = np.zeros((3, 3))
    nmag = np.zeros(3)
    if lib().orc_geometry(nx, ny, nz, jp, ctypes.byref(det), _p(nvec), _p(nmag)):
        raise ValueError("bad geometry")
    return det.value, nvec, nmag


# --------------------------------------------------------------------------- residual
def residual(p, n, U, zeta, nu, T, jac=None):
    """R = -div F + S over the periodic lattice n = (nx, ny, nz) (Table 1, stages 1-6)."""
    nx, ny, nz = n
    U = _f64(U)
    R = np.zeros_like(U)
    j, jp = _jac(jac)
    if lib().orc_residual(p, nx, ny, nz, jp, zeta, nu, T, _p(U), _p(R)):
        raise ValueError("bad arguments")
    return R


def residual_elems(p, n, U, elems, zeta, nu, T, jac=None):
    """Residual of the listed elements only, shape [len(elems), 13, m^3]."""
    nx, ny, nz = n
    U = _f64(U)
    sel = np.ascontiguousarray(elems, dtype=np.int64)
    m = p + 1
    R = np.zeros((len(sel), NV, m ** 3))
    j, jp = _jac(jac)
    if lib().orc_residual_elems(p, nx, ny, nz, jp, zeta, nu, T, _p(U), len(sel),
                                sel.ctypes.data_as(_i64p), _p(R)):
        raise ValueError("bad arguments")
    return R


def rk4(p, n, U, zeta, nu, T, dt, nsteps, jac=None):
    """nsteps classical RK4 steps of dU/dt = R(U); returns the new state."""
    nx, ny, nz = n
    U = _f64(U).copy()
    j, jp = _jac(jac)
    if lib().orc_rk4(p, nx, ny, nz, jp, zeta, nu, T, _p(U), dt, nsteps):
        raise ValueError("bad arguments")
    return U


def dual_step(p, n, U0, Un, Unm1, zeta, nu, T, dt, dtau, tol, max_iters, order=2, jac=None):
    """One BDF physical step by RK4 pseudo-time iteration.

    Returns (U, iters, resid, rc) with rc 0 (converged), -5 (no convergence),
    -4 (non-finite residual)."""
    nx, ny, nz = n
    U = _f64(U0).copy()
    Un = _f64(Un)
    Unm1 = _f64(Unm1) if Unm1 is not None else Un
    it = ctypes.c_int()
    res = ctypes.c_double()
    j, jp = _jac(jac)
    rc = lib().orc_dual_step(p, nx, ny, nz, jp, zeta, nu, T, _p(U), _p(Un), _p(Unm1), order,
                             dt, dtau, tol, max_iters, ctypes.byref(it), ctypes.byref(res))
    return U, it.value, res.value, rc


def extrap(Un, Unm1, Unm2, order, keep_p=False, ns=None):
    """Polynomial extrapolation of past states to the next physical step; with
    keep_p the pressure (variable 0 of each element's ns points) is taken from
    Un instead (it has no physical time derivative in Sec. 2.2's system)."""
    Un, Unm1 = _f64(Un), _f64(Unm1)
    Unm2 = _f64(Unm2) if Unm2 is not None else Un
    G = np.zeros_like(Un)
    if lib().orc_extrap(Un.size, _p(Un), _p(Unm1), _p(Unm2), order, _p(G)):
        raise ValueError("bad order")
    if keep_p:
        G.reshape(-1, NV, ns)[:, 0] = Un.reshape(-1, NV, ns)[:, 0]
    return G


# --------------------------------------------------------------------------- MLP
MLP_SHAPES = (("W1", (64, 12)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (4, 64)), ("b3", (4,)))


def bf16_round(x):
    """The bfloat16 rounding of the operand mode (binary32 first, then 8
    significant bits, nearest, ties to even), elementwise, as float64."""
    x = _f64(x)
    y = np.zeros_like(x)
    lib().orc_bf16(x.size, _p(x), _p(y))
    return y


def mlp_forward(X, params, return_hidden=False, bf16_operands=False):
    """Pointwise network 12 -> 64 -> 64 -> 4 (tanh hidden layers), FP64; with
    bf16_operands every matrix-product operand is rounded to bfloat16 first
    (accumulation stays in double; see mlp_oracle.c)."""
    X = _f64(X).reshape(-1, 12)
    P = [_f64(params[k]) for k, _ in MLP_SHAPES]
    Y = np.zeros((X.shape[0], 4))
    H = np.zeros((X.shape[0], 128)) if return_hidden else None
    lib().orc_mlp_forward(X.shape[0], _p(X), *[_p(a) for a in P], _p(Y),
                          _p(H) if H is not None else None, int(bool(bf16_operands)))
    return (Y, H) if return_hidden else Y


def mlp_loss_grad(X, Tg, params, bf16_operands=False):
    """Mean-squared error and its parameter gradients (textbook back-propagation);
    bf16_operands rounds every operand of every forward and backward matrix
    product to bfloat16 (mlp_oracle.c)."""
    X = _f64(X).reshape(-1, 12)
    Tg = _f64(Tg).reshape(-1, 4)
    P = [_f64(params[k]) for k, _ in MLP_SHAPES]
    G = [np.zeros(s) for _, s in MLP_SHAPES]
    loss = lib().orc_mlp_loss_grad(X.shape[0], _p(X), _p(Tg), *[_p(a) for a in P],
                                   *[_p(g) for g in G], int(bool(bf16_operands)))
    return loss, {k: g for (k, _), g in zip(MLP_SHAPES, G)}


def adam(param, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place on float64 arrays (bias-corrected, step >= 1)."""
    for a in (param, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(grad)
    lib().orc_adam(param.size, _p(param), _p(g), _p(m), _p(v), lr, beta1, beta2, eps, step)
