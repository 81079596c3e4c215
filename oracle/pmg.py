"""P-multigrid dual time stepping -- TEST INFRASTRUCTURE ONLY (part of the oracle).

Plain numpy on top of the oracle's serial C residual.  The paper accelerates
its pseudo-time iterations with a P-multigrid cycle (Sec. 5 and its cycle figure:
[(4,1), (3,1), (2,1), (1,4), (2,1), (3,1), (4,7)] of (order, pseudo-steps),
with the pseudo-step grown by a constant factor of 1.75 per level below the
finest).  The paper gives the cycle and the factor only; the rest is the
standard full-approximation-scheme (FAS) multigrid, read as follows:

  * level l solves dU/dtau = R*_l(U) + d_l with the BDF pseudo-residual
      R*_l(U) = R_l(U) - M_V (a U + B_l),  a = 3/(2 dt) (BDF2) or 1/dt (BDF1),
      B = (U^{n-1} - 4 U^n)/(2 dt) or -U^n/dt on the finest level,
    B_l its restriction, d_l the FAS defect (zero on the finest level);
  * going down from order h to l = h - 1:  r_h = R*_h(U_h) + d_h,
    U_l = I U_h (kept as U_l^0), d_l = I r_h - R*_l(U_l);
  * going up from l to h:  U_h += P (U_l - U_l^0);
  * I is the L2 projection onto degree l per direction (exact Gauss quadrature
    of the fine points), P the interpolation of the degree-l nodal
    polynomial at the fine points; both act per element as tensor products;
  * every level takes classical RK4 pseudo-steps of dtau * factor^(P - l);
  * convergence is tested before each cycle on RMS(R*_V) of the finest level;
    the count is of completed cycles.
Pins: tests/test_oracle_pmg.py.
"""
import numpy as np
from numpy.polynomial import legendre as npleg

from . import NV, gauss_legendre, lagrange_eval, residual
from . import rk34


def default_cycle(P):
    """The paper's cycle shape for a finest order P (its cycle figure, P = 4): one
    pseudo-step per level going down, four on order 1, one per level going up
    and seven on the finest order."""
    if P == 1:
        return [(1, 1)]
    down = [(p, 1) for p in range(P, 1, -1)]
    up = [(p, 1) for p in range(2, P)]
    return down + [(1, 4)] + up + [(P, 7)]


def check_cycle(P, cycle):
    if not cycle or cycle[0][0] != P or cycle[-1][0] != P:
        raise ValueError("a cycle starts and ends on the finest order")
    for (a, _), (b, _) in zip(cycle, cycle[1:]):
        if abs(a - b) != 1 or min(a, b) < 1:
            raise ValueError("consecutive levels differ by one order")
    for _, n in cycle:
        if n < 0:
            raise ValueError("negative step count")


def operators_1d(ph, pl):
    """(I, Pm): I[i, j] maps fine nodal values (order ph) to the nodal values at
    the coarse points (order pl) of their L2 projection onto degree pl; Pm[i, a]
    = l_a(x_i^h) interpolates a coarse nodal polynomial at the fine points."""
    xh, wh = gauss_legendre(ph + 1)
    xl, _ = gauss_legendre(pl + 1)
    I = np.zeros((pl + 1, ph + 1))
    for k in range(pl + 1):
        c = np.zeros(k + 1)
        c[k] = 1.0
        norm = (2 * k + 1) / 2.0   # 1 / int P_k^2
        I += norm * np.outer(npleg.legval(xl, c), npleg.legval(xh, c) * wh)
    Pm = np.array([lagrange_eval(xl, t) for t in xh])
    return I, Pm


def apply3(A, X, m_in):
    """Tensor product A (x) A (x) A applied to every [element][variable] block
    of X (last axis m_in^3, index i + m (j + m k))."""
    lead = X.shape[:-1]
    Y = X.reshape(lead + (m_in, m_in, m_in))              # [..., k, j, i]
    Y = np.einsum("ck,bj,ai,...kji->...cba", A, A, A, Y)
    return Y.reshape(lead + (A.shape[0] ** 3,))


class Level:
    def __init__(self, p, n, zeta, nu, T, jac):
        self.p, self.n, self.zeta, self.nu, self.T, self.jac = p, n, zeta, nu, T, jac
        self.ne = n[0] * n[1] * n[2]
        self.ns = (p + 1) ** 3

    def shape(self, nvar=NV):
        return (self.ne, nvar, self.ns)

    def pseudo_residual(self, U, a, B, D):
        """R*(U) + D with R* = R(U) - M_V (a U + B)."""
        R = residual(self.p, self.n, U.reshape(-1), self.zeta, self.nu, self.T, self.jac)
        R = R.reshape(self.shape())
        R[:, 1:4] -= a * U[:, 1:4] + B
        if D is not None:
            R = R + D
        return R

    def rk4_steps(self, U, a, B, D, dtau, nsteps):
        """Classical RK4 pseudo-steps of dU/dtau = R*(U) + D."""
        for _ in range(nsteps):
            k1 = self.pseudo_residual(U, a, B, D)
            k2 = self.pseudo_residual(U + 0.5 * dtau * k1, a, B, D)
            k3 = self.pseudo_residual(U + 0.5 * dtau * k2, a, B, D)
            k4 = self.pseudo_residual(U + dtau * k3, a, B, D)
            U = U + dtau * (k1 / 6.0 + k2 / 3.0 + k3 / 3.0 + k4 / 6.0)
        return U


    def rk34_steps(self, U, a, B, D, h, h0, atol, nsteps):
        """RK34 steps with the locally adaptive step field h (oracle/rk34.py)."""
        for _ in range(nsteps):
            U, h = rk34.step(lambda X: self.pseudo_residual(X, a, B, D), U, h, h0, atol)
        return U, h


def bdf_terms(fine, Un, Unm1, dt):
    """(a, B) of the BDF pseudo-residual on the finest level."""
    Unv = np.asarray(Un, dtype=np.float64).reshape(fine.shape())[:, 1:4]
    if Unm1 is None:
        return 1.0 / dt, -Unv / dt
    Um = np.asarray(Unm1, dtype=np.float64).reshape(fine.shape())[:, 1:4]
    return 1.5 / dt, (Um - 4.0 * Unv) / (2.0 * dt)


def dual_step_local(p, n, U0, Un, Unm1, zeta, nu, T, dt, dtau, tol, max_iters, h=None, jac=None):
    """One BDF physical step by RK34 pseudo-steps with locally adaptive steps
    (initial step dtau everywhere unless a field h is passed in), tested on
    RMS(R*_V) before every pseudo-step.  Returns (U, iters, resid, rc, h)."""
    lv = Level(p, n, zeta, nu, T, jac)
    a, B = bdf_terms(lv, Un, Unm1, dt)
    U = np.array(U0, dtype=np.float64).reshape(lv.shape())
    h = np.full(U.shape, dtau) if h is None else np.array(h, dtype=np.float64).reshape(U.shape)
    it, rc = 0, -5
    while True:
        res = velocity_rms(lv.pseudo_residual(U, a, B, None))
        if not np.isfinite(res):
            rc = -4
            break
        if res < tol:
            rc = 0
            break
        if it >= max_iters:
            break
        U, h = lv.rk34_steps(U, a, B, None, h, dtau, tol, 1)
        it += 1
    return U.reshape(-1), it, res, rc, h.reshape(-1)


def velocity_rms(Rs):
    return float(np.sqrt(np.mean(Rs[:, 1:4] ** 2)))


def pmg_dual_step(P, n, U0, Un, Unm1, zeta, nu, T, dt, dtau, tol, max_cycles, cycle=None,
                  factor=1.75, jac=None, forcing=None, scheme="rk4", fields=None):
    """One BDF physical step (BDF2, or BDF1 when Unm1 is None) by P-multigrid
    cycles of RK4 pseudo-steps.  Returns (U, cycles, resid, rc): rc 0 converged,
    -5 max_cycles completed without convergence, -4 non-finite residual.
    forcing (tests only) is a fixed source added on the finest level, where the
    FAS defect is otherwise zero.  scheme "rk34" takes RK34 steps with locally
    adaptive step fields on every level (initial step dtau * factor^(P - l),
    the convergence tolerance as the controller's atol); fields (a dict order ->
    step field) carries them between calls and is updated in place."""
    cycle = default_cycle(P) if cycle is None else [tuple(c) for c in cycle]
    check_cycle(P, cycle)
    levels = {p: Level(p, n, zeta, nu, T, jac) for p in {c[0] for c in cycle}}
    ops = {p: operators_1d(p + 1, p) for p in levels if p + 1 in levels}
    fine = levels[P]
    F = None if forcing is None else np.asarray(forcing, dtype=np.float64).reshape(fine.shape())
    U = np.array(U0, dtype=np.float64).reshape(fine.shape())
    Unv = np.asarray(Un, dtype=np.float64).reshape(fine.shape())[:, 1:4]
    if Unm1 is None:
        a, B = 1.0 / dt, -Unv / dt
    else:
        Um = np.asarray(Unm1, dtype=np.float64).reshape(fine.shape())[:, 1:4]
        a, B = 1.5 / dt, (Um - 4.0 * Unv) / (2.0 * dt)
    # restricted BDF constants
    Bs = {P: B}
    for p in range(P - 1, 0, -1):
        if p in levels:
            Bs[p] = apply3(ops[p][0], Bs[p + 1], p + 2)
    cycles, res, rc = 0, float("nan"), -5
    while True:
        res = velocity_rms(fine.pseudo_residual(U, a, B, F))
        if not np.isfinite(res):
            rc = -4
            break
        if res < tol:
            rc = 0
            break
        if cycles >= max_cycles:
            rc = -5
            break
        Us = {P: U}
        U0s, Ds = {}, {P: F}
        prev = None
        for p, nst in cycle:
            if prev is not None and p < prev:
                h = prev
                rh = levels[h].pseudo_residual(Us[h], a, Bs[h], Ds[h])
                I = ops[p][0]
                Us[p] = apply3(I, Us[h], h + 1)
                U0s[p] = Us[p].copy()
                Ds[p] = apply3(I, rh, h + 1) - levels[p].pseudo_residual(Us[p], a, Bs[p], None)
            elif prev is not None and p > prev:
                l = prev
                Us[p] = Us[p] + apply3(ops[l][1], Us[l] - U0s[l], l + 1)
            h0 = dtau * factor ** (P - p)
            if scheme == "rk34":
                if fields is None:
                    fields = {}
                hp = fields.get(p)
                if hp is None or hp.shape != Us[p].shape:
                    hp = np.full(Us[p].shape, h0)
                Us[p], fields[p] = levels[p].rk34_steps(Us[p], a, Bs[p], Ds[p], hp, h0, tol, nst)
            else:
                Us[p] = levels[p].rk4_steps(Us[p], a, Bs[p], Ds[p], h0, nst)
            prev = p
        U = Us[P]
        cycles += 1
    return U.reshape(-1), cycles, res, rc
