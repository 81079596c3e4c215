"""Helpers for the GPU parity tests: run the HIP library through the C ABI on
seeded inputs and compare with the CPU oracle."""
import sys

import numpy as np

from paper_2107_14027_amd import binding as B

ZETA, NU = 4.0, 1.0 / 1600.0
T_CFG = (1.0 / (2.0 * np.pi)) ** 2 / NU     # relaxation length 1/(2 pi): T = Lr^2 / nu
TOL = {B.FR_F64: 1e-12, B.FR_F32: 1e-5}     # relative 2-norm bound on the residual
# Per-group infinity-norm bound: the largest of N rounding errors of similar
# spread is about sqrt(2 ln N) ~ 4-6 times their RMS for N = 1e3..1e8 values,
# so the group bound is five times the 2-norm bound.
GROUP_TOL = {B.FR_F64: 5e-12, B.FR_F32: 5e-5}
GROUPS = (("P", slice(0, 1)), ("momentum", slice(1, 4)), ("aux", slice(4, 13)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def group_errors(R, Ro, U=None, zeta=ZETA, T=T_CFG):
    """Infinity-norm error of each variable group (P, momentum, auxiliary) of a
    residual R against the reference Ro, relative to the group's own scale: the
    largest reference value of the group or, when the state U is given, the
    largest operand of the group's residual, whichever is larger.  The operands
    matter where the residual cancels: R_P = -zeta div V (+ dissipation) with
    zeta |q_x| + zeta |r_y| + zeta |s_z| as its terms, and the auxiliary residual
    (grad V - S) / T with |S| / T as its terms, which nearly cancel on smooth
    fields with exact-gradient auxiliary variables."""
    R = np.asarray(R)
    assert R.ndim >= 2 and R.shape[-2] == 13, R.shape    # [..., variable, point]
    R = R.reshape(-1, 13, R.shape[-1])
    Ro = np.asarray(Ro).reshape(R.shape)
    ops = {}
    if U is not None:
        Uv = np.asarray(U).reshape(R.shape)
        ops["P"] = zeta * float(np.max(np.abs(Uv[:, 4]) + np.abs(Uv[:, 8]) + np.abs(Uv[:, 12])))
        ops["aux"] = float(np.max(np.abs(Uv[:, 4:13]))) / T
    out = {}
    for name, sl in GROUPS:
        err = float(np.max(np.abs(R[:, sl] - Ro[:, sl])))
        scale = max(float(np.max(np.abs(Ro[:, sl]))), ops.get(name, 0.0), 1e-300)
        out[name] = err / scale
    return out


def check_groups(R, Ro, precision, U=None, zeta=ZETA, T=T_CFG, what=""):
    """Assert every group's infinity-norm error is within GROUP_TOL; prints them."""
    g = group_errors(R, Ro, U, zeta, T)
    say("group errors %s: %s" % (what, " ".join("%s %.2e" % kv for kv in g.items())))
    for k, v in g.items():
        assert v <= GROUP_TOL[precision], (what, k, v)
    return g


def gpu_residual(p, n, U, zeta=ZETA, nu=NU, T=T_CFG, jac=None, precision=B.FR_F64,
                 variant=B.FR_FUSED, block=0, plan=None, form=B.FR_FORM_AUTO):
    import torch
    own = plan is None
    if own:
        plan = B.Plan(p, n, zeta, nu, T, jac, precision, variant, block)
        plan.set(B.FR_OPT_FORM, form)
    dt = torch.float64 if precision == B.FR_F64 else torch.float32
    Ud = torch.from_numpy(np.ascontiguousarray(U)).to("cuda").to(dt)
    Rd = torch.empty_like(Ud)
    B.fr_residual(plan.handle, Ud, Rd)
    torch.cuda.synchronize()
    out = Rd.double().cpu().numpy().reshape(U.shape)
    if own:
        plan.close()
    return out
