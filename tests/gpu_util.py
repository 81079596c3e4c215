"""Helpers for the GPU parity tests: run the HIP library through the C ABI on
seeded inputs and compare with the CPU oracle."""
import sys

import numpy as np

from paper_2107_14027_amd import binding as B

ZETA, NU = 4.0, 1.0 / 1600.0
T_CFG = (1.0 / (2.0 * np.pi)) ** 2 / NU     # relaxation length 1/(2 pi): T = Lr^2 / nu
TOL = {B.FR_F64: 1e-12, B.FR_F32: 1e-5}     # relative 2-norm bound on the residual


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def gpu_residual(p, n, U, zeta=ZETA, nu=NU, T=T_CFG, jac=None, precision=B.FR_F64,
                 variant=B.FR_FUSED, block=0, plan=None):
    import torch
    own = plan is None
    if own:
        plan = B.Plan(p, n, zeta, nu, T, jac, precision, variant, block)
    dt = torch.float64 if precision == B.FR_F64 else torch.float32
    Ud = torch.from_numpy(np.ascontiguousarray(U)).to("cuda").to(dt)
    Rd = torch.empty_like(Ud)
    B.fr_residual(plan.handle, Ud, Rd)
    torch.cuda.synchronize()
    out = Rd.double().cpu().numpy().reshape(U.shape)
    if own:
        plan.close()
    return out
