"""Taylor-Green vortex run (Sec. 5): BDF2 dual time stepping with P-multigrid
cycles from t = 0 to t_end, recording the kinetic energy and the enstrophy
(fr_diagnostics) every `every` physical steps.

Protocol: Re 1600 on [0, 2 pi]^3 with the paper's constants for this run,
zeta = 2.5 and the relaxation time T = 5e-3 (the auxiliary variables then
follow the velocity gradient within a few pseudo-steps, so the enstrophy
formed from them is that of the velocity field); step 1 is BDF1 from the
initial state, later steps BDF2 from the linear extrapolation 2 U^n - U^{n-1}
of the velocity and auxiliary variables with the pressure of U^n (keep_p; the
pressure has no physical time derivative, and extrapolating the part of it an
unconverged step leaves makes the run diverge); pseudo-step dtau = dt / 10 on the
finest order, the paper's cycle shape, classical RK4 pseudo-steps on every level
(pseudo=1: RK34 with locally adaptive steps); the paper's single-precision tolerance
on the velocity pseudo-residual is 2e-4.  The kinetic-energy decay rate
-dKE/dt (central differences of the recorded series) is reported beside the
enstrophy, which equals it in the incompressible limit.
Every arithmetic step runs in the HIP library; torch only holds the arrays.

    python -m paper_2107_14027_amd.tgv '{"p": 4, "N": 32, "precision": 1}'
"""
import json
import sys
import time

import numpy as np

from . import binding as B
from . import inputs


def log(*a):
    print("[tgv]", *a, file=sys.stderr, flush=True)


def run(p=4, N=32, dt=1e-2, t_end=10.0, tol=2e-4, precision=B.FR_F64, every=10, max_cycles=200,
        zeta=2.5, Re=1600.0, T=5e-3, pseudo=0, factor=1.75, keep_p=True, log_seconds=20.0):
    import torch
    nu = 1.0 / Re
    n = (N, N, N)
    plan = B.Plan(p, n, zeta, nu, T, precision=precision)
    plan.set(B.FR_OPT_PSEUDO, pseudo)
    mg = B.Pmg(plan, None, factor)
    nsteps = int(round(t_end / dt))
    U = torch.tensor(inputs.tgv(p, n), device="cuda")
    prev = None
    series = [(0.0,) + B.fr_diagnostics(plan.handle, U) + (0,)]
    cycles_total, capped = 0, 0
    t0 = last = time.time()
    for s in range(1, nsteps + 1):
        G = torch.empty_like(U)
        if prev is None:
            G.copy_(U)
        else:
            B.fr_guess_extrap(plan.handle, U, prev, None, 1 | (B.FR_GUESS_KEEP_P if keep_p else 0), G)
        rc, cyc, res = mg.dual_step(G, U, prev, dt, dt / 10.0, tol, max_cycles,
                                    raise_on_error=False)
        if rc not in (B.FR_OK, B.FR_ENOCONV):
            raise RuntimeError("step %d failed: status %d, residual %g" % (s, rc, res))
        capped += rc != B.FR_OK
        cycles_total += cyc
        prev, U = U, G
        if s % every == 0 or s == nsteps:
            ke, ens = B.fr_diagnostics(plan.handle, U)
            series.append((s * dt, ke, ens, cyc))
        if time.time() - last > log_seconds:
            last = time.time()
            log("t = %.2f: KE %.6f, enstrophy %.6e, %d cycles this step (%.0f s)" %
                (s * dt, series[-1][1], series[-1][2], cyc, last - t0))
    wall = time.time() - t0
    mg.close()
    plan.close()
    t = np.array([r[0] for r in series])
    ke = np.array([r[1] for r in series])
    ens = np.array([r[2] for r in series])
    rate = -np.gradient(ke, t)
    ipk = int(np.argmax(ens))
    return {
        "config": {"p": p, "lattice": N, "dt": dt, "t_end": t_end, "tol": tol, "pseudo": pseudo,
                   "keep_p": keep_p,
                   "factor": factor,
                   "precision": "f32" if precision == B.FR_F32 else "f64", "zeta": zeta, "nu": nu,
                   "T": T, "every": every, "max_cycles": max_cycles},
        "series": {"t": t.tolist(), "ke": ke.tolist(), "enstrophy": ens.tolist(),
                   "ke_decay_rate": rate.tolist(), "cycles": [r[3] for r in series]},
        "enstrophy_peak": {"t": float(t[ipk]), "value": float(ens[ipk])},
        "cycles_mean": cycles_total / nsteps,
        "capped_steps": int(capped),
        "seconds": wall,
    }


if __name__ == "__main__":
    kw = json.loads(sys.argv[1]) if len(sys.argv) > 1 else {}
    print(json.dumps(run(**kw)), flush=True)
