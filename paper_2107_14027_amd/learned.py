"""Learned initial guess study: pseudo-iterations per physical step with the
MLP guess versus polynomial extrapolation, at an identical tolerance.

Protocol (dual time stepping, BDF2, RK4 pseudo-steps, Taylor-Green field):
  step 1 BDF1 from the initial state, step 2 linear extrapolation, steps >= 3
  quadratic extrapolation; training rows (raw features, converged target) are
  sampled from every converged step >= 3 of the training phase; the network is fitted
  (normalisation from the rows, Adam); then the evaluation phase runs four
  times from the identical state at the end of training: with quadratic
  extrapolation, with linear extrapolation, with the network, and with the
  library's checked guess (fr_mlp_guess_checked: the network kept only where
  its initial pseudo-residual is not larger than that of the extrapolation it
  corrects), recording the completed pseudo-steps of every physical step.  The
  network corrects the extrapolation chosen by guess_base.  A ratio between
  two modes is reported only if neither capped a step (a capped step did not
  reach the tolerance, so the counts would not compare equal work).
  With solver="pmg" every physical step runs P-multigrid cycles instead (the
  paper's cycle shape for order p, pseudo-step x1.75 per level), and the counts
  are completed cycles.
Defaults: p = 3 on 16^3 hexes, dt = 5e-2 with dtau = dt/10 (the paper's ratio),
tolerance 1e-6; the iteration counts are set by the slowest (k = 1) pressure
mode, whose rate does not depend on the lattice.
Every arithmetic step runs in the HIP library; torch only holds the arrays.
"""
import json
import math
import sys
import time

import numpy as np

from . import binding as B
from . import inputs


class Diverged(RuntimeError):
    pass


def log(*a):
    print("[learned]", *a, file=sys.stderr, flush=True)


def run(p=3, N=16, dt=5e-2, dtau=5e-3, tol=1e-6, max_iters=3000, train_steps=20,
        eval_steps=20, samples_per_step=1 << 14, epochs=2000, lr=2e-3, batch=1 << 16,
        zeta=4.0, Re=1600.0, Lr=1.0 / (2.0 * math.pi), seed=5, precision=B.FR_F64, guess_base=2,
        solver="rk4", max_cycles=400, train_guess=2,
        modes=("extrap", "extrap1", "mlp", "mlp_fallback"), progress_every=5):
    import torch
    nu, T = inputs.nu_T_from_length(Re, Lr)
    n = (N, N, N)
    plan = B.Plan(p, n, zeta, nu, T, precision=precision)
    plan.set(B.FR_OPT_GUESS_BASE, guess_base)
    if solver not in ("rk4", "pmg"):
        raise ValueError("solver %r" % solver)
    mg = B.Pmg(plan) if solver == "pmg" else None
    unit = "cycles" if mg is not None else "pseudo-steps"
    ns = plan.state_len
    npts = ns // 13
    U0 = inputs.tgv(p, n)
    hist = [torch.tensor(U0, device="cuda")]
    rng = np.random.default_rng(seed)

    def step(guess, Un, Unm1):
        U = guess.clone()
        if mg is None:
            rc, it, res = B.fr_dual_step(plan.handle, U, Un, Unm1, dt, dtau, tol, max_iters,
                                         raise_on_error=False)
        else:
            rc, it, res = mg.dual_step(U, Un, Unm1, dt, dtau, tol, max_cycles, raise_on_error=False)
        if rc not in (B.FR_OK, B.FR_ENOCONV):
            raise Diverged("pseudo-iteration failed (status %d, residual %g after %d steps)"
                           % (rc, res, it))
        return U, it, res, rc

    def initial_residual(guess, Un, Unm1):
        U = guess.clone()
        rc, it, res = B.fr_dual_step(plan.handle, U, Un, Unm1, dt, dtau, tol, 0,
                                     raise_on_error=True)
        return res

    G = torch.empty_like(hist[0])
    X = torch.zeros((train_steps * samples_per_step, 12), dtype=torch.float32, device="cuda")
    Y = torch.zeros((train_steps * samples_per_step, 4), dtype=torch.float32, device="cuda")
    nrows = 0
    train_log = []
    t0 = time.time()
    for s in range(1, train_steps + 1):
        if s == 1:
            U, it, res, rc = step(hist[-1], hist[-1], None)
        else:
            order = 1 if s == 2 else train_guess
            B.fr_guess_extrap(plan.handle, hist[-1], hist[-2], hist[-3] if order == 2 else None,
                              order, G)
            U, it, res, rc = step(G, hist[-1], hist[-2])
            if s >= 3 and samples_per_step and rc == 0:
                stride = max(1, npts // samples_per_step)
                k = min(samples_per_step, (npts - 1) // stride + 1)
                off = int(rng.integers(0, npts - (k - 1) * stride))
                B.fr_mlp_sample(plan.handle, hist[-1], hist[-2], hist[-3], U, off, stride, k,
                                X[nrows:nrows + k], Y[nrows:nrows + k])
                nrows += k
        train_log.append((it, res, rc))
        hist.append(U)
        hist = hist[-3:]
        if s % progress_every == 0 or s <= 3:
            log("train step %d: %d %s, residual %.3e, rc %d (%.0f s)" %
                (s, it, unit, res, rc, time.time() - t0))
    # fit the network
    state = B.mlp_new_state(seed)
    Xr, Yr = X[:nrows], Y[:nrows]
    B.fr_mlp_fit_norm(plan.handle, state, Xr, Yr)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    for e in range(1, epochs + 1):
        idx = torch.randint(0, nrows, (min(batch, nrows),), device="cuda", generator=gen)
        B.fr_mlp_train_step(plan.handle, state, Xr[idx].contiguous(), Yr[idx].contiguous(), lr, e,
                            loss)
        if e == 1 or e % 250 == 0:
            torch.cuda.synchronize()
            losses.append((e, float(loss.item())))
    log("training loss (normalised MSE): %s" % losses)
    # evaluation from the identical state
    start = [h.clone() for h in hist]
    E = torch.empty_like(G)
    res_by = {}
    for mode in modes:
        hs = [h.clone() for h in start]
        its, r0s, rcs, fallback = [], [], [], 0
        t1 = time.time()
        for s in range(eval_steps):
            B.fr_guess_extrap(plan.handle, hs[-1], hs[-2], hs[-3], 1 if mode == "extrap1" else 2, E)
            guess = E
            if mode == "mlp":
                B.fr_mlp_guess(plan.handle, state, hs[-1], hs[-2], hs[-3], G)
                guess = G
            elif mode == "mlp_fallback":
                used, _, _ = B.fr_mlp_guess_checked(plan.handle, state, hs[-1], hs[-2], hs[-3],
                                                    dt, G)
                guess = G
                fallback += 0 if used else 1
            r0 = initial_residual(guess, hs[-1], hs[-2])
            r0s.append(r0)
            U, it, res, rc = step(guess, hs[-1], hs[-2])
            its.append(it)
            rcs.append(rc)
            hs.append(U)
            hs = hs[-3:]
            if s % progress_every == 0:
                log("%s step %d: %d %s, initial residual %.3e, rc %d" % (mode, s, it, unit, r0, rc))
        res_by[mode] = {"iters": its, "initial_residual": r0s, "rc": rcs, "fallback": fallback,
                        "seconds": time.time() - t1}
        log("%s: mean %.2f %s/step, median initial residual %.3e, %d capped, %d fallbacks" %
            (mode, np.mean(its), unit, np.median(r0s), sum(1 for r in rcs if r != 0), fallback))
    if mg is not None:
        mg.close()
    plan.close()
    summary = {}
    for mode, r in res_by.items():
        summary[mode] = {"iters_mean": float(np.mean(r["iters"])),
                         "ms_per_step": 1e3 * r["seconds"] / max(1, len(r["iters"])),
                         "capped": int(sum(1 for c in r["rc"] if c != 0)),
                         "initial_residual_median": float(np.median(r["initial_residual"])),
                         "fallbacks": r["fallback"], "iters": r["iters"],
                         "initial_residual": r["initial_residual"]}

    def ratio(a, b):
        if a not in summary or b not in summary:
            return None
        ma, mb = summary[a], summary[b]
        if ma["capped"] or mb["capped"]:
            return None
        return ma["iters_mean"] / max(1e-9, mb["iters_mean"])

    return {
        "config": {"p": p, "lattice": N, "dt": dt, "dtau": dtau, "tol": tol,
                   "max_iters": max_iters, "train_steps": train_steps, "eval_steps": eval_steps,
                   "samples": nrows, "epochs": epochs, "lr": lr, "zeta": zeta, "nu": nu, "T": T,
                   "guess_base": guess_base, "solver": solver, "train_guess": train_guess,
                   "max_cycles": max_cycles if solver == "pmg" else None},
        "train_iters_mean": float(np.mean([t[0] for t in train_log])),
        "train_capped": int(sum(1 for t in train_log if t[2] != 0)),
        "loss_curve": losses,
        "modes": summary,
        "mlp_vs_quadratic_iters": ratio("mlp", "extrap"),
        "mlp_vs_linear_iters": ratio("mlp", "extrap1"),
        "checked_vs_linear_iters": ratio("mlp_fallback", "extrap1"),
    }

if __name__ == "__main__":
    kw = json.loads(sys.argv[1]) if len(sys.argv) > 1 else {}
    try:
        out = run(**kw)
    except Diverged as e:
        out = {"config": kw, "diverged": str(e)}
    print(json.dumps(out), flush=True)
