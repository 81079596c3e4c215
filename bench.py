#!/usr/bin/env python3
"""Throughput of the fused ACM-HD flux-reconstruction residual on one MI355X.

Workload (order sweep): periodic box [0, 2 pi]^3 of 128^3, 85^3, 64^3, 51^3,
43^3, 40^3 hexahedra for p = 1..6 (16.6-22.0 M solution points each, 13
unknowns per point), seeded random Fourier velocity/pressure fields (|k| <= 4,
unit RMS) with exact-gradient auxiliary variables, zeta = 4, nu = 1/1600,
T = (1/(2 pi))^2 / nu.  One step = one fused double-precision residual
R = -div F + S at every order, all inputs resident in HBM.

Prints ONE JSON line on stdout; progress goes to stderr.
  value      GDOF/s = sum over orders of ne (p+1)^3 13, divided by the step time
  roofline   the dominant kernel (largest share of the step), HBM bound:
             algorithmic bytes per launch (the floor: read U once, write R
             once, 26 values per point) / its mean launch time, timed with HIP
             events on the launch stream inside the timed region; the bytes
             this design moves (the neighbours' face traces as well) are
             reported beside it
  sweep      per order: fused vs unfused, FP64 vs FP32 GDOF/s and each kernel's
             fraction of the 8 TB/s HBM peak
  cpu_baseline  the serial C oracle on a bounded sample of the same workload
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2107_14027_amd import bytemodel as BM  # noqa: E402

LATTICE = {1: 128, 2: 85, 3: 64, 4: 51, 5: 43, 6: 40}
ZETA, NU = 4.0, 1.0 / 1600.0
TRELAX = (1.0 / (2.0 * 3.141592653589793)) ** 2 / NU
HBM_PEAK_GBS = 8000.0
NV = 13


def rnd4(x):
    return None if x is None else round(x, 4)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def floor_bytes(p, ne, esz):
    """Algorithmic HBM bytes of one residual: read U and write R once (26 values
    per point)."""
    return BM.bytes_per_launch(BM.floor_values(), ne * (p + 1) ** 3, esz)


def fused_bytes(p, ne, esz):
    """Bytes the fused kernel moves by design: read U, the neighbours' face traces
    (6 faces x 7 values x m^2 points per element), write R."""
    return BM.bytes_per_launch(BM.fused_values(p + 1), ne * (p + 1) ** 3, esz)


def trace_bytes(p, ne, esz):
    """Face-trace kernel: read U once, write 6 x 7 x m^2 trace values per element."""
    return BM.bytes_per_launch(BM.trace_values(p + 1), ne * (p + 1) ** 3, esz)


# residual forms as the library reports them (FR_INFO_RESIDUAL_FORM)
FORM_NAMES = {1: "point", 2: "lines", 3: "halo"}


PAPER_CONTEXT = {
    "kernel_fusion_speedup": "3-4x fused vs unfused flux and divergence kernels, NVIDIA TITAN V, "
                             "CUDA 11.2 (abstract, Sec. 4); bandwidth bound 4x (stages 2+3) and "
                             "5.346x (2+3+6), Sec. 3",
    "end_to_end": "about 2.3x (FP32) and 2.2x (FP64) ACM-HD with fused kernels against standard "
                  "ACM, Taylor-Green to t = 10, NVIDIA V100 (Sec. 5)",
}


def read_traffic(kernel_name):
    """HBM traffic per launch from a committed rocprofv3 counter summary, if it was
    taken on the current kernel source; None otherwise."""
    from paper_2107_14027_amd.rocprof_summary import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "traffic_%s.txt" % kernel_name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def hbm_reference(torch, gib=2.0, reps=20):
    """Measured device bandwidth of plain torch copy (read+write), fill (write) and
    sum (read) over a `gib` GiB array: the practical ceilings for HBM streams."""
    n = int(gib * (1 << 30)) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn, nbytes in (("copy", lambda: y.copy_(x), 16 * n), ("fill", lambda: x.fill_(2.0), 8 * n),
                             ("read", lambda: x.sum(), 8 * n)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_gbs"] = round(nbytes / (e0.elapsed_time(e1) / reps) / 1e6, 1)
    del x, y
    torch.cuda.empty_cache()
    return out


def time_residual(B, torch, plan, U, R, reps, warm=1):
    for _ in range(warm):
        B.fr_residual(plan.handle, U, R)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        B.fr_residual(plan.handle, U, R)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(orders, lattices, host_states, budget_s):
    """Serial C oracle on a sample of elements of each order's lattice."""
    import numpy as np
    import oracle
    tot_dof, tot_t, sample = 0, 0.0, []
    per = budget_s / len(orders)
    for p in orders:
        n = lattices[p]
        ne = n[0] * n[1] * n[2]
        U = host_states[p]
        m = p + 1
        # calibrate on a few elements, then size the sample to the time budget
        rng = np.random.default_rng(p)
        probe = rng.choice(ne, size=min(64, ne), replace=False)
        t0 = time.perf_counter()
        oracle.residual_elems(p, n, U, probe, ZETA, NU, TRELAX)
        dt = (time.perf_counter() - t0) / len(probe)
        ns = int(max(min(64, ne), min(ne, per / max(dt, 1e-7))))
        sel = rng.choice(ne, size=ns, replace=False)
        t0 = time.perf_counter()
        oracle.residual_elems(p, n, U, sel, ZETA, NU, TRELAX)
        t = time.perf_counter() - t0
        tot_dof += ns * NV * m ** 3
        tot_t += t
        sample.append("p=%d: %d of %d elements" % (p, ns, ne))
        log("cpu oracle p=%d: %d elements in %.2f s" % (p, ns, t))
    return tot_dof / tot_t / 1e9, "; ".join(sample)


def time_steps(p=3, N=64, steps=5):
    """Wall time of one RK4 step and one dual pseudo-step (BDF2, norm every 10th)
    on a p=3, 64^3 FP64 Taylor-Green state, with the stage update in the fused
    kernel's epilogue and with the separate stage kernel."""
    import torch
    from paper_2107_14027_amd import binding as B
    from paper_2107_14027_amd import inputs
    nu, T = inputs.nu_T_from_length(1600.0, 1.0 / (2.0 * math.pi))
    n = (N, N, N)
    U0 = torch.tensor(inputs.tgv(p, n), device="cuda")
    out = {"workload": "Taylor-Green, p=%d on %d^3 hexes, FP64; ms per RK4 step (dt 1e-4) and per "
                       "BDF2 pseudo-step (dtau 5e-3)" % (p, N)}
    for fuse in (1, 0):
        plan = B.Plan(p, n, 4.0, nu, T)
        plan.set(B.FR_OPT_FUSE_STAGE, fuse)
        V = U0.clone()
        B.fr_rk_step(plan.handle, V, 1e-4, 1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        B.fr_rk_step(plan.handle, V, 1e-4, steps)
        torch.cuda.synchronize()
        rk = 1e3 * (time.perf_counter() - t) / steps
        W = U0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, it, res = B.fr_dual_step(plan.handle, W, U0, U0, 5e-2, 5e-3, 1e-30, 2 * steps,
                                     check_every=10, raise_on_error=False)
        torch.cuda.synchronize()
        du = 1e3 * (time.perf_counter() - t) / max(1, it)
        key = "stage_epilogue" if fuse else "separate_stage_kernel"
        out[key] = {"rk4_step_ms": round(rk, 3), "pseudo_step_ms": round(du, 3),
                    "path": {B.FR_STAGE_SEPARATE: "residual + separate stage kernel",
                             B.FR_STAGE_POINT: "point-form kernel with the epilogue",
                             B.FR_STAGE_HALO: "halo-form kernel with the epilogue"}[
                        B.fr_plan_get_int(plan.handle, B.FR_INFO_STAGE_PATH)]}
        plan.close()
        del V, W
    torch.cuda.empty_cache()
    return out


def time_acm(p=4, N=51, reps=10):
    """Standard ACM with LDG viscous fluxes (the paper's comparison system,
    beta = 0.5, tau = 0.1) against ACM-HD on the same p, N^3 FP64 box: ms per
    residual by HIP events on the launch stream.  The ACM state is the first
    four variables (P, V) of the sweep's Fourier state."""
    import torch
    from paper_2107_14027_amd import binding as B
    from paper_2107_14027_amd import inputs
    n = (N, N, N)
    plan = B.Plan(p, n, ZETA, NU, TRELAX)
    U13 = inputs.fourier(p, n, seed=1000 + p, device="cuda")
    R13 = torch.empty_like(U13)
    hd = time_residual(B, torch, plan, U13, R13, reps)
    acm = B.Acm(plan, 0.5, 0.1)
    U4 = U13.view(-1, NV, (p + 1) ** 3)[:, :4].contiguous().view(-1)
    del R13
    R4 = torch.empty_like(U4)
    acm.residual(U4, R4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        acm.residual(U4, R4)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    acm.close()
    plan.close()
    del U13, U4, R4
    torch.cuda.empty_cache()
    npts = N ** 3 * (p + 1) ** 3
    return {"workload": "one residual, p=%d on %d^3 hexes (%d solution points), FP64" % (p, N, npts),
            "acm_ldg_residual_ms": round(ms, 3), "acm_hd_fused_residual_ms": round(hd, 3),
            "acm_ldg_Mpoints_per_s": round(npts / ms / 1e3, 1),
            "acm_hd_Mpoints_per_s": round(npts / hd / 1e3, 1),
            "acm_ldg_over_acm_hd_time": round(ms / hd, 3)}


def time_lhex(p=4, N=51, reps=10):
    """ACM-HD residual on linear hexahedra (corners only, metric evaluated in
    the kernels) on a randomly distorted p, N^3 mesh, FP64: ms per residual by
    HIP events on the launch stream, with the sweep's Fourier state."""
    import torch
    from paper_2107_14027_amd import binding as B
    from paper_2107_14027_amd import inputs
    n = (N, N, N)
    plan = B.Plan(p, n, ZETA, NU, TRELAX)
    lh = B.LinearHex(plan)
    C = torch.tensor(inputs.linear_hex_corners(n, amp=0.2, seed=7, smooth=0.1), device="cuda")
    U = inputs.fourier(p, n, seed=1000 + p, device="cuda")
    R = torch.empty_like(U)
    lh.residual(C, U, R)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lh.residual(C, U, R)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    lh.close()
    plan.close()
    del U, R, C
    torch.cuda.empty_cache()
    npts = N ** 3 * (p + 1) ** 3
    return {"workload": "one ACM-HD residual on a distorted mesh of linear hexahedra, p=%d on %d^3 "
                        "(%d solution points), FP64" % (p, N, npts),
            "residual_ms": round(ms, 3), "GDOF_per_s": round(npts * NV / ms / 1e6, 2)}


def compare_dual(p=3, N=32, dt=1e-2, dtaus=(2e-3, 8e-3), tol=1e-4, max_iters=400):
    """One BDF1 physical step of the Taylor-Green vortex (Re 1600, zeta = 2.5,
    T = 5e-3, FP64) from its initial state by classical RK4 pseudo-steps of a
    fixed size, for standard ACM with LDG and for ACM-HD: pseudo-steps to reach
    tol and wall time (the norm is read back every pseudo-step in both)."""
    import torch
    from paper_2107_14027_amd import binding as B
    from paper_2107_14027_amd import inputs
    nu, _ = inputs.nu_T_from_length(1600.0, 1.0 / (2.0 * math.pi))
    n = (N, N, N)
    plan = B.Plan(p, n, 2.5, nu, 5e-3)
    acm = B.Acm(plan, 0.5, 0.1)
    U0 = torch.tensor(inputs.tgv(p, n), device="cuda")
    A0 = U0.view(-1, NV, (p + 1) ** 3)[:, :4].contiguous().view(-1)
    out = {"workload": "one BDF1 step (dt %g) of the Taylor-Green vortex from t = 0, p=%d on %d^3, "
                       "Re 1600, FP64, RK4 pseudo-steps to RMS(R*_V) < %g" % (dt, p, N, tol)}
    for dtau in dtaus:
        row = {}
        for name in ("acm_hd", "acm_ldg"):
            W = (U0 if name == "acm_hd" else A0).clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            if name == "acm_hd":
                rc, it, res = B.fr_dual_step(plan.handle, W, U0, None, dt, dtau, tol, max_iters,
                                             check_every=1, raise_on_error=False)
            else:
                rc, it, res = acm.dual_step(W, A0, None, dt, dtau, tol, max_iters, raise_on_error=False)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t)
            row[name] = {"converged": rc == B.FR_OK, "pseudo_steps": it, "ms": round(ms, 2),
                         "ms_per_pseudo_step": round(ms / max(1, it), 3)}
        out["dtau_%g" % dtau] = row
    acm.close()
    plan.close()
    del U0, A0
    torch.cuda.empty_cache()
    return out


def sines_operator(p, n):
    """-div F + S of ACM-HD in closed form for P = u = v = w = f = sin x sin y sin z
    with exact-gradient auxiliary variables (g = grad f): R_P = -zeta (g_x + g_y + g_z),
    R_u_i = -2 f (g_x + g_y + g_z) - g_i - 3 nu f (the viscous term's divergence is
    nu lap f = -3 nu f), R_aux = 0.  Returns (ne, 4, m^3) for P, u, v, w."""
    import numpy as np
    from paper_2107_14027_amd import inputs
    C = inputs.point_coords(p, n)
    x, y, z = C[:, 0], C[:, 1], C[:, 2]
    f = np.sin(x) * np.sin(y) * np.sin(z)
    g = (np.cos(x) * np.sin(y) * np.sin(z), np.sin(x) * np.cos(y) * np.sin(z),
         np.sin(x) * np.sin(y) * np.cos(z))
    sg = g[0] + g[1] + g[2]
    out = np.empty((f.shape[0], 4, f.shape[1]))
    out[:, 0] = -ZETA * sg
    for i in range(3):
        out[:, 1 + i] = -2.0 * f * sg - g[i] - 3.0 * NU * f
    return out


def mfma_config4(p=4, N=64, reps=10):
    """The matrix-core form (FR_MFMA: the per-direction operator block on
    v_mfma_f32_16x16x4f32, single-precision operands and accumulation) beside the
    double- and single-precision VALU fused residual on P = u = v = w =
    sin x sin y sin z, p = 4, N^3 hexes: time per residual, and the max and RMS
    error of P, u, v, w against the closed-form operator (the auxiliary residual
    is exactly zero there), with the same for n = 4, 8, 16, 32 and the observed
    orders of accuracy."""
    import math
    import numpy as np
    import torch
    from paper_2107_14027_amd import binding as B
    from paper_2107_14027_amd import inputs
    forms = (("f64_valu", B.FR_F64, B.FR_FUSED), ("f32_valu", B.FR_F32, B.FR_FUSED),
             ("f32_mfma", B.FR_F32, B.FR_MFMA))

    def run(n, timed):
        U = torch.from_numpy(inputs.sines(p, n)).to("cuda")
        E = torch.from_numpy(sines_operator(p, n)).to("cuda")
        out = {}
        for key, prec, var in forms:
            plan = B.Plan(p, n, ZETA, NU, TRELAX, precision=prec, variant=var)
            Ui = U if prec == B.FR_F64 else U.float()
            R = torch.empty_like(Ui)
            ms = time_residual(B, torch, plan, Ui, R, reps) if timed else None
            B.fr_residual(plan.handle, Ui, R)
            torch.cuda.synchronize()
            d = R[:, :4].double() - E
            out[key] = {"max_err": float(d.abs().max()), "rms_err": float(d.pow(2).mean().sqrt()),
                        "ms": ms, "R": R[:, :4].double() if timed else None}
            plan.close()
            del R
        scale = float(E.abs().max())
        del U, E
        torch.cuda.empty_cache()
        return out, scale

    n = (N, N, N)
    big, scale = run(n, True)
    ref = big["f64_valu"]["R"]
    res = {"workload": "P = u = v = w = sin x sin y sin z, exact-gradient auxiliary variables, "
                       "p=%d on %d^3 hexes (%d solution points); errors of P, u, v, w against "
                       "the closed-form operator (max |R| = %.3f)" % (p, N, N ** 3 * (p + 1) ** 3, scale)}
    npts = N ** 3 * (p + 1) ** 3
    for key, *_ in forms:
        r = big[key]
        res[key] = {"ms": round(r["ms"], 4),
                    "GDOF_per_s": round(npts * NV / (r["ms"] * 1e-3) / 1e9, 2),
                    "max_err": float("%.4g" % r["max_err"]), "rms_err": float("%.4g" % r["rms_err"])}
        if key != "f64_valu":
            d = r["R"] - ref
            res[key]["max_diff_vs_f64"] = float("%.4g" % float(d.abs().max()))
            res[key]["rel_l2_diff_vs_f64"] = float("%.4g" % float(d.norm() / ref.norm()))
    del big, ref
    torch.cuda.empty_cache()
    ns = (4, 8, 16, 32)
    errs = {key: [] for key, *_ in forms}
    for nn in ns:
        o, _ = run((nn, nn, nn), False)
        for key in errs:
            errs[key].append(o[key]["max_err"])
    res["convergence"] = {"n": list(ns)}
    for key, e in errs.items():
        res["convergence"][key] = {
            "max_err": [float("%.4g" % v) for v in e],
            "order": [round(math.log(e[i] / e[i + 1]) / math.log(ns[i + 1] / ns[i]), 2)
                      for i in range(len(ns) - 1)]}
    return res


def time_mlp(p=3, N=64, rows=1 << 16, reps=10):
    """The learned guess's kernels on their own: one network guess over every
    point of a p=3, 64^3 FP64 state (three states read, one written: 416 B per
    point; 2 x (12*64 + 64*64 + 64*4) flop per point) and one training step
    (forward, backward, Adam) on a batch of `rows` samples, by HIP events on
    the launch stream."""
    import torch
    from paper_2107_14027_amd import binding as B
    n = (N, N, N)
    plan = B.Plan(p, n, ZETA, NU, TRELAX)
    ns = plan.state_len
    npts = ns // NV
    st = B.mlp_new_state(5)
    g = torch.Generator(device="cuda").manual_seed(3)
    U = [torch.randn(ns, dtype=torch.float64, device="cuda", generator=g) for _ in range(3)]
    G = torch.empty_like(U[0])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        B.fr_mlp_guess(plan.handle, st, U[0], U[1], U[2], G)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        B.fr_mlp_guess(plan.handle, st, U[0], U[1], U[2], G)
    e1.record()
    torch.cuda.synchronize()
    gms = e0.elapsed_time(e1) / reps
    flop_pt = 2 * (12 * 64 + 64 * 64 + 64 * 4)
    bytes_pt = 4 * NV * 8
    X = torch.randn(rows, 12, dtype=torch.float32, device="cuda", generator=g)
    Y = torch.randn(rows, 4, dtype=torch.float32, device="cuda", generator=g)
    B.fr_mlp_fit_norm(plan.handle, st, X, Y)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for i in range(2):
        B.fr_mlp_train_step(plan.handle, st, X, Y, 1e-3, i + 1, loss)
    torch.cuda.synchronize()
    e0.record()
    for i in range(2 * reps):
        B.fr_mlp_train_step(plan.handle, st, X, Y, 1e-3, i + 3, loss)
    e1.record()
    torch.cuda.synchronize()
    tms = e0.elapsed_time(e1) / (2 * reps)
    plan.close()
    del U, G
    torch.cuda.empty_cache()
    return {"workload": "network guess on p=%d, %d^3 (%d points, FP64 states); training step on %d rows"
                        % (p, N, npts, rows),
            "guess_ms": round(gms, 4), "guess_GB_per_s": round(bytes_pt * npts / gms / 1e6, 1),
            "guess_frac_hbm": round(bytes_pt * npts / gms / 1e6 / HBM_PEAK_GBS, 4),
            "guess_TFLOP_per_s": round(flop_pt * npts / gms / 1e9, 2),
            "train_step_ms": round(tms, 4)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--orders", default="1,2,3,4,5,6")
    ap.add_argument("--no-sweep", action="store_true", help="skip the fused/unfused x FP64/FP32 table")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-hbm-ref", action="store_true", help="skip the copy/fill/read reference")
    ap.add_argument("--lattice", default=None,
                    help="NX,NY,NZ: one lattice for every order given (default: the sweep lattices)")
    ap.add_argument("--no-timestep", action="store_true",
                    help="skip the RK4 / dual pseudo-step timing (stage epilogue vs separate stage kernel)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-guess study (pseudo-iterations per physical step)")
    ap.add_argument("--no-acm", action="store_true",
                    help="skip the comparison-system timings: standard ACM (LDG) beside ACM-HD, "
                         "and ACM-HD on linear hexahedra")
    ap.add_argument("--learned64", default="5,2",
                    help="TRAIN,EVAL physical steps of the learned-guess study on the 64^3 lattice "
                         "(p=3, dt 1e-2, dtau 1e-3, tol 1e-6, P-multigrid); 0,0 skips it")
    ap.add_argument("--no-mfma", action="store_true",
                    help="skip the matrix-core precision form (p=4, 64^3 manufactured solution)")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="run a plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU; --gpus %d is not supported "
              "(sharding across GPUs is not implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    orders = [int(x) for x in args.orders.split(",")]

    import torch
    from paper_2107_14027_amd import binding as B
    from paper_2107_14027_amd import inputs
    B.lib()
    dev = "cuda"
    torch.cuda.init()

    if args.calib_copy_gib > 0:
        nb = int(args.calib_copy_gib * (1 << 30)) // 8
        a = torch.ones(nb, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy of %d bytes done" % (nb * 8))
        del a, b

    hbm_ref = None if args.no_hbm_ref else hbm_reference(torch)
    if hbm_ref:
        log("reference bandwidth: %s" % hbm_ref)

    work = []
    lattices = {}
    lat = tuple(int(x) for x in args.lattice.split(",")) if args.lattice else None
    for p in orders:
        N = LATTICE[p]
        n = lat or (N, N, N)
        lattices[p] = n
        t0 = time.perf_counter()
        U = inputs.fourier(p, n, seed=1000 + p, device=dev)
        R = torch.empty_like(U)
        plan = B.Plan(p, n, ZETA, NU, TRELAX, precision=B.FR_F64, variant=B.FR_FUSED)
        torch.cuda.synchronize()
        work.append((p, n, plan, U, R))
        log("order %d: %s hexes, %.1f M points, inputs in %.1f s" %
            (p, "x".join(map(str, n)), n[0] * n[1] * n[2] * (p + 1) ** 3 / 1e6, time.perf_counter() - t0))

    dof_step = sum(n[0] * n[1] * n[2] * NV * (p + 1) ** 3 for p, n, *_ in work)

    for _ in range(args.warmup):
        for p, n, plan, U, R in work:
            B.fr_residual(plan.handle, U, R)
    torch.cuda.synchronize()
    log("warmup done")
    for p, n, plan, U, R in work:
        plan.set(B.FR_OPT_PROFILE, 1)
        B.fr_plan_kernel_stats(plan.handle, 0, reset=True)

    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        for p, n, plan, U, R in work:
            B.fr_residual(plan.handle, U, R)
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    value = dof_step / (ms_step * 1e-3) / 1e9
    log("timed %d steps: %.3f ms/step, %.1f GDOF/s (wall %.3f s)" % (args.steps, ms_step, value, t_wall))

    kstats = {}
    for p, n, plan, U, R in work:
        ne = n[0] * n[1] * n[2]
        tr_ms, tr_n = B.fr_plan_kernel_stats(plan.handle, 0)
        fu_ms, fu_n = B.fr_plan_kernel_stats(plan.handle, 1)
        plan.set(B.FR_OPT_PROFILE, 0)
        fms, tms = fu_ms / max(fu_n, 1), tr_ms / max(tr_n, 1)
        form = B.fr_plan_get_int(plan.handle, B.FR_INFO_RESIDUAL_FORM)
        halo = form == B.FR_FORM_HALO
        # the halo form has no trace kernel: its one kernel is the whole residual
        design = floor_bytes(p, ne, 8) if halo else fused_bytes(p, ne, 8)
        kstats[p] = dict(trace_ms=tms, fused_ms=fms, fused_total=fu_ms, launches=fu_n, form=form,
                         design_bytes=design,
                         fused_floor_gbs=floor_bytes(p, ne, 8) / fms / 1e6,
                         fused_gbs=design / fms / 1e6,
                         trace_gbs=trace_bytes(p, ne, 8) / tms / 1e6 if tr_n else None,
                         residual_floor_gbs=floor_bytes(p, ne, 8) / (fms + tms) / 1e6)
    pdom = max(kstats, key=lambda p: kstats[p]["fused_total"])
    ndom = lattices[pdom]
    nedom = ndom[0] * ndom[1] * ndom[2]
    dom_bytes = floor_bytes(pdom, nedom, 8)
    achieved = dom_bytes / kstats[pdom]["fused_ms"] / 1e6
    form = kstats[pdom]["form"]
    kname = "%s_p%d_f64" % ({B.FR_FORM_LINES: "k_lines", B.FR_FORM_HALO: "k_lines_halo"}.get(form, "k_fused"),
                             pdom)
    traffic = read_traffic(kname)
    design = kstats[pdom]["design_bytes"]
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "bytes_per_launch": dom_bytes,
                "bytes_per_point": 26 * 8,
                "points_per_launch": nedom * (pdom + 1) ** 3,
                "mean_launch_ms": round(kstats[pdom]["fused_ms"], 4),
                "design_bytes_per_launch": design,
                "design_frac": round(design / kstats[pdom]["fused_ms"] / 1e6 / HBM_PEAK_GBS, 4),
                "whole_residual_frac": round(kstats[pdom]["residual_floor_gbs"] / HBM_PEAK_GBS, 4),
                "measured_reference_gbs": hbm_ref,
                "frac_of_measured_copy": (round(achieved / hbm_ref["copy_gbs"], 4) if hbm_ref else None)}

    sweep = {}
    if not args.no_sweep:
        for p, n, plan, U, R in work:
            ne = n[0] * n[1] * n[2]
            m = p + 1
            dof = ne * NV * m ** 3
            ks = kstats[p]
            row = {"form_f64": FORM_NAMES[ks["form"]],
                   "fused_f64": dof / (ks["fused_ms"] + ks["trace_ms"]) / 1e6,
                   "fused_kernel_f64_floor_frac": ks["fused_floor_gbs"] / HBM_PEAK_GBS,
                   "fused_kernel_f64_design_frac": ks["fused_gbs"] / HBM_PEAK_GBS,
                   "trace_kernel_f64_hbm_frac": (ks["trace_gbs"] / HBM_PEAK_GBS
                                                 if ks["trace_gbs"] is not None else None),
                   "fused_residual_f64_floor_frac": ks["residual_floor_gbs"] / HBM_PEAK_GBS}
            pu = B.Plan(p, n, ZETA, NU, TRELAX, precision=B.FR_F64, variant=B.FR_UNFUSED)
            pu.set(B.FR_OPT_PROFILE, 1)
            row["unfused_f64"] = dof / time_residual(B, torch, pu, U, R, 3) / 1e6
            # each unfused kernel's bandwidth by its own byte model (Table 1's arrays)
            uv = BM.unfused_values(m)
            for kid, stage in zip(range(2, 8), ("stage1", "stage2", "stage3", "stage4", "stage5",
                                                "stage6")):
                kms, kn = B.fr_plan_kernel_stats(pu.handle, kid)
                row["unfused_%s_f64_hbm_frac" % stage] = (
                    BM.bytes_per_launch(uv[stage], ne * m ** 3, 8) / (kms / max(kn, 1)) / 1e6
                    / HBM_PEAK_GBS)
            pu.close()
            U32 = U.float()
            R32 = torch.empty_like(U32)
            for var, key in ((B.FR_FUSED, "fused_f32"), (B.FR_UNFUSED, "unfused_f32")):
                pf = B.Plan(p, n, ZETA, NU, TRELAX, precision=B.FR_F32, variant=var)
                pf.set(B.FR_OPT_PROFILE, 1)
                row[key] = dof / time_residual(B, torch, pf, U32, R32, 3) / 1e6
                if var == B.FR_FUSED:
                    fu_ms, fu_n = B.fr_plan_kernel_stats(pf.handle, 1)
                    tr_ms, tr_n = B.fr_plan_kernel_stats(pf.handle, 0)
                    fms, tms = fu_ms / max(fu_n, 1), tr_ms / max(tr_n, 1)
                    halo32 = B.fr_plan_get_int(pf.handle, B.FR_INFO_RESIDUAL_FORM) == B.FR_FORM_HALO
                    d32 = floor_bytes(p, ne, 4) if halo32 else fused_bytes(p, ne, 4)
                    row["form_f32"] = FORM_NAMES[B.fr_plan_get_int(pf.handle, B.FR_INFO_RESIDUAL_FORM)]
                    row["fused_kernel_f32_floor_frac"] = (floor_bytes(p, ne, 4) / fms / 1e6
                                                          / HBM_PEAK_GBS)
                    row["fused_kernel_f32_design_frac"] = d32 / fms / 1e6 / HBM_PEAK_GBS
                    row["fused_residual_f32_floor_frac"] = (floor_bytes(p, ne, 4) / (fms + tms)
                                                            / 1e6 / HBM_PEAK_GBS)
                pf.close()
            del U32, R32
            torch.cuda.empty_cache()
            row["speedup_fused_vs_unfused_f64"] = row["fused_f64"] / row["unfused_f64"]
            row["speedup_fused_vs_unfused_f32"] = row["fused_f32"] / row["unfused_f32"]
            # the byte-model bound on that speed-up: unfused bytes / fused-residual bytes
            row["byte_model_speedup_bound"] = (sum(uv.values()) / BM.fused_residual_values(
                m, halo=ks["form"] == B.FR_FORM_HALO))
            sweep[str(p)] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in row.items()}
            log("sweep p=%d: %s" % (p, sweep[str(p)]))

    cpu = None
    if not args.no_cpu:
        import numpy as np
        host = {}
        for p, n, plan, U, R in work:
            host[p] = U.cpu().numpy()
        val, sample = cpu_baseline(orders, lattices, host, args.cpu_seconds)
        cpu = {"value": round(val, 6), "unit": "GDOF/s", "cores": 1, "kind": "oracle",
               "sample": "serial C oracle residual on randomly chosen elements of the same "
                         "lattices and fields: " + sample}
        del host

    timestep = None
    if not args.no_timestep:
        timestep = time_steps()
        log("time steps: %s" % timestep)

    acm = lhex = None
    if not args.no_acm:
        acm = time_acm()
        acm["dual_step"] = compare_dual()
        log("standard ACM: %s" % acm)
        lhex = time_lhex()
        log("linear hexahedra: %s" % lhex)

    mfma = None
    if not args.no_mfma:
        mfma = mfma_config4()
        log("matrix-core precision form: %s" % mfma)

    learned = None
    if not args.no_learned:
        from paper_2107_14027_amd import learned as L
        kern = time_mlp()
        log("mlp kernels: %s" % kern)
        t0 = time.perf_counter()
        r = L.run(guess_base=1)
        t1 = time.perf_counter()
        rp = L.run(guess_base=1, solver="pmg")
        mp = rp["modes"]
        m = r["modes"]
        learned = {
            "unit": "pseudo-iterations per physical step (mean over the evaluation steps)",
            "workload": "dual time stepping BDF2 + RK4 pseudo-steps, Taylor-Green Re 1600, p=%d, "
                        "%d^3 hexes, dt=%g, dtau=%g, tol %g, cap %d; %d training steps, %d "
                        "evaluation steps from the identical state" %
                        (r["config"]["p"], r["config"]["lattice"], r["config"]["dt"],
                         r["config"]["dtau"], r["config"]["tol"], r["config"]["max_iters"],
                         r["config"]["train_steps"], r["config"]["eval_steps"]),
            "learned": round(m["mlp"]["iters_mean"], 2),
            "quadratic_extrap": round(m["extrap"]["iters_mean"], 2),
            "linear_extrap": round(m["extrap1"]["iters_mean"], 2),
            "learned_checked": round(m["mlp_fallback"]["iters_mean"], 2),
            "capped": {k: m[v]["capped"] for k, v in (("learned", "mlp"), ("quadratic_extrap", "extrap"),
                                                      ("linear_extrap", "extrap1"))},
            "learned_vs_quadratic": rnd4(r["mlp_vs_quadratic_iters"]),
            "learned_vs_linear": rnd4(r["mlp_vs_linear_iters"]),
            "checked_vs_linear": rnd4(r["checked_vs_linear_iters"]),
            "training_loss": r["loss_curve"][-1][1],
            "seconds": round(t1 - t0, 1),
            "pmg_solver": {
                "unit": "P-multigrid cycles per physical step (cycle [(p,1),...,(1,4),...,(p,7)], "
                        "pseudo-step x1.75 per level), same protocol",
                "learned": round(mp["mlp"]["iters_mean"], 2),
                "quadratic_extrap": round(mp["extrap"]["iters_mean"], 2),
                "linear_extrap": round(mp["extrap1"]["iters_mean"], 2),
                "learned_checked": round(mp["mlp_fallback"]["iters_mean"], 2),
                "capped": {k: mp[v]["capped"] for k, v in (("learned", "mlp"),
                                                           ("quadratic_extrap", "extrap"),
                                                           ("linear_extrap", "extrap1"))},
                "ms_per_step": {k: round(mp[v]["ms_per_step"], 1) for k, v in
                                (("learned", "mlp"), ("quadratic_extrap", "extrap"),
                                 ("linear_extrap", "extrap1"))},
                "rk4_ms_per_step": {k: round(m[v]["ms_per_step"], 1) for k, v in
                                    (("learned", "mlp"), ("quadratic_extrap", "extrap"),
                                     ("linear_extrap", "extrap1"))},
                "learned_vs_quadratic": rnd4(rp["mlp_vs_quadratic_iters"]),
                "learned_vs_linear": rnd4(rp["mlp_vs_linear_iters"]),
                "checked_vs_linear": rnd4(rp["checked_vs_linear_iters"]),
                "seconds": round(time.perf_counter() - t1, 1)},
            "kernels": kern}
        tr64, ev64 = (int(x) for x in args.learned64.split(","))
        if tr64 > 0 and ev64 > 0:
            t2 = time.perf_counter()
            r6 = L.run(p=3, N=64, dt=1e-2, dtau=1e-3, tol=1e-6, solver="pmg", max_cycles=400,
                       train_steps=tr64, eval_steps=ev64, guess_base=1, samples_per_step=1 << 16,
                       modes=("extrap", "extrap1", "mlp"), progress_every=1)
            m6 = r6["modes"]
            learned["lattice_64"] = {
                "unit": "P-multigrid cycles per physical step (mean over the evaluation steps)",
                "workload": "dual time stepping BDF2 + P-multigrid RK4 pseudo-steps, Taylor-Green Re 1600, "
                            "p=3, 64^3 hexes, dt=0.01, dtau=0.001, tol 1e-06, cap 400 cycles; %d training "
                            "steps (65536 sampled points each), %d evaluation steps from the identical "
                            "state" % (tr64, ev64),
                "learned": round(m6["mlp"]["iters_mean"], 2),
                "quadratic_extrap": round(m6["extrap"]["iters_mean"], 2),
                "linear_extrap": round(m6["extrap1"]["iters_mean"], 2),
                "capped": {k: m6[v]["capped"] for k, v in (("learned", "mlp"), ("quadratic_extrap", "extrap"),
                                                           ("linear_extrap", "extrap1"))},
                "learned_vs_quadratic": rnd4(r6["mlp_vs_quadratic_iters"]),
                "learned_vs_linear": rnd4(r6["mlp_vs_linear_iters"]),
                "training_loss": r6["loss_curve"][-1][1],
                "seconds": round(time.perf_counter() - t2, 1)}
        log("learned guess: %s" % learned)

    out = {
        "metric": "fused RHS GDOF/s vs plain FP64 (p=1..6); pseudo-iters/step learned vs extrap",
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded random Fourier velocity and pressure (|k|<=4, unit RMS), "
                "exact-gradient auxiliary variables",
        "config": {"workload": "order sweep p=%s, fused FP64 ACM-HD FR residual, periodic box "
                               "[0,2pi]^3, lattices %s hexes" %
                               (",".join(map(str, orders)),
                                "/".join("x".join(map(str, lattices[p])) for p in orders)),
                   "orders": orders,
                   "points_per_order": {str(p): lattices[p][0] * lattices[p][1] * lattices[p][2] *
                                        (p + 1) ** 3 for p in orders},
                   "dof_per_step": dof_step, "zeta": ZETA, "nu": NU, "T": TRELAX,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "time_step": timestep,
        "standard_acm_ldg": acm,
        "linear_hexahedra": lhex,
        "mfma_config4": mfma,
        "learned_guess": learned,
        "sweep": sweep,
        "kernel_ms": {str(p): {"trace": round(kstats[p]["trace_ms"], 4),
                               "fused": round(kstats[p]["fused_ms"], 4)} for p in kstats},
    }
    print(json.dumps(out), flush=True)
    for p, n, plan, U, R in work:
        plan.close()


if __name__ == "__main__":
    main()
