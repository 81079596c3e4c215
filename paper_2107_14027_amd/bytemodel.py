"""Algorithmic HBM traffic of the residual kernels, in values per solution point.

Multiply by the bytes per value (8 in double, 4 in single precision) and by the
number of solution points to get bytes per launch.  m = p + 1 points per
direction, 13 unknowns per point (P, V, grad V), 7 face-trace values per face
point (P, V and the three components of grad V . n_hat), 6 faces of m^2 points.

Paper accounting (Sec. 3, Table 1 and the bandwidth model that follows it):
every array a stage reads or writes crosses global memory once.  Stage 2 reads
the solution and writes the d fluxes, stage 3 reads the fluxes and writes the
divergence, stage 6 reads the divergence and the variables its source term
depends on (the d^2 auxiliary variables of eq. acmhd_nd) and writes the result.
A kernel that fuses stages 2 and 3 (and 6) reads the solution once and writes
the result once.
"""
NV = 13
NTR = 7


def paper_stage_values(d=3):
    """Values per solution point moved by Table 1's stages 2, 3 and 6 and by the
    fused kernels that replace them (Sec. 3)."""
    nv = 1 + d + d * d
    return {
        "stage2": nv + d * nv,             # read U, write F_s (d components)
        "stage3": d * nv + nv,             # read F_s, write the divergence
        "stage6": nv + d * d + nv,         # read the divergence and the d^2 source inputs, write
        "fused23": nv + nv,                # read U once, write once
        "fused236": nv + nv,
    }


def paper_speedups(d=3):
    """Bandwidth-bound speed-ups of the fused kernels over the separate stages."""
    s = paper_stage_values(d)
    return {"fused_23": (s["stage2"] + s["stage3"]) / s["fused23"],
            "fused_236": (s["stage2"] + s["stage3"] + s["stage6"]) / s["fused236"]}


def floor_values():
    """Read every unknown once and write every residual once."""
    return 2 * NV


def trace_values(m):
    """Face-trace kernel: read U, write 7 values on each of the 6 faces."""
    return NV + 6 * NTR / m


def fused_values(m):
    """Fused kernel (stages 2-6): read U and the neighbours' traces, write R."""
    return 2 * NV + 6 * NTR / m


def fused_residual_values(m, halo=False):
    """Both kernels of the fused residual; with halo, the one kernel that
    recomputes the neighbours' face traces from their states (read through the
    caches: by design only U and R cross HBM)."""
    return floor_values() if halo else trace_values(m) + fused_values(m)


def unfused_values(m):
    """The six kernels of the unfused pipeline (Table 1), each through HBM:
    1 project U to the faces (13 values on 6 faces), 2 flux, 3 divergence,
    4 common flux (both sides read, 3 faces of 13 written), 5 correction
    (6 faces read, divergence read, result written), 6 negative and source."""
    s = paper_stage_values(3)
    return {"stage1": NV + 6 * NV / m,
            "stage2": s["stage2"],
            "stage3": s["stage3"],
            "stage4": 6 * NV / m + 3 * NV / m,
            "stage5": 6 * NV / m + 2 * NV,
            "stage6": s["stage6"]}


def bytes_per_launch(values_per_point, npoints, esz):
    return values_per_point * npoints * esz
