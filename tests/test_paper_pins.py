"""Values the paper prints that the byte model and the physical constants must
reproduce (tests/golden/paper_constants.txt, each line citing its source):
the bandwidth-bound speed-ups of fusing Table 1's stages 2+3 (4x) and 2+3+6
(5.346x) from Sec. 3, and the enstrophy plot scale nu/|Omega| of Sec. 5."""
import math
import os

import pytest

from paper_2107_14027_amd import bytemodel, inputs


def golden():
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()[:2]
                vals[k] = float(v)
    return vals


def test_stage_counts_follow_table1():
    """Stage 2 reads U and writes d fluxes; stage 3 the reverse; stage 6 reads the
    divergence and the d^2 auxiliary variables of the source and writes."""
    s = bytemodel.paper_stage_values(3)
    assert (s["stage2"], s["stage3"], s["stage6"], s["fused236"]) == (52, 52, 35, 26)
    # 2D check of the same accounting: 7 unknowns
    s2 = bytemodel.paper_stage_values(2)
    assert (s2["stage2"], s2["stage3"], s2["stage6"], s2["fused23"]) == (21, 21, 18, 14)


def test_fused_23_speedup_is_four():
    """Sec. 3: four reads and four writes against one read and one write."""
    assert bytemodel.paper_speedups(3)["fused_23"] == pytest.approx(golden()["fused_23_speedup"],
                                                                    rel=1e-12)


def test_fused_236_speedup_matches_paper():
    """Sec. 3: 5.346x when the source term (stage 6) is fused as well."""
    sp = bytemodel.paper_speedups(3)["fused_236"]
    assert round(sp, 3) == golden()["fused_236_speedup"]
    # the model's other plausible readings miss the printed value: a stage 6 that
    # reads all 13 unknowns, or none of them
    assert round((52 + 52 + 39) / 26, 3) != golden()["fused_236_speedup"]
    assert round((52 + 52 + 26) / 26, 3) != golden()["fused_236_speedup"]


def test_unfused_pipeline_uses_the_same_accounting():
    """The unfused kernels of this library move Table 1's arrays; their stages
    2, 3 and 6 are the paper's counts, and the floor is one read + one write."""
    for m in range(2, 8):
        u = bytemodel.unfused_values(m)
        s = bytemodel.paper_stage_values(3)
        assert (u["stage2"], u["stage3"], u["stage6"]) == (s["stage2"], s["stage3"], s["stage6"])
        assert bytemodel.floor_values() == s["fused236"]
        assert bytemodel.fused_values(m) == pytest.approx(26 + 42 / m)
        assert sum(u.values()) == pytest.approx(178 + 273 / m)


def test_viscosity_matches_enstrophy_scale():
    """Sec. 5 scales the enstrophy integral by nu/|Omega| = 2.5197e-6 on [0, 2 pi]^3:
    pins nu = 1/Re = 1/1600 to five digits."""
    g = golden()
    nu, T = inputs.nu_T_from_length(g["tgv_reynolds"], 1.0 / (2.0 * math.pi))
    assert nu / (2.0 * math.pi) ** 3 == pytest.approx(g["nu_over_volume"], rel=2e-5)
    # a viscosity off by the first neglected digit fails
    assert (nu * 1.0001) / (2.0 * math.pi) ** 3 != pytest.approx(g["nu_over_volume"], rel=2e-5)
    assert T == pytest.approx((1.0 / (2.0 * math.pi)) ** 2 / nu)
