"""GPU flow diagnostics (fr_diagnostics) against the oracle's quadrature, the
Taylor-Green closed forms at t = 0, and a short Taylor-Green run whose kinetic
energy decays at the rate the enstrophy gives (they agree in the
incompressible limit)."""
import numpy as np
import pytest

from oracle.diagnostics import diagnostics
from paper_2107_14027_amd import binding as B
from paper_2107_14027_amd import inputs
from gpu_util import NU, T_CFG, ZETA, say

pytestmark = pytest.mark.gpu


def dev(U):
    import torch
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda")


@pytest.mark.parametrize("p,n", [(1, (5, 3, 4)), (2, (3, 4, 2)), (3, (4, 4, 4)), (4, (3, 2, 3)),
                                 (5, (2, 3, 2)), (6, (2, 2, 2))])
def test_matches_oracle(p, n):
    U = inputs.fourier(p, n, seed=40 + p)
    U = U + inputs.noise(U.shape, 0.1, seed=p)
    plan = B.Plan(p, n, ZETA, NU, T_CFG)
    say("diagnostics p=%d n=%s" % (p, n))
    ke, ens = B.fr_diagnostics(plan.handle, dev(U))
    ko, eo = diagnostics(p, n, U, NU)
    assert ke == pytest.approx(ko, rel=1e-12)
    assert ens == pytest.approx(eo, rel=1e-12)
    plan.close()


def test_taylor_green_t0():
    p, N = 5, 8
    plan = B.Plan(p, (N, N, N), ZETA, NU, T_CFG)
    ke, ens = B.fr_diagnostics(plan.handle, dev(inputs.tgv(p, (N, N, N))))
    assert abs(ke - 0.125) < 1e-10 * 0.125
    assert abs(ens - 0.75 * NU) < 1e-10 * 0.75 * NU
    plan.close()


def test_short_run_energy_balance():
    """p = 3 on 8^3 hexes to t = 0.2 (20 steps, the paper's zeta = 2.5 and
    T = 5e-3): the kinetic energy decays at the enstrophy's rate.  Central
    differences of the series recorded every 2 steps; the first two points
    carry the BDF1 start and the one-sided difference at t = 0 (measured: 1%
    after them at tol 2e-5 with the extrapolated pressure as the guess; with the
    pressure of the last step kept the rate falls up to 2.3% below)."""
    from paper_2107_14027_amd import tgv
    say("tgv short run")
    r = tgv.run(p=3, N=8, dt=1e-2, t_end=0.2, tol=2e-5, every=2, max_cycles=100, keep_p=False)
    s = r["series"]
    assert r["capped_steps"] <= 4
    ke, ens, rate = np.array(s["ke"]), np.array(s["enstrophy"]), np.array(s["ke_decay_rate"])
    assert ke[0] == pytest.approx(0.125, rel=1e-6)
    assert np.all(np.diff(ke) < 0)
    inner = slice(2, -1)
    assert np.max(np.abs(rate[inner] - ens[inner]) / ens[inner]) < 0.02, (rate, ens)


def test_run_with_the_pressure_kept_converges_every_step():
    """The paper's constants on 8^3 hexes, p = 3, to t = 1 with the pressure of
    the last step as its guess: no step reaches the cycle cap, the kinetic
    energy decays, and FP32 tracks FP64 to round-off."""
    from paper_2107_14027_amd import tgv
    say("tgv to t=1, pressure kept")
    out = {}
    for prec in (B.FR_F64, B.FR_F32):
        r = tgv.run(p=3, N=8, dt=1e-2, t_end=1.0, tol=2e-4, every=10, max_cycles=60, precision=prec)
        assert r["capped_steps"] == 0, r["series"]["cycles"]
        ke = np.array(r["series"]["ke"])
        assert np.all(np.diff(ke) < 0)
        out[prec] = np.array(r["series"]["enstrophy"])
    assert np.max(np.abs(out[B.FR_F32] - out[B.FR_F64]) / out[B.FR_F64]) < 1e-5
