"""The time integrators replay one captured HIP graph per (pseudo-)step; the
results must carry the same bits as plain launches, on the first call that
captures the graph, on later calls that replay it (with other GPU work in
between), and after anything baked into it (a pointer, dt) changes."""
import numpy as np
import pytest

from paper_2107_14027_amd import binding as B
from paper_2107_14027_amd import inputs
from gpu_util import NU, T_CFG, ZETA, say

pytestmark = pytest.mark.gpu


def dev(U):
    import torch
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda")


def plan_pair(p, n, prec, var):
    plans = []
    for graph in (1, 0):
        pl = B.Plan(p, n, ZETA, NU, T_CFG, None, prec, var)
        pl.set(B.FR_OPT_GRAPH, graph)
        plans.append(pl)
    return plans


def busy(x):
    # unrelated GPU work between calls on the same stream
    return (x * 1.0001).sum().item()


@pytest.mark.parametrize("prec", [B.FR_F64, B.FR_F32])
@pytest.mark.parametrize("var", [B.FR_FUSED, B.FR_UNFUSED])
def test_rk_graph_bitwise(prec, var):
    import torch
    p, n = 3, (4, 5, 3)
    U0 = inputs.tgv(p, n, noise=1e-3, seed=11)
    g, e = plan_pair(p, n, prec, var)
    say("rk graph prec=%d var=%d" % (prec, var))
    Ug, Ue = dev(U0), dev(U0)
    for dt, steps in ((1e-3, 5), (1e-3, 3), (2e-3, 4), (2e-3, 1)):
        B.fr_rk_step(g.handle, Ug, dt, steps)
        busy(Ug)
        B.fr_rk_step(e.handle, Ue, dt, steps)
        torch.cuda.synchronize()
        assert torch.equal(Ug, Ue), (dt, steps)
    # a new state array (another pointer baked into the graph)
    Vg, Ve = Ug.clone(), Ue.clone()
    B.fr_rk_step(g.handle, Vg, 2e-3, 3)
    B.fr_rk_step(e.handle, Ve, 2e-3, 3)
    torch.cuda.synchronize()
    assert torch.equal(Vg, Ve)
    g.close()
    e.close()


@pytest.mark.parametrize("prec", [B.FR_F64, B.FR_F32])
@pytest.mark.parametrize("every", [1, 3])
def test_dual_graph_bitwise(prec, every):
    import torch
    p, n = 2, (3, 2, 4)
    g, e = plan_pair(p, n, prec, B.FR_FUSED)
    say("dual graph prec=%d every=%d" % (prec, every))
    # two consecutive physical states: four RK4 steps of 2.5e-3 apart
    Unm1 = inputs.tgv(p, n, noise=1e-4, seed=2)
    dUm = dev(Unm1)
    dUn = dUm.clone()
    B.fr_rk_step(e.handle, dUn, 2.5e-3, 4)
    torch.cuda.synchronize()
    Un = dUn.cpu().numpy()
    G0 = 2 * Un - Unm1
    cases = [(1e-2, 1e-3, 1e-3, 400), (1e-2, 1e-3, 1e-3, 400), (1e-2, 1e-3, 1e-12, 17),
             (2e-2, 2e-3, 2e-3, 400)]
    for dt, dtau, tol, maxit in cases:
        outs = []
        for pl in (g, e):
            U = dev(G0)
            rc, it, res = B.fr_dual_step(pl.handle, U, dUn, dUm, dt, dtau, tol, maxit,
                                         check_every=every, raise_on_error=False)
            busy(U)
            torch.cuda.synchronize()
            outs.append((rc, it, res, U))
        (rg, ig, sg, Ug), (re, ie, se, Ue) = outs
        assert (rg, ig) == (re, ie), (dt, tol, maxit)
        assert sg == se or (np.isnan(sg) and np.isnan(se))
        assert torch.equal(Ug, Ue)
        if every == 1 or maxit == 17:
            assert rg == (B.FR_ENOCONV if maxit == 17 else B.FR_OK)
        if maxit == 17:
            assert ig == 17
    # BDF1 (no Unm1) on the same plans: a different key
    for pl_pair in ((g, e),):
        outs = []
        for pl in pl_pair:
            U = dev(Un)
            rc, it, res = B.fr_dual_step(pl.handle, U, dUn, None, 1e-2, 1e-3, 1e-4, 400,
                                         check_every=every, raise_on_error=False)
            torch.cuda.synchronize()
            outs.append((rc, it, res, U))
        assert outs[0][:3] == outs[1][:3]
        assert torch.equal(outs[0][3], outs[1][3])
    g.close()
    e.close()


def test_graph_option_roundtrip():
    pl = B.Plan(1, (2, 2, 2), ZETA, NU, T_CFG)
    assert B.fr_plan_get_int(pl.handle, B.FR_OPT_GRAPH) == 0
    pl.set(B.FR_OPT_GRAPH, 1)
    assert B.fr_plan_get_int(pl.handle, B.FR_OPT_GRAPH) == 1
    with pytest.raises(Exception):
        pl.set(B.FR_OPT_GRAPH, 2)
    pl.close()
