"""The RK4 stage update applied in the fused kernel's epilogue (no residual
array) against the residual kernel followed by the separate stage kernel: the
states must carry the same bits, for RK4 and for dual time stepping (BDF
source on the velocity, pseudo-residual norm), every order, both precisions,
diagonal and general Jacobians, and ragged lattices whose last workgroup batch
is partial.  The dual step's norm is summed per workgroup in the epilogue, so
only its rounding may differ."""
import numpy as np
import pytest

from paper_2107_14027_amd import binding as B
from paper_2107_14027_amd import inputs
from gpu_util import NU, T_CFG, ZETA, say

pytestmark = pytest.mark.gpu
SKEW = np.array([[0.30, 0.05, -0.02], [0.01, 0.25, 0.04], [-0.03, 0.02, 0.35]])


def dev(U):
    import torch
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda")


def pair(p, n, prec, jac, form=B.FR_FORM_POINT):
    """Two plans of the same residual form (point: k_fused; halo: the line
    tasks that form the neighbours' traces themselves), with and without the
    stage epilogue."""
    out = []
    for fuse in (1, 0):
        pl = B.Plan(p, n, ZETA, NU, T_CFG, jac, prec, B.FR_FUSED)
        pl.set(B.FR_OPT_FUSE_STAGE, fuse)
        pl.set(B.FR_OPT_FORM, form)
        out.append(pl)
    return out


FORMS = [B.FR_FORM_POINT, B.FR_FORM_HALO]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("prec", [B.FR_F64, B.FR_F32])
@pytest.mark.parametrize("p,n,jac", [(1, (5, 3, 4), None), (2, (3, 4, 5), None), (3, (5, 3, 3), None),
                                     (4, (3, 2, 3), None), (5, (2, 3, 2), None), (6, (2, 2, 3), None),
                                     (3, (3, 4, 2), "skew"), (6, (2, 1, 2), "skew"),
                                     (1, (37, 2, 3), None)])
def test_rk_epilogue_bitwise(form, prec, p, n, jac):
    import torch
    if jac and form == B.FR_FORM_HALO:
        pytest.skip("the halo form needs a diagonal Jacobian")
    J = SKEW if jac else None
    U0 = inputs.tgv(p, n, noise=1e-3, seed=p)
    g, e = pair(p, n, prec, J, form)
    say("rk epilogue form=%d p=%d n=%s prec=%d jac=%s" % (form, p, n, prec, jac))
    Ug, Ue = dev(U0), dev(U0)
    for dt, steps in ((1e-3, 3), (2e-3, 2)):
        B.fr_rk_step(g.handle, Ug, dt, steps)
        B.fr_rk_step(e.handle, Ue, dt, steps)
        torch.cuda.synchronize()
        assert torch.equal(Ug, Ue), (dt, steps)
    assert not torch.equal(Ug, dev(U0))
    g.close()
    e.close()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("prec", [B.FR_F64, B.FR_F32])
@pytest.mark.parametrize("p,n,every,tol", [(2, (3, 2, 4), 1, 1e-3), (3, (2, 3, 3), 3, 1e-3),
                                           (6, (2, 1, 2), 2, 3e-3), (1, (6, 5, 4), 1, 1e-3)])
def test_dual_epilogue_bitwise(form, prec, p, n, every, tol):
    import torch
    g, e = pair(p, n, prec, None, form)
    say("dual epilogue form=%d p=%d n=%s prec=%d every=%d" % (form, p, n, prec, every))
    Unm1 = inputs.tgv(p, n, noise=1e-4, seed=7)
    dUm = dev(Unm1)
    dUn = dUm.clone()
    B.fr_rk_step(e.handle, dUn, 2.5e-3, 4)
    torch.cuda.synchronize()
    G0 = (2 * dUn - dUm).cpu().numpy()
    for Um, tol, maxit in ((dUm, tol, 500), (None, tol, 500), (dUm, 1e-12, 9)):
        outs = []
        for pl in (g, e):
            U = dev(G0)
            rc, it, res = B.fr_dual_step(pl.handle, U, dUn, Um, 1e-2, 1e-3, tol, maxit,
                                         check_every=every, raise_on_error=False)
            torch.cuda.synchronize()
            outs.append((rc, it, res, U))
        (rg, ig, sg, Ug), (re, ie, se, Ue) = outs
        assert (rg, ig) == (re, ie), (Um is None, tol)
        assert abs(sg - se) <= 1e-12 * abs(se)
        assert torch.equal(Ug, Ue)
        assert rg == (B.FR_ENOCONV if maxit == 9 else B.FR_OK)
    g.close()
    e.close()


@pytest.mark.parametrize("prec", [B.FR_F64, B.FR_F32])
def test_halo_epilogue_workgroups_take_several_batches(prec):
    """More batches than the epilogue has partial sums (8192): each workgroup
    of the halo form's stage epilogue then updates several batches."""
    import torch
    p, n = 1, (64, 64, 40)
    g, e = pair(p, n, prec, None, B.FR_FORM_HALO)
    say("halo epilogue, several batches per workgroup, prec=%d" % prec)
    U0 = inputs.tgv(p, n, noise=1e-3, seed=11)
    Ug, Ue = dev(U0), dev(U0)
    B.fr_rk_step(g.handle, Ug, 1e-3, 2)
    B.fr_rk_step(e.handle, Ue, 1e-3, 2)
    torch.cuda.synchronize()
    assert torch.equal(Ug, Ue)
    outs = []
    for pl in (g, e):
        U = Ue.clone()
        rc, it, res = B.fr_dual_step(pl.handle, U, Ue, None, 1e-2, 1e-3, 1e-12, 3,
                                     check_every=1, raise_on_error=False)
        torch.cuda.synchronize()
        outs.append((rc, it, res, U))
    (rg, ig, sg, Ugd), (re_, ie, se, Ued) = outs
    assert (rg, ig) == (re_, ie) and rg == B.FR_ENOCONV
    assert abs(sg - se) <= 1e-12 * abs(se)
    assert torch.equal(Ugd, Ued)
    g.close()
    e.close()


# FR_FORM_AUTO's stage path per order (diagonal Jacobian), as documented
AUTO_STAGE = {B.FR_F64: {1: B.FR_STAGE_HALO, 2: B.FR_STAGE_HALO, 3: B.FR_STAGE_HALO,
                         4: B.FR_STAGE_POINT, 5: B.FR_STAGE_HALO, 6: B.FR_STAGE_HALO},
              B.FR_F32: {1: B.FR_STAGE_HALO, 2: B.FR_STAGE_HALO, 3: B.FR_STAGE_HALO,
                         4: B.FR_STAGE_HALO, 5: B.FR_STAGE_POINT, 6: B.FR_STAGE_HALO}}


@pytest.mark.parametrize("prec", [B.FR_F64, B.FR_F32])
def test_auto_stage_path_is_reported_and_runs(prec):
    """FR_INFO_STAGE_PATH names what fr_rk_step runs, and the automatic choice
    gives the bits of the explicit form it names."""
    import torch
    for p in range(1, 7):
        n = (3, 2, 2)
        auto = B.Plan(p, n, ZETA, NU, T_CFG, None, prec, B.FR_FUSED)
        path = B.fr_plan_get_int(auto.handle, B.FR_INFO_STAGE_PATH)
        assert path == AUTO_STAGE[prec][p], (p, path)
        ref = B.Plan(p, n, ZETA, NU, T_CFG, None, prec, B.FR_FUSED)
        if path == B.FR_STAGE_SEPARATE:
            ref.set(B.FR_OPT_FUSE_STAGE, 0)
        else:
            ref.set(B.FR_OPT_FORM, B.FR_FORM_HALO if path == B.FR_STAGE_HALO else B.FR_FORM_POINT)
        assert B.fr_plan_get_int(ref.handle, B.FR_INFO_STAGE_PATH) == path
        say("auto stage path p=%d prec=%d path=%d" % (p, prec, path))
        U0 = inputs.tgv(p, n, noise=1e-3, seed=p + 20)
        Ua, Ur = dev(U0), dev(U0)
        B.fr_rk_step(auto.handle, Ua, 1e-3, 2)
        B.fr_rk_step(ref.handle, Ur, 1e-3, 2)
        torch.cuda.synchronize()
        assert torch.equal(Ua, Ur), p
        auto.set(B.FR_OPT_FUSE_STAGE, 0)
        assert B.fr_plan_get_int(auto.handle, B.FR_INFO_STAGE_PATH) == B.FR_STAGE_SEPARATE
        auto.close()
        ref.close()
    pl = B.Plan(3, (2, 2, 2), ZETA, NU, T_CFG, SKEW, prec, B.FR_FUSED)
    assert B.fr_plan_get_int(pl.handle, B.FR_INFO_STAGE_PATH) == B.FR_STAGE_POINT
    pl.close()
    pl = B.Plan(3, (2, 2, 2), ZETA, NU, T_CFG, None, prec, B.FR_UNFUSED)
    assert B.fr_plan_get_int(pl.handle, B.FR_INFO_STAGE_PATH) == B.FR_STAGE_SEPARATE
    pl.close()


def test_fuse_stage_option():
    pl = B.Plan(1, (2, 2, 2), ZETA, NU, T_CFG)
    assert B.fr_plan_get_int(pl.handle, B.FR_OPT_FUSE_STAGE) == 1
    pl.set(B.FR_OPT_FUSE_STAGE, 0)
    assert B.fr_plan_get_int(pl.handle, B.FR_OPT_FUSE_STAGE) == 0
    with pytest.raises(Exception):
        pl.set(B.FR_OPT_FUSE_STAGE, 3)
    pl.close()
