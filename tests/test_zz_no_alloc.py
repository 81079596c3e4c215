"""The allocation-free residual entry point (fr_residual_noalloc), through the
C ABI: the same result as fr_residual on two calls in a row, the second with a
smaller lattice, in both precisions and in the matrix-core variant, against
the CPU oracle too; plans too large for its fixed trace array, and the
unfused variant, are refused before any work is enqueued."""
import numpy as np
import pytest

import oracle
from paper_2107_14027_amd import binding as B
from gpu_util import NU, T_CFG, TOL, ZETA, check_groups, rel, say

pytestmark = pytest.mark.gpu


def rand_U(p, n, seed):
    rng = np.random.default_rng(seed)
    U = 0.3 * rng.standard_normal((n[0] * n[1] * n[2], 13, (p + 1) ** 3))
    U[:, :4] += np.array([1.0, 0.4, -0.3, 0.2])[None, :, None]
    return U


def both(p, n, U, precision, variant, form):
    """fr_residual_noalloc and fr_residual on the same plan and input."""
    import torch
    plan = B.Plan(p, n, ZETA, NU, T_CFG, None, precision, variant)
    plan.set(B.FR_OPT_FORM, form)
    dt = torch.float64 if precision == B.FR_F64 else torch.float32
    Ud = torch.from_numpy(U).to("cuda", dt)
    Rn = torch.full_like(Ud, float("nan"))
    Rr = torch.full_like(Ud, float("nan"))
    B.fr_residual_noalloc(plan.handle, Ud, Rn)
    B.fr_residual(plan.handle, Ud, Rr)
    torch.cuda.synchronize()
    plan.close()
    return Rn.double().cpu().numpy(), Rr.double().cpu().numpy(), Ud.double().cpu().numpy()


@pytest.mark.parametrize("form", [B.FR_FORM_POINT, B.FR_FORM_AUTO])
@pytest.mark.parametrize("precision,variant", [(B.FR_F64, B.FR_FUSED), (B.FR_F32, B.FR_FUSED),
                                               (B.FR_F32, B.FR_MFMA)])
def test_noalloc_matches_residual_two_calls(precision, variant, form):
    # first call on a larger lattice, second on a smaller one: the second must
    # not see anything the first left in the shared array
    for p, n, seed in ((3, (6, 5, 7), 11), (2, (3, 2, 2), 12)):
        say("noalloc p=%d n=%s precision=%d variant=%d form=%d" % (p, n, precision, variant, form))
        U = rand_U(p, n, seed)
        Rn, Rr, Uin = both(p, n, U, precision, variant, form)
        assert np.all(np.isfinite(Rn))
        assert np.array_equal(Rn, Rr), float(np.max(np.abs(Rn - Rr)))
        Ro = oracle.residual(p, n, Uin.reshape(U.shape), ZETA, NU, T_CFG)
        assert rel(Rn.reshape(U.shape), Ro) <= TOL[precision]
        check_groups(Rn.reshape(U.shape), Ro, precision, Uin.reshape(U.shape), what="noalloc")


def test_noalloc_refuses_large_and_unfused():
    import torch
    # p = 3 in FP64: 6 * ne * 112 doubles of traces; 24^3 elements need 92.9 MB > 64 MiB
    # (the point form; the halo form uses no trace array and accepts the plan)
    p, n = 3, (24, 24, 24)
    plan = B.Plan(p, n, ZETA, NU, T_CFG)
    plan.set(B.FR_OPT_FORM, B.FR_FORM_POINT)
    Ud = torch.zeros(plan.state_len, dtype=torch.float64, device="cuda")
    Rd = torch.full_like(Ud, 7.0)
    with pytest.raises(B.FrError) as ei:
        B.fr_residual_noalloc(plan.handle, Ud, Rd)
    assert ei.value.code == B.FR_EINVAL
    plan.set(B.FR_OPT_FORM, B.FR_FORM_HALO)
    Rh = torch.full_like(Ud, 7.0)
    B.fr_residual_noalloc(plan.handle, Ud, Rh)
    torch.cuda.synchronize()
    assert float(Rh.abs().max()) == 0.0   # a zero state has a zero residual
    plan.close()
    plan = B.Plan(2, (2, 2, 2), ZETA, NU, T_CFG, variant=B.FR_UNFUSED)
    Ud = torch.zeros(plan.state_len, dtype=torch.float64, device="cuda")
    Rs = torch.full_like(Ud, 7.0)
    with pytest.raises(B.FrError) as ei:
        B.fr_residual_noalloc(plan.handle, Ud, Rs)
    assert ei.value.code == B.FR_EUNSUPPORTED
    torch.cuda.synchronize()
    # nothing was enqueued: the outputs keep their fill
    assert bool(torch.all(Rd == 7.0)) and bool(torch.all(Rs == 7.0))
    plan.close()
