"""GPU parity of RK34 pseudo-stepping with locally adaptive steps
(FR_OPT_PSEUDO = 1) against the oracle (oracle/rk34.py, oracle/pmg.py): fixed
numbers of pseudo-steps compared element by element, converged steps, the
step field carried from one call to the next, and inside P-multigrid cycles."""
import numpy as np
import pytest

import oracle
from oracle import pmg as opmg
from paper_2107_14027_amd import binding as B
from paper_2107_14027_amd import inputs
from gpu_util import NU, T_CFG, ZETA, rel, say

pytestmark = pytest.mark.gpu


def dev(U):
    import torch
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda")


def case(P, n, seed=1):
    Unm1 = inputs.tgv(P, n, noise=1e-4, seed=seed)
    Un = oracle.rk4(P, n, Unm1, ZETA, NU, T_CFG, 2.5e-3, 4)
    return 2 * Un - Unm1, Un, Unm1


def plan34(P, n, prec=B.FR_F64, var=B.FR_FUSED):
    pl = B.Plan(P, n, ZETA, NU, T_CFG, None, prec, var)
    pl.set(B.FR_OPT_PSEUDO, 1)
    return pl


def dual(pl, G, Un, Unm1, dt, dtau, tol, maxit):
    import torch
    U = dev(G)
    rc, it, res = B.fr_dual_step(pl.handle, U, dev(Un), None if Unm1 is None else dev(Unm1), dt, dtau,
                                 tol, maxit, raise_on_error=False)
    torch.cuda.synchronize()
    return U.cpu().numpy().reshape(-1), rc, it, res


@pytest.mark.parametrize("P,n,bdf2", [(2, (3, 2, 4), True), (3, (2, 3, 2), True), (3, (2, 2, 3), False)])
def test_fixed_steps_match_oracle(P, n, bdf2):
    G, Un, Unm1 = case(P, n)
    Um = Unm1 if bdf2 else None
    say("rk34 fixed P=%d n=%s bdf2=%s" % (P, n, bdf2))
    pl = plan34(P, n)
    Ug, rc, it, res = dual(pl, G, Un, Um, 1e-2, 1e-3, 1e-30, 25)
    Uo, ito, reso, rco, h = opmg.dual_step_local(P, n, G, Un, Um, ZETA, NU, T_CFG, 1e-2, 1e-3, 1e-30, 25)
    assert rc == B.FR_ENOCONV and rco == -5 and it == ito == 25
    assert rel(Ug, Uo) <= 1e-11
    assert rel(Ug - G.reshape(-1), Uo - G.reshape(-1)) <= 1e-9
    assert abs(res - reso) <= 1e-9 * reso
    pl.close()


@pytest.mark.parametrize("var", [B.FR_FUSED, B.FR_UNFUSED])
def test_fp32_and_unfused(var):
    P, n = 3, (3, 2, 2)
    G, Un, Unm1 = case(P, n, seed=3)
    say("rk34 fp32 var=%d" % var)
    Uo, _, reso, _, _ = opmg.dual_step_local(P, n, G, Un, Unm1, ZETA, NU, T_CFG, 1e-2, 1e-3, 1e-30, 20)
    pl = plan34(P, n, B.FR_F32, var)
    U32, rc, it, res = dual(pl, G, Un, Unm1, 1e-2, 1e-3, 1e-30, 20)
    assert it == 20 and rel(U32, Uo) <= 1e-5
    pl.close()
    pl = plan34(P, n, B.FR_F64, var)
    U64, rc, it, res = dual(pl, G, Un, Unm1, 1e-2, 1e-3, 1e-30, 20)
    assert rel(U64, Uo) <= 1e-11
    pl.close()


def test_converged():
    P, n = 3, (2, 2, 2)
    G, Un, Unm1 = case(P, n, seed=2)
    tol = 1.2e-3
    say("rk34 converged")
    pl = plan34(P, n)
    Ug, rc, it, res = dual(pl, G, Un, Unm1, 1e-2, 1e-3, tol, 2000)
    Uo, ito, reso, rco, h = opmg.dual_step_local(P, n, G, Un, Unm1, ZETA, NU, T_CFG, 1e-2, 1e-3, tol, 2000)
    assert rc == B.FR_OK and rco == 0 and res < tol
    assert abs(it - ito) <= 1
    if it == ito:
        assert rel(Ug, Uo) <= 1e-11
    pl.close()


def test_field_carried_over():
    """Two physical steps on one plan: the second starts from the step field the
    first left (the oracle is handed the same field); a different initial step
    resets it."""
    P, n = 3, (2, 2, 2)
    G, Un, Unm1 = case(P, n, seed=6)
    say("rk34 carried field")
    pl = plan34(P, n)
    Ug, rc, it, res = dual(pl, G, Un, Unm1, 1e-2, 1e-3, 1e-30, 15)
    Uo, ito, reso, rco, h = opmg.dual_step_local(P, n, G, Un, Unm1, ZETA, NU, T_CFG, 1e-2, 1e-3, 1e-30, 15)
    assert it == ito == 15 and rel(Ug, Uo) <= 1e-11
    G2 = 2 * Uo - Un.reshape(-1)
    Ug2, rc2, it2, res2 = dual(pl, G2, Uo, Un, 1e-2, 1e-3, 1e-30, 12)
    Uo2, ito2, _, _, _ = opmg.dual_step_local(P, n, G2, Uo, Un, ZETA, NU, T_CFG, 1e-2, 1e-3, 1e-30, 12,
                                              h=h)
    assert it2 == ito2 == 12
    assert rel(Ug2, Uo2) <= 1e-11
    Ug3, _, _, _ = dual(pl, G2, Uo, Un, 1e-2, 2e-3, 1e-30, 5)
    Uo3, _, _, _, _ = opmg.dual_step_local(P, n, G2, Uo, Un, ZETA, NU, T_CFG, 1e-2, 2e-3, 1e-30, 5)
    assert rel(Ug3, Uo3) <= 1e-11
    pl.close()


def test_pmg_with_rk34_matches_oracle():
    import torch
    P, n = 3, (2, 3, 2)
    G, Un, Unm1 = case(P, n, seed=5)
    say("pmg + rk34")
    pl = plan34(P, n)
    mg = B.Pmg(pl)
    U = dev(G)
    rc, cyc, res = mg.dual_step(U, dev(Un), dev(Unm1), 1e-2, 1e-3, 1e-30, 2, raise_on_error=False)
    torch.cuda.synchronize()
    Uo, co, reso, rco = opmg.pmg_dual_step(P, n, G, Un, Unm1, ZETA, NU, T_CFG, 1e-2, 1e-3, 1e-30, 2,
                                           scheme="rk34")
    assert cyc == co == 2
    assert rel(U.cpu().numpy().reshape(-1), Uo) <= 1e-11
    mg.close()
    pl.close()


def test_option_roundtrip():
    pl = B.Plan(1, (2, 2, 2), ZETA, NU, T_CFG)
    assert B.fr_plan_get_int(pl.handle, B.FR_OPT_PSEUDO) == 0
    pl.set(B.FR_OPT_PSEUDO, 1)
    assert B.fr_plan_get_int(pl.handle, B.FR_OPT_PSEUDO) == 1
    with pytest.raises(B.FrError):
        pl.set(B.FR_OPT_PSEUDO, 2)
    pl.close()
