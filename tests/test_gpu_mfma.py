"""GPU parity of the matrix-core variant (FR_MFMA: the partially corrected
divergence and the correction on v_mfma_f32_16x16x4f32, single-precision
operands and accumulation) against the CPU oracle on the single-precision
state, through the C ABI: every order on ragged lattices, cubic and general
Jacobians, the Taylor-Green configuration with noise, RK4 steps, agreement
with the VALU single-precision kernel, the precision it rejects, and the
design order of accuracy on the manufactured solution sin x sin y sin z at
p = 4 for n = 4 .. 32."""
import math

import numpy as np
import pytest

import oracle
from paper_2107_14027_amd import binding as B
from paper_2107_14027_amd import inputs
from gpu_util import NU, T_CFG, TOL, ZETA, check_groups, gpu_residual, rel, say
from test_oracle_residual import sines_exact_residual

pytestmark = pytest.mark.gpu

SKEW = np.array([[0.30, 0.05, -0.02], [0.01, 0.25, 0.04], [-0.03, 0.02, 0.35]])
CASES = [(1, (5, 3, 4)), (2, (3, 5, 2)), (3, (3, 2, 5)), (4, (2, 3, 3)), (5, (3, 1, 2)),
         (6, (1, 2, 3))]
F32 = B.FR_F32


def rand_U(p, n, seed):
    rng = np.random.default_rng(seed)
    U = 0.3 * rng.standard_normal((n[0] * n[1] * n[2], 13, (p + 1) ** 3))
    U[:, :4] += np.array([1.0, 0.4, -0.3, 0.2])[None, :, None]
    return U


def r32(U):
    """The state the single-precision kernel receives."""
    return U.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("p,n", CASES)
@pytest.mark.parametrize("jac", [None, "skew"])
def test_mfma_orders_ragged(p, n, jac):
    J = SKEW if jac == "skew" else None
    U = rand_U(p, n, seed=100 + p)
    say("mfma p=%d n=%s jac=%s" % (p, n, jac))
    R = gpu_residual(p, n, U, precision=F32, variant=B.FR_MFMA, jac=J)
    Ro = oracle.residual(p, n, r32(U), ZETA, NU, T_CFG, J)
    say("  rel %.2e" % rel(R, Ro))
    assert rel(R, Ro) <= TOL[F32]
    check_groups(R, Ro, F32, U, what="mfma p=%d jac=%s" % (p, jac))
    # the VALU single-precision kernel: both within single-precision rounding
    Rv = gpu_residual(p, n, U, precision=F32, variant=B.FR_FUSED, jac=J)
    assert rel(R, Rv) <= 2 * TOL[F32]


def test_mfma_config1_tgv_noise():
    p, n = 2, (4, 4, 4)
    U = inputs.tgv(p, n, noise=1e-3, seed=20210729)
    say("mfma config1")
    R = gpu_residual(p, n, U, precision=F32, variant=B.FR_MFMA)
    Ro = oracle.residual(p, n, r32(U), ZETA, NU, T_CFG)
    assert rel(R, Ro) <= TOL[F32]
    check_groups(R, Ro, F32, U, what="mfma config1")


def test_mfma_needs_single_precision():
    import torch
    plan = B.Plan(3, (2, 2, 2), ZETA, NU, T_CFG, precision=B.FR_F64, variant=B.FR_MFMA)
    U = torch.zeros(plan.state_len, dtype=torch.float64, device="cuda")
    with pytest.raises(B.FrError) as e:
        B.fr_residual(plan.handle, U, torch.empty_like(U))
    assert "(-6)" in str(e.value) and "single precision" in str(e.value)
    plan.close()


def test_mfma_rk4_steps():
    """RK4 with the matrix-core residual (separate stage kernel) against the oracle."""
    import torch
    p, n = 2, (4, 4, 4)
    U0 = inputs.tgv(p, n, noise=1e-3, seed=20210729)
    plan = B.Plan(p, n, ZETA, NU, T_CFG, precision=F32, variant=B.FR_MFMA)
    Ud = torch.from_numpy(U0.copy()).to("cuda")
    say("mfma rk4")
    B.fr_rk_step(plan.handle, Ud, 1e-3, 10)
    torch.cuda.synchronize()
    Uo = oracle.rk4(p, n, U0, ZETA, NU, T_CFG, 1e-3, 10)
    G = Ud.cpu().numpy()
    assert rel(G, Uo) <= 1e-5
    assert rel(G - U0, Uo - U0) <= 1e-4
    plan.close()


def test_mfma_manufactured_convergence_p4():
    """Config 4's field P = u = v = w = sin x sin y sin z at p = 4: the max-norm
    error of the matrix-core residual against the closed-form operator falls at
    the design rate while it is above single-precision rounding (n = 4 .. 16),
    and sits at that rounding level at n = 32 (the double-precision path's
    truncation error there is about 3e-6, the single-precision input rounding
    alone about 5e-5)."""
    p = 4
    errs, scale = [], 0.0
    ns = (4, 8, 16, 32)
    for nn in ns:
        n = (nn, nn, nn)
        U = inputs.sines(p, n)
        E = sines_exact_residual(p, n)
        R = gpu_residual(p, n, U, precision=F32, variant=B.FR_MFMA)
        errs.append(float(np.max(np.abs(R[:, :4] - E[:, :4]))))
        scale = max(scale, float(np.max(np.abs(E[:, :4]))))
    rates = [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(3)]
    say("mfma p=4 convergence errors %s rates %s" % (errs, rates))
    assert rates[0] > p - 0.2, (errs, rates)
    assert rates[1] > p - 1.0, (errs, rates)
    assert errs[3] < errs[1] and errs[3] <= 1e-4 * scale, (errs, rates)
