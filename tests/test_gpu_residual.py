"""GPU parity of the residual (fused and unfused, FP64 and FP32) against the
CPU oracle, through the C ABI, on seeded inputs: several tiles with a ragged
tail for every order, general Jacobians, degenerate lattices, run-to-run
determinism and invariance to the workgroup size."""
import numpy as np
import pytest

import oracle
from paper_2107_14027_amd import binding as B
from paper_2107_14027_amd import inputs
from gpu_util import NU, T_CFG, TOL, ZETA, check_groups, gpu_residual, rel, say

pytestmark = pytest.mark.gpu

def fused_emax(p, prec):
    """Elements per batch of the fused kernel's launch shape for order p."""
    return B.fr_launch_shape(p, B.FR_F64 if prec == "D" else B.FR_F32, B.FR_K_FUSED)[0]


SKEW = np.array([[0.30, 0.05, -0.02], [0.01, 0.25, 0.04], [-0.03, 0.02, 0.35]])
PREC = [B.FR_F64, B.FR_F32]
VAR = [B.FR_FUSED, B.FR_UNFUSED]


def rand_U(p, n, seed):
    rng = np.random.default_rng(seed)
    U = 0.3 * rng.standard_normal((n[0] * n[1] * n[2], 13, (p + 1) ** 3))
    U[:, :4] += np.array([1.0, 0.4, -0.3, 0.2])[None, :, None]
    return U


@pytest.mark.parametrize("prec", PREC)
@pytest.mark.parametrize("var", VAR)
def test_config1_tgv_noise(prec, var):
    """4^3 periodic box, p = 2, Taylor-Green + N(0, 1e-3) noise, zeta = 4."""
    p, n = 2, (4, 4, 4)
    U = inputs.tgv(p, n, noise=1e-3, seed=20210729)
    say("config1 prec=%d var=%d" % (prec, var))
    R = gpu_residual(p, n, U, precision=prec, variant=var)
    Ro = oracle.residual(p, n, U, ZETA, NU, T_CFG)
    assert rel(R, Ro) <= TOL[prec]
    check_groups(R, Ro, prec, U, what="config1")


# lattices sized so that every order spans several workgroups with a ragged tail
CASES = [(1, (5, 3, 4)), (2, (3, 5, 2)), (3, (3, 2, 5)), (4, (2, 3, 3)), (5, (3, 1, 2)),
         (6, (1, 2, 3))]


@pytest.mark.parametrize("p,n", CASES)
@pytest.mark.parametrize("prec", PREC)
@pytest.mark.parametrize("var", VAR)
@pytest.mark.parametrize("jac", [None, "skew"])
def test_orders_ragged(p, n, prec, var, jac):
    J = SKEW if jac == "skew" else None
    U = rand_U(p, n, seed=100 + p)
    say("orders p=%d n=%s prec=%d var=%d jac=%s" % (p, n, prec, var, jac))
    R = gpu_residual(p, n, U, precision=prec, variant=var, jac=J)
    Ro = oracle.residual(p, n, U, ZETA, NU, T_CFG, J)
    assert rel(R, Ro) <= TOL[prec], rel(R, Ro)
    check_groups(R, Ro, prec, U, what="p=%d jac=%s" % (p, jac))


FORMS = [B.FR_FORM_POINT, B.FR_FORM_LINES, B.FR_FORM_HALO]


@pytest.mark.parametrize("p,n", CASES)
@pytest.mark.parametrize("prec", PREC)
@pytest.mark.parametrize("form", FORMS)
def test_forms_ragged(p, n, prec, form):
    """Both kernel forms of the fused residual against the oracle (diagonal
    Jacobian: the periodic box)."""
    U = rand_U(p, n, seed=300 + p)
    say("forms p=%d n=%s prec=%d form=%d" % (p, n, prec, form))
    R = gpu_residual(p, n, U, precision=prec, form=form)
    Ro = oracle.residual(p, n, U, ZETA, NU, T_CFG)
    assert rel(R, Ro) <= TOL[prec], rel(R, Ro)
    check_groups(R, Ro, prec, U, what="p=%d form=%d" % (p, form))


@pytest.mark.parametrize("form", [B.FR_FORM_LINES, B.FR_FORM_HALO])
def test_line_forms_need_diagonal_jacobian(form):
    with pytest.raises(B.FrError) as ei:
        gpu_residual(2, (2, 2, 2), rand_U(2, (2, 2, 2), 1), jac=SKEW, form=form)
    assert ei.value.code == B.FR_EUNSUPPORTED


@pytest.mark.parametrize("n", [(1, 1, 1), (1, 2, 1), (2, 1, 1)])
@pytest.mark.parametrize("prec", PREC)
def test_degenerate_lattices(n, prec):
    """An element can be its own neighbour across a periodic face."""
    p = 3
    U = rand_U(p, n, seed=7)
    say("degenerate n=%s prec=%d" % (n, prec))
    for var, form in ((B.FR_FUSED, B.FR_FORM_POINT), (B.FR_FUSED, B.FR_FORM_LINES),
                      (B.FR_FUSED, B.FR_FORM_HALO), (B.FR_UNFUSED, B.FR_FORM_AUTO)):
        R = gpu_residual(p, n, U, precision=prec, variant=var, form=form)
        Ro = oracle.residual(p, n, U, ZETA, NU, T_CFG)
        assert rel(R, Ro) <= TOL[prec]
        check_groups(R, Ro, prec, U, what="degenerate")


@pytest.mark.parametrize("p", [2, 4, 6])
@pytest.mark.parametrize("prec", PREC)
def test_unfused_odd_lengths(p, prec):
    """13 ne m^3 odd: the unfused pipeline's last stage runs 16-byte vectors
    that straddle two variables' blocks and a scalar tail, in both precisions."""
    n = (3, 1, 1)
    U = rand_U(p, n, seed=500 + p)
    say("unfused odd length p=%d prec=%d" % (p, prec))
    R = gpu_residual(p, n, U, precision=prec, variant=B.FR_UNFUSED)
    Ro = oracle.residual(p, n, U, ZETA, NU, T_CFG)
    assert rel(R, Ro) <= TOL[prec], rel(R, Ro)
    check_groups(R, Ro, prec, U, what="odd length p=%d" % p)


def test_free_stream_and_paper_T():
    """Uniform state gives a zero residual; the paper's own T = 5e-3, zeta = 2.5."""
    p, n = 4, (3, 2, 2)
    vals = np.zeros(13)
    vals[:4] = [1.3, 0.4, -0.7, 0.2]
    U = inputs.uniform(p, n, vals)
    say("free stream")
    R = gpu_residual(p, n, U, zeta=2.5, T=5e-3, jac=SKEW)
    assert np.max(np.abs(R)) < 1e-12
    U = inputs.tgv(p, n, noise=1e-3, seed=1)
    R = gpu_residual(p, n, U, zeta=2.5, T=5e-3)
    Ro = oracle.residual(p, n, U, 2.5, NU, 5e-3)
    assert rel(R, Ro) <= 1e-12
    check_groups(R, Ro, B.FR_F64, U, zeta=2.5, T=5e-3, what="paper T")


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_block_size_invariance_and_determinism(p):
    """FP64 results do not depend on elements per workgroup and repeat bitwise."""
    n = (4, 3, 3) if p < 5 else (2, 2, 3)
    U = rand_U(p, n, seed=11)
    say("block invariance p=%d" % p)
    pt = B.FR_FORM_POINT
    ref = gpu_residual(p, n, U, form=pt)
    again = gpu_residual(p, n, U, form=pt)
    assert np.array_equal(ref, again)
    emax = fused_emax(p, "D")   # largest batch the point-form kernel accepts
    for E in (1, 2, 3):
        if E <= emax:
            assert np.array_equal(gpu_residual(p, n, U, block=E, form=pt), ref), E
    with pytest.raises(B.FrError):
        gpu_residual(p, n, U, block=emax + 1, form=pt)
    lines = gpu_residual(p, n, U, form=B.FR_FORM_LINES)
    assert np.array_equal(lines, gpu_residual(p, n, U, form=B.FR_FORM_LINES))
    assert rel(lines, ref) <= 1e-13
    # the halo form forms the neighbours' traces itself with the trace kernel's
    # arithmetic: the same bits as the line form
    assert np.array_equal(gpu_residual(p, n, U, form=B.FR_FORM_HALO), lines)


def test_auto_form_choice_is_reported():
    """FR_INFO_RESIDUAL_FORM names the kernel form fr_residual runs: the halo
    form at the orders the automatic choice documents (every order, diagonal
    Jacobian), else the point form; 0 for the unfused and matrix-core
    variants."""
    halo = {B.FR_F64: {1, 2, 3, 4, 5, 6}, B.FR_F32: {1, 2, 3, 4, 5, 6}}
    for prec in PREC:
        for p in range(1, 7):
            plan = B.Plan(p, (2, 2, 2), ZETA, NU, T_CFG, precision=prec)
            want = B.FR_FORM_HALO if p in halo[prec] else B.FR_FORM_POINT
            assert B.fr_plan_get_int(plan.handle, B.FR_INFO_RESIDUAL_FORM) == want, (prec, p)
            plan.set(B.FR_OPT_FORM, B.FR_FORM_POINT)
            assert B.fr_plan_get_int(plan.handle, B.FR_INFO_RESIDUAL_FORM) == B.FR_FORM_POINT
            plan.close()
            plan = B.Plan(p, (2, 2, 2), ZETA, NU, T_CFG, SKEW, prec)
            assert B.fr_plan_get_int(plan.handle, B.FR_INFO_RESIDUAL_FORM) == B.FR_FORM_POINT
            plan.close()
    plan = B.Plan(3, (2, 2, 2), ZETA, NU, T_CFG, variant=B.FR_UNFUSED)
    assert B.fr_plan_get_int(plan.handle, B.FR_INFO_RESIDUAL_FORM) == 0
    plan.close()
