"""The trained network against the method without it: a short dual-time run
(Taylor-Green, p = 3 on 16^3 hexes, dt = 5e-2, dtau = dt/10, tol 1e-6) trains
the pointwise network on solver-generated steps with the library's own
forward/backward/Adam kernels, then runs the same evaluation steps from the
identical state with quadratic extrapolation, linear extrapolation and the
network (correcting the linear extrapolation).  The converged residual decides
every step, so only the number of pseudo-iterations may change."""
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_learned_guess_cuts_pseudo_iterations():
    from paper_2107_14027_amd import learned
    say("learned guess study (short)")
    r = learned.run(train_steps=12, eval_steps=8, epochs=600, guess_base=1)
    m = r["modes"]
    for mode in ("extrap", "extrap1", "mlp"):
        assert m[mode]["capped"] == 0, (mode, m[mode]["iters"])
    # training lowered the normalised loss well below the zero network's 1.0
    assert r["loss_curve"][-1][1] < 0.5 * r["loss_curve"][0][1], r["loss_curve"]
    # fewer pseudo-iterations than the quadratic extrapolation it replaces (about
    # 22% fewer after this short training; 66% after 20 training steps and 2000
    # Adam steps), and within 10% of linear extrapolation
    assert m["mlp"]["iters_mean"] < 0.9 * m["extrap"]["iters_mean"], m
    assert m["mlp"]["iters_mean"] <= 1.1 * m["extrap1"]["iters_mean"], m


def test_learned_guess_with_pmg_solver():
    """The default study with P-multigrid cycles as the solver (counts are
    cycles; about 20 s).  Measured: 16.5 cycles with the network, 19.3 with
    linear and 62.6 with quadratic extrapolation."""
    from paper_2107_14027_amd import learned
    say("learned guess study, P-multigrid")
    r = learned.run(guess_base=1, solver="pmg")
    m = r["modes"]
    for mode in ("extrap", "extrap1", "mlp"):
        assert m[mode]["capped"] == 0, (mode, m[mode]["iters"])
    assert m["mlp"]["iters_mean"] < 0.5 * m["extrap"]["iters_mean"], m
    assert m["mlp"]["iters_mean"] < 0.95 * m["extrap1"]["iters_mean"], m
