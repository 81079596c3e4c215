"""GPU parity of the learned initial guess (pointwise 12-64-64-4 network on
BF16 matrix cores) through the C ABI: forward and gradients against the CPU
oracle in its bfloat16-operand mode (every matrix-product operand rounded,
double accumulation) to 1e-3 relative, Adam against the oracle, training rows
and normalisation against numpy, and the guess against extrapolation."""
import numpy as np
import pytest

import oracle
from paper_2107_14027_amd import binding as B
from paper_2107_14027_amd import inputs
from gpu_util import NU, T_CFG, ZETA, say

pytestmark = pytest.mark.gpu
NAMES = [k for k, _ in B.MLP_SHAPES]


def torch():
    import torch as t
    return t


def random_state(seed, scale=0.3):
    t = torch()
    st = B.mlp_new_state(seed)
    rng = np.random.default_rng(seed)
    P = B.mlp_params(st)
    for k, shp in B.MLP_SHAPES:
        P[k].copy_(t.tensor(rng.standard_normal(shp) * scale, dtype=t.float32))
    st[5252:5264] = t.tensor(rng.standard_normal(12) * 0.1, dtype=t.float32)          # mu
    st[5264:5276] = t.tensor(1.0 + 0.5 * rng.random(12), dtype=t.float32)            # inv_sd
    st[5276:5280] = t.tensor(0.5 + rng.random(4), dtype=t.float32)                    # y_sd
    return st


def host_params(st):
    return {k: v.double().cpu().numpy() for k, v in B.mlp_params(st).items()}


def norm_x(st, X):
    s = st.cpu().numpy()
    mu, isd = s[5252:5264], s[5264:5276]
    return ((X.astype(np.float32) - mu) * isd).astype(np.float32)


def test_init_state():
    st = B.mlp_new_state(7).cpu().numpy()
    assert st.size == B.fr_mlp_state_floats()
    P = B.mlp_params(B.mlp_new_state(7))
    assert float(P["W3"].abs().max()) == 0.0 and float(P["b3"].abs().max()) == 0.0
    assert np.all(st[5264:5276] == 1.0) and np.all(st[5276:5280] == 1.0)
    assert 0.1 < np.abs(st[:768]).max() <= np.sqrt(6.0 / 76) + 1e-6


@pytest.mark.parametrize("n", [1, 37, 4096 + 5])
def test_forward_matches_oracle(n):
    t = torch()
    plan = B.Plan(2, (2, 2, 2), ZETA, NU, T_CFG)
    st = random_state(11)
    rng = np.random.default_rng(n)
    X = (rng.standard_normal((n, 12)) * 0.8).astype(np.float32)
    Xd = t.tensor(X, device="cuda")
    Yd = t.zeros((n, 4), dtype=t.float32, device="cuda")
    say("mlp forward n=%d" % n)
    B.fr_mlp_forward(plan.handle, st, Xd, Yd)
    t.cuda.synchronize()
    y = Yd.cpu().numpy()
    xn = norm_x(st, X)
    # the oracle rounds every matrix-product operand to bfloat16 itself
    yo = oracle.mlp_forward(xn, host_params(st), bf16_operands=True)
    err = np.max(np.abs(y - yo)) / max(1.0, np.abs(yo).max())
    say("  max error %.2e" % err)
    assert err <= 1e-3
    plan.close()


def test_gradients_match_oracle():
    t = torch()
    plan = B.Plan(2, (2, 2, 2), ZETA, NU, T_CFG)
    st = random_state(12)
    n = 3000
    rng = np.random.default_rng(5)
    X = (rng.standard_normal((n, 12)) * 0.8).astype(np.float32)
    Y = (rng.standard_normal((n, 4)) * 0.7).astype(np.float32)
    g = t.zeros(B.MLP_NPAR, dtype=t.float32, device="cuda")
    loss = t.zeros(1, dtype=t.float32, device="cuda")
    say("mlp gradients")
    B.fr_mlp_grad(plan.handle, st, t.tensor(X, device="cuda"), t.tensor(Y, device="cuda"), g, loss)
    t.cuda.synchronize()
    s = st.cpu().numpy()
    ysd = s[5276:5280]
    lo, go = oracle.mlp_loss_grad(norm_x(st, X), Y / ysd, host_params(st),
                                  bf16_operands=True)
    say("  loss %.6e oracle %.6e" % (float(loss.item()), lo))
    assert abs(float(loss.item()) - lo) <= 1e-3 * lo
    gg = g.cpu().numpy()
    o = 0
    for k, shp in B.MLP_SHAPES:
        sz = int(np.prod(shp))
        a, b = gg[o:o + sz].reshape(shp), go[k]
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        say("  grad %s rel %.2e" % (k, e))
        assert e <= 1e-3, k
        o += sz
    # deterministic: the fixed-order reduction repeats bitwise
    g2 = t.zeros_like(g)
    B.fr_mlp_grad(plan.handle, st, t.tensor(X, device="cuda"), t.tensor(Y, device="cuda"), g2)
    t.cuda.synchronize()
    assert t.equal(g, g2)
    plan.close()


def test_train_step_is_adam_on_the_gradient():
    t = torch()
    plan = B.Plan(2, (2, 2, 2), ZETA, NU, T_CFG)
    st = random_state(13)
    n = 1024
    rng = np.random.default_rng(6)
    Xd = t.tensor((rng.standard_normal((n, 12))).astype(np.float32), device="cuda")
    Yd = t.tensor((rng.standard_normal((n, 4))).astype(np.float32), device="cuda")
    say("mlp adam")
    p0 = st[:B.MLP_NPAR].double().cpu().numpy()
    m = np.zeros(B.MLP_NPAR)
    v = np.zeros(B.MLP_NPAR)
    p = p0.copy()
    g = t.zeros(B.MLP_NPAR, dtype=t.float32, device="cuda")
    for step in (1, 2, 3):
        B.fr_mlp_grad(plan.handle, st, Xd, Yd, g)
        t.cuda.synchronize()
        oracle.adam(p, g.double().cpu().numpy(), m, v, 1e-3, step)
        B.fr_mlp_train_step(plan.handle, st, Xd, Yd, 1e-3, step)
        t.cuda.synchronize()
        assert np.allclose(st[:B.MLP_NPAR].double().cpu().numpy(), p, rtol=1e-5, atol=2e-7)
    plan.close()


def test_sample_and_normalisation():
    t = torch()
    p, n = 2, (3, 2, 2)
    plan = B.Plan(p, n, ZETA, NU, T_CFG)
    rng = np.random.default_rng(8)
    Us = [inputs.tgv(p, n, noise=0.01, seed=k) for k in range(4)]
    Ud = [t.tensor(u, device="cuda") for u in Us]
    npts = 12 * 27
    ns = npts // 2
    X = t.zeros((ns, 12), dtype=t.float32, device="cuda")
    Y = t.zeros((ns, 4), dtype=t.float32, device="cuda")
    say("mlp sample")
    plan.set(B.FR_OPT_GUESS_BASE, 1)
    Y1 = t.zeros((ns, 4), dtype=t.float32, device="cuda")
    B.fr_mlp_sample(plan.handle, Ud[2], Ud[1], Ud[0], Ud[3], 1, 2, ns, X, Y1)
    plan.set(B.FR_OPT_GUESS_BASE, 2)
    B.fr_mlp_sample(plan.handle, Ud[2], Ud[1], Ud[0], Ud[3], 1, 2, ns, X, Y)
    t.cuda.synchronize()
    pts = 1 + 2 * np.arange(ns)
    e, q = pts // 27, pts % 27
    raw = np.zeros((ns, 12))
    tgt = np.zeros((ns, 4))
    for c in range(4):
        a, b, d, f = (Us[k][e, c, q] for k in (2, 1, 0, 3))
        raw[:, c], raw[:, 4 + c], raw[:, 8 + c] = a, a - b, (a - b) - (b - d)
        tgt[:, c] = f - (3.0 * (a - b) + d)
    assert np.array_equal(X.cpu().numpy(), raw.astype(np.float32))
    assert np.array_equal(Y.cpu().numpy(), tgt.astype(np.float32))
    tgt1 = np.stack([Us[3][e, c, q] - (2.0 * Us[2][e, c, q] - Us[1][e, c, q]) for c in range(4)], 1)
    assert np.array_equal(Y1.cpu().numpy(), tgt1.astype(np.float32))
    st = B.mlp_new_state(0)
    B.fr_mlp_fit_norm(plan.handle, st, X, Y)
    t.cuda.synchronize()
    s = st.cpu().numpy()
    Xf, Yf = X.double().cpu().numpy(), Y.double().cpu().numpy()
    assert np.allclose(s[5252:5264], Xf.mean(0), rtol=1e-5, atol=1e-7)
    assert np.allclose(s[5264:5276], 1.0 / Xf.std(0), rtol=1e-4)
    assert np.allclose(s[5276:5280], Yf.std(0), rtol=1e-4)
    plan.close()


@pytest.mark.parametrize("p,n", [(3, (2, 3, 2)), (2, (1, 2, 3)), (1, (3, 3, 5)), (2, (30, 30, 30))])
def test_guess_is_extrapolation_plus_network(p, n):
    """64 points per wave: 768 points fill 12 groups, 162 and 360 end in a
    ragged group; 729,000 points at p = 2 exceed one sweep of the launch grid
    (2048 workgroups x 4 waves x 64 points), so waves take a second group, with
    a point index that wraps (27 does not divide the sweep)."""
    t = torch()
    plan = B.Plan(p, n, ZETA, NU, T_CFG)
    ne, ns = n[0] * n[1] * n[2], (p + 1) ** 3
    Us = [t.tensor(inputs.tgv(p, n, noise=0.01, seed=k), device="cuda") for k in range(3)]
    G = t.empty_like(Us[0])
    E = t.empty_like(Us[0])
    say("mlp guess")
    st = B.mlp_new_state(3)
    for base in (1, 2):        # zero last layer: exactly the extrapolation the network corrects
        plan.set(B.FR_OPT_GUESS_BASE, base)
        B.fr_guess_extrap(plan.handle, Us[2], Us[1], Us[0], base, E)
        B.fr_mlp_guess(plan.handle, st, Us[2], Us[1], Us[0], G)
        t.cuda.synchronize()
        assert t.equal(G, E), base
    plan.set(B.FR_OPT_GUESS_BASE, 2)
    B.fr_guess_extrap(plan.handle, Us[2], Us[1], Us[0], 2, E)
    st = random_state(14, scale=0.2)
    B.fr_mlp_guess(plan.handle, st, Us[2], Us[1], Us[0], G)
    npts = ne * ns
    X = t.zeros((npts, 12), dtype=t.float32, device="cuda")
    Y = t.zeros((npts, 4), dtype=t.float32, device="cuda")
    B.fr_mlp_sample(plan.handle, Us[2], Us[1], Us[0], None, 0, 1, npts, X, Y)
    y = t.zeros((npts, 4), dtype=t.float32, device="cuda")
    B.fr_mlp_forward(plan.handle, st, X, y)
    t.cuda.synchronize()
    ysd = st[5276:5280].double()
    g4 = G.view(ne, 13, ns)[:, :4].permute(0, 2, 1).reshape(npts, 4)
    e4 = E.view(ne, 13, ns)[:, :4].permute(0, 2, 1).reshape(npts, 4)
    # the same features and products as the forward kernel: only the final
    # FP32 product and FP64 additions round differently
    assert t.allclose(g4 - e4, y.double() * ysd, rtol=0, atol=1e-6)
    assert t.equal(G.view(ne, 13, ns)[:, 4:], E.view(ne, 13, ns)[:, 4:])
    plan.close()


def test_training_reduces_loss():
    """Fit a random teacher network: 300 Adam steps cut the loss by 5x."""
    t = torch()
    plan = B.Plan(2, (2, 2, 2), ZETA, NU, T_CFG)
    rng = np.random.default_rng(9)
    n = 1 << 14
    X = rng.standard_normal((n, 12))
    teacher = {k: rng.standard_normal(s) * 0.4 for k, s in B.MLP_SHAPES}
    Yt = oracle.mlp_forward(X, teacher)
    Xd = t.tensor(X.astype(np.float32), device="cuda")
    Yd = t.tensor(Yt.astype(np.float32), device="cuda")
    st = B.mlp_new_state(1)
    B.fr_mlp_fit_norm(plan.handle, st, Xd, Yd)
    loss = t.zeros(1, dtype=t.float32, device="cuda")
    say("mlp training")
    losses = []
    for step in range(1, 301):
        B.fr_mlp_train_step(plan.handle, st, Xd, Yd, 3e-3, step, loss)
        if step in (1, 300):
            t.cuda.synchronize()
            losses.append(float(loss.item()))
    assert losses[1] < 0.2 * losses[0], losses
    plan.close()
