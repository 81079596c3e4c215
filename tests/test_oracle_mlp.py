"""Pins of the oracle's pointwise MLP (12 -> 64 -> 64 -> 4, tanh): gradients
against central finite differences and against torch autograd, Adam against
torch.optim.Adam, all in float64 on the CPU."""
import numpy as np
import pytest
import torch

import oracle


def init_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return {k: rng.standard_normal(s) * scale for k, s in oracle.MLP_SHAPES}


def torch_mlp(params, X):
    W1, b1, W2, b2, W3, b3 = (params[k] for k, _ in oracle.MLP_SHAPES)
    h1 = torch.tanh(X @ W1.T + b1)
    h2 = torch.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3


def test_forward_matches_torch():
    p = init_params(0)
    X = np.random.default_rng(1).standard_normal((37, 12))
    Y = oracle.mlp_forward(X, p)
    tp = {k: torch.tensor(v) for k, v in p.items()}
    assert np.allclose(Y, torch_mlp(tp, torch.tensor(X)).numpy(), atol=1e-14)


def test_gradients_match_autograd_and_finite_differences():
    p = init_params(2)
    rng = np.random.default_rng(3)
    X, Tg = rng.standard_normal((29, 12)), rng.standard_normal((29, 4))
    loss, g = oracle.mlp_loss_grad(X, Tg, p)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    tl = torch.mean((torch_mlp(tp, torch.tensor(X)) - torch.tensor(Tg)) ** 2)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-14
    for k, _ in oracle.MLP_SHAPES:
        assert np.allclose(g[k], tp[k].grad.numpy(), atol=1e-14, rtol=1e-12), k
    # central differences on a few entries of every tensor
    h = 1e-6
    for k, s in oracle.MLP_SHAPES:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = oracle.mlp_loss_grad(X, Tg, p)
            flat[idx] = old - h
            lm, _ = oracle.mlp_loss_grad(X, Tg, p)
            flat[idx] = old
            assert abs((lp - lm) / (2 * h) - g[k].ravel()[idx]) < 1e-8


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    w = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tw = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([tw], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        oracle.adam(w, g, m, v, 1e-2, step)
        tw.grad = torch.tensor(g)
        opt.step()
        assert np.allclose(w, tw.detach().numpy(), atol=1e-14, rtol=1e-13)


# --- bfloat16 operand mode -------------------------------------------------------------------

def torch_round(x):
    """binary64 -> binary32 -> bfloat16 with torch's conversions (nearest, ties to even)."""
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def test_bf16_rounding_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [0.0, -0.0, 1.0, -3.5, 1e-30, 6e37]])
    assert np.array_equal(oracle.bf16_round(x), torch_round(torch.tensor(x)).numpy())
    # exact ties between two bfloat16 neighbours round to the even one
    ulp = 2.0 ** -7                                     # bfloat16 spacing in [1, 2)
    assert oracle.bf16_round(np.array([1 + ulp / 2]))[0] == 1.0
    assert oracle.bf16_round(np.array([1 + 3 * ulp / 2]))[0] == 1 + 2 * ulp
    assert oracle.bf16_round(np.array([1 + ulp / 2 + 2.0 ** -20]))[0] == 1 + ulp


class RoundedLinear(torch.autograd.Function):
    """x W^T with both operands rounded to bfloat16 in the forward product, and
    the incoming gradient rounded with the operand it meets in both backward
    products (the gradients flow through products with rounded operands)."""

    @staticmethod
    def forward(ctx, x, W):
        ctx.save_for_backward(x, W)
        return torch_round(x) @ torch_round(W).T

    @staticmethod
    def backward(ctx, g):
        x, W = ctx.saved_tensors
        gr = torch_round(g)
        return gr @ torch_round(W), gr.T @ torch_round(x)


def torch_mlp_rounded(params, X):
    W1, b1, W2, b2, W3, b3 = (params[k] for k, _ in oracle.MLP_SHAPES)
    h1 = torch.tanh(RoundedLinear.apply(X, W1) + b1)
    h2 = torch.tanh(RoundedLinear.apply(h1, W2) + b2)
    return RoundedLinear.apply(h2, W3) + b3


def test_bf16_operand_mode_matches_autograd_through_rounded_products():
    p = init_params(8)
    rng = np.random.default_rng(9)
    X, Tg = rng.standard_normal((41, 12)), rng.standard_normal((41, 4))
    Y = oracle.mlp_forward(X, p, bf16_operands=True)
    loss, g = oracle.mlp_loss_grad(X, Tg, p, bf16_operands=True)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    ty = torch_mlp_rounded(tp, torch.tensor(X))
    assert np.allclose(Y, ty.detach().numpy(), atol=1e-13, rtol=1e-12)
    tl = torch.mean((ty - torch.tensor(Tg)) ** 2)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-13
    for k, _ in oracle.MLP_SHAPES:
        assert np.allclose(g[k], tp[k].grad.numpy(), atol=1e-14, rtol=1e-11), k
    # the rounding changes the results, by about the bfloat16 unit
    Y0 = oracle.mlp_forward(X, p)
    d = np.max(np.abs(Y - Y0)) / np.max(np.abs(Y0))
    assert 1e-4 < d < 5e-2, d
    _, g0 = oracle.mlp_loss_grad(X, Tg, p)
    assert np.linalg.norm(g0["W2"] - g["W2"]) > 1e-4 * np.linalg.norm(g0["W2"])
