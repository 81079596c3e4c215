"""GPU parity of the ACM-HD residual on linear hexahedra (fr_lhex_*) against
the oracle (oracle/linear_hex.py): randomly distorted meshes at p = 1..6 on
ragged lattices, affine corners against the constant-Jacobian fused residual,
free stream, every element of a p = 4, 51^3 lattice tiled from a distorted
3^3 block, and argument errors."""
import numpy as np
import pytest

from oracle import linear_hex as L
from paper_2107_14027_amd import binding as B
from paper_2107_14027_amd import inputs
from gpu_util import T_CFG, ZETA, say

pytestmark = pytest.mark.gpu

NU_V = 0.05


def rand_state(p, ne, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ne, 13, (p + 1) ** 3)) * 0.5


def run(p, n, U, C, nu=NU_V, T=T_CFG):
    import torch
    plan = B.Plan(p, n, ZETA, nu, T)
    lh = B.LinearHex(plan)
    Ud = torch.from_numpy(np.ascontiguousarray(U)).to("cuda")
    Rd = torch.empty_like(Ud)
    lh.residual(torch.from_numpy(np.ascontiguousarray(C)).to("cuda"), Ud, Rd)
    torch.cuda.synchronize()
    out = Rd.cpu().numpy()
    lh.close()
    plan.close()
    return out


@pytest.mark.parametrize("p,n,amp", [(1, (3, 2, 2), 0.25), (2, (2, 3, 2), 0.2), (3, (3, 2, 2), 0.25),
                                     (4, (2, 2, 3), 0.15), (5, (2, 2, 2), 0.2), (6, (2, 1, 2), 0.1)])
def test_distorted_mesh_matches_oracle(p, n, amp):
    C = inputs.linear_hex_corners(n, amp=amp, seed=p, smooth=0.1)
    U = rand_state(p, n[0] * n[1] * n[2], 30 + p)
    say("lhex p=%d n=%s amp=%g" % (p, n, amp))
    R = run(p, n, U, C)
    Ro = L.residual(p, n, U, C, ZETA, NU_V, T_CFG)
    assert np.max(np.abs(R - Ro)) <= 1e-12 * np.max(np.abs(Ro))


def test_affine_equals_fused_residual():
    import torch
    from gpu_util import gpu_residual
    p, n = 3, (3, 2, 4)
    U = rand_state(p, 24, 5)
    J = inputs.box_jacobian(n)
    e = np.arange(24)
    org = np.stack([e % 3, (e // 3) % 2, e // 6], axis=1).astype(float)
    C = np.stack([(2 * org + 1 + L.SIGNS[c][None, :]) @ J.T for c in range(8)], axis=1)
    say("lhex affine")
    R = run(p, n, U, C, nu=1.0 / 1600.0)
    Rf = gpu_residual(p, n, U, nu=1.0 / 1600.0)
    assert np.max(np.abs(R - Rf)) <= 1e-12 * np.max(np.abs(Rf))


def test_free_stream():
    p, n = 4, (3, 2, 2)
    C = inputs.linear_hex_corners(n, amp=0.25, seed=9)
    vals = np.array([0.7, 0.3, -0.2, 0.5] + list(np.linspace(-0.4, 0.4, 9)))
    U = np.broadcast_to(vals[None, :, None], (12, 13, 125)).copy()
    say("lhex free stream")
    R = run(p, n, U, C)
    src = np.concatenate([np.zeros(4), -vals[4:] / T_CFG])
    assert np.max(np.abs(R - src[None, :, None])) <= 1e-11


def test_full_size_tiled_mesh():
    """p = 4, 51^3: the mesh and state repeat every 3 elements per direction, so
    the residual is the 3^3 block's (only tangents of the map enter)."""
    import torch
    p, blk, reps = 4, 3, 17
    N = blk * reps
    h = 2 * np.pi / N
    Cb = inputs.linear_hex_corners((blk, blk, blk), amp=0.2, seed=11, smooth=0.1) * (blk / N)
    rng = np.random.default_rng(12)
    Ub = rng.standard_normal((blk ** 3, 13, 125)) * 0.5
    e = np.arange(N ** 3)
    ex, ey, ez = e % N, (e // N) % N, e // (N * N)
    bi = (ex % blk) + blk * ((ey % blk) + blk * (ez % blk))
    shift = blk * h * np.stack([ex // blk, ey // blk, ez // blk], axis=1).astype(float)
    C = Cb[bi] + shift[:, None, :]
    U = Ub[bi]
    say("lhex tiled p=%d N=%d" % (p, N))
    R = run(p, (N, N, N), U, C, nu=1.0 / 1600.0)
    Rb = L.residual(p, (blk, blk, blk), Ub, Cb, ZETA, 1.0 / 1600.0, T_CFG)
    assert np.max(np.abs(R - Rb[bi])) <= 1e-12 * np.max(np.abs(Rb))


def test_errors():
    import torch
    plan = B.Plan(2, (2, 2, 2), ZETA, NU_V, T_CFG)
    lh = B.LinearHex(plan)
    U = torch.zeros(plan.state_len, dtype=torch.float64, device="cuda")
    C = torch.zeros(8 * 24, dtype=torch.float64, device="cuda")
    with pytest.raises(B.FrError):
        lh.residual(C, U, U)
    with pytest.raises(ValueError):
        lh.residual(C[:-1].contiguous(), U, torch.empty_like(U))
    lh.close()
    plan.close()
