"""Pins of the oracle MLP against PyTorch CPU library routines (bfloat16 conversion, exact
GELU, float64 autograd, torch.optim.Adam) and finite differences."""
import numpy as np
import pytest
import torch

from oracle.mlp import MLP, adam_step, bf16_round, gelu, gelu_d, pad32


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 10000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -2.5e-38], dtype=np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(bf16_round(x), ref)


def test_gelu_matches_torch_and_limits():
    z = np.linspace(-9, 9, 1001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    assert np.allclose(gelu(z), ref, atol=1e-15, rtol=1e-13)
    assert gelu(np.array(0.0)) == 0.0
    h = 1e-6
    assert np.allclose(gelu_d(z), (gelu(z + h) - gelu(z - h)) / (2 * h), atol=1e-8)


def _net(widths, seed, rounding):
    rng = np.random.default_rng(seed)
    W = [rng.standard_normal((pad32(widths[l + 1]), pad32(widths[l]))) / np.sqrt(widths[l]) for l in range(len(widths) - 1)]
    for l in range(len(W)):
        W[l][widths[l + 1]:, :] = 0
        W[l][:, widths[l]:] = 0
    b = [0.1 * rng.standard_normal(pad32(widths[l + 1])) for l in range(len(widths) - 1)]
    for l in range(len(b)):
        b[l][widths[l + 1]:] = 0
    return MLP(widths, W, b, rounding)


def test_forward_backward_match_autograd_without_rounding():
    widths = [49, 128, 128, 128, 41]
    net = _net(widths, 1, rounding=False)
    rng = np.random.default_rng(2)
    B = 37
    x = np.zeros((B, pad32(49)))
    x[:, :49] = rng.standard_normal((B, 49))
    t = np.zeros((B, pad32(41)))
    t[:, :41] = rng.standard_normal((B, 41))
    zs, acts = net.forward(x)
    dW, db, loss = net.backward(x, zs, acts, t)
    Wt = [torch.tensor(w, requires_grad=True) for w in net.W]
    bt = [torch.tensor(v, requires_grad=True) for v in net.b]
    a = torch.tensor(x)
    for l in range(len(Wt)):
        a = a @ Wt[l].T + bt[l]
        if l < len(Wt) - 1:
            a = torch.nn.functional.gelu(a)
    y = a[:, :41]
    lt = 0.5 * ((y - torch.tensor(t[:, :41])) ** 2).sum() / B
    lt.backward()
    assert np.allclose(acts[-1], a.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert abs(loss - lt.item()) < 1e-12 * abs(loss)
    for l in range(len(Wt)):
        assert np.allclose(dW[l], Wt[l].grad.numpy(), rtol=1e-10, atol=1e-13)
        assert np.allclose(db[l], bt[l].grad.numpy(), rtol=1e-10, atol=1e-13)


def test_rounding_points():
    """With rounding on, each product sees BF16 operands: equal to the unrounded network
    applied to pre-rounded weights and inputs for a single linear layer."""
    net = _net([20, 7], 3, rounding=True)
    rng = np.random.default_rng(4)
    x = np.zeros((5, 32))
    x[:, :20] = rng.standard_normal((5, 20))
    zs, acts = net.forward(x)
    ref = bf16_round(x).astype(np.float64) @ bf16_round(net.W[0]).astype(np.float64).T + net.b[0]
    assert np.allclose(zs[0], ref, rtol=0, atol=1e-14)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    p = p0.copy()
    m1 = np.zeros(50)
    m2 = np.zeros(50)
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        p, m1, m2 = adam_step(p, g, m1, m2, step, 1e-3)
        opt.zero_grad()
        pt.grad = torch.tensor(g)
        opt.step()
        assert np.allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)
