"""Pins of the reference MLP of the surrogate: finite differences, torch on the CPU, bf16 rounding."""
import numpy as np
import pytest
import torch

from oracle import mlp as M


def init(widths, seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return [(rng.normal(size=(o, i)) * scale / np.sqrt(i), rng.normal(size=o) * 0.1)
            for i, o in zip(widths[:-1], widths[1:])]


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, 10000), [1 + 2 ** -8, 1 + 3 * 2 ** -8, -0.0]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def test_forward_matches_torch_modules():
    widths = [4, 16, 16, 6]
    layers = init(widths)
    x = np.random.default_rng(2).normal(size=(9, 4))
    net = torch.nn.Sequential(torch.nn.Linear(4, 16), torch.nn.SiLU(), torch.nn.Linear(16, 16), torch.nn.SiLU(),
                              torch.nn.Linear(16, 6)).double()
    with torch.no_grad():
        for lin, (W, b) in zip([net[0], net[2], net[4]], layers):
            lin.weight.copy_(torch.tensor(W))
            lin.bias.copy_(torch.tensor(b))
    y, _ = M.forward(layers, x)
    assert np.abs(y - net(torch.tensor(x)).detach().numpy()).max() < 1e-13


def test_gradients_against_finite_differences():
    widths = [4, 8, 8, 6]
    layers = init(widths, seed=3)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(5, 4))
    t = rng.normal(size=(5, 3))
    loss, grads = M.loss_and_grads(layers, x, t)
    flat = M.pack(layers)
    g = M.pack(grads)
    h = 1e-6
    for k in range(flat.size):
        e = np.zeros_like(flat)
        e[k] = h
        lp = M.nll(M.forward(M.unpack(widths, flat + e), x)[0], t)[0]
        lm = M.nll(M.forward(M.unpack(widths, flat - e), x)[0], t)[0]
        assert abs((lp - lm) / (2 * h) - g[k]) < 1e-7 * max(1.0, abs(g[k])), k


def test_loss_is_the_gaussian_nll():
    rng = np.random.default_rng(5)
    B, D = 7, 3
    y = rng.normal(size=(B, 2 * D))
    t = rng.normal(size=(B, D))
    loss, _ = M.nll(y, t)
    var = np.exp(y[:, D:])
    ref = -torch.distributions.Normal(torch.tensor(y[:, :D]), torch.tensor(np.sqrt(var))).log_prob(torch.tensor(t))
    ref = (ref.numpy() - 0.5 * np.log(2 * np.pi)).mean()  # without the constant term
    assert abs(loss - ref) < 1e-12


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    w0 = rng.normal(size=20)
    opt = M.Adam(20, lr=1e-2)
    p = torch.tensor(w0.copy(), requires_grad=True)
    topt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w = w0.copy()
    for k in range(5):
        g = rng.normal(size=20)
        w = opt.step(w, g)
        p.grad = torch.tensor(g)
        topt.step()
    assert np.abs(w - p.detach().numpy()).max() < 1e-13
