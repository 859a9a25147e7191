"""Pins of the FP64 MLP oracle: torch (independent implementation, FP64 autograd),
central finite differences, the closed form of the first Adam step, and torch's
BF16 rounding."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import mlp as M
from paper_1409_4923_amd import workloads as W


def _torch_model(p):
    q = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in M.unpack(p.astype(np.float64)).items()}
    return q


def _torch_forward(q, u):
    g = lambda z: torch.nn.functional.gelu(z, approximate="tanh")
    a1 = g(u @ q["W1"].T + q["b1"])
    a2 = g(a1 @ q["W2"].T + q["b2"])
    a3 = g(a2 @ q["W3"].T + q["b3"])
    return a3 @ q["W4"] + q["b4"][0]


def test_gelu_and_derivative_vs_torch():
    z = torch.linspace(-8, 8, 2001, dtype=torch.float64, requires_grad=True)
    y = torch.nn.functional.gelu(z, approximate="tanh")
    (dz,) = torch.autograd.grad(y.sum(), z)
    zn = z.detach().numpy()
    assert np.allclose(M.gelu(zn), y.detach().numpy(), rtol=0, atol=1e-15)
    assert np.allclose(M.gelu_grad(zn), dz.numpy(), rtol=0, atol=1e-13)


def test_normalise_maps_domain_corners():
    lo = np.array([[0.0, 1.0, -0.5, 1e-4, 0.5]])
    hi = np.array([[8.0, 10.0, 0.5, 1e-1, 2.0]])
    assert np.allclose(M.normalise(lo), -1.0, atol=1e-15)
    assert np.allclose(M.normalise(hi), 1.0, atol=1e-15)


def test_forward_and_backward_vs_torch_autograd():
    p = W.mlp_params(1, seed=3)[0].astype(np.float64)
    x = W.surrogate_queries(64, seed=4).astype(np.float64)
    t = np.sin(x[:, 0]) * 0.1
    q = _torch_model(p)
    y = _torch_forward(q, torch.tensor(M.normalise(x)))
    L = torch.mean((y - torch.tensor(t)) ** 2)
    L.backward()
    yo, _ = M.forward(p, x)
    assert np.allclose(yo, y.detach().numpy(), rtol=0, atol=1e-12)
    lo, g = M.backward(p, x, t)
    assert abs(lo - L.item()) < 1e-14
    gt = np.concatenate([q[name].grad.numpy().reshape(-1) for name, _ in M.SIZES])
    assert np.allclose(g, gt, rtol=1e-10, atol=1e-14)


def test_backward_vs_central_differences():
    p = W.mlp_params(1, seed=5)[0].astype(np.float64)
    x = W.surrogate_queries(32, seed=6).astype(np.float64)
    t = np.cos(x[:, 1]) * 0.2
    _, g = M.backward(p, x, t)
    rng = np.random.default_rng(7)
    # coordinates from every parameter group
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SIZES])
    idx = np.concatenate([rng.integers(offs[i], offs[i + 1], 6) for i in range(len(M.SIZES))])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss(p + e, x, t) - M.loss(p - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_adam_first_step_closed_form_and_torch():
    rng = np.random.default_rng(8)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m1, v1 = M.adam(p, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    tp = torch.tensor(p, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    pp, m, v = p.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 4):
        gs = g * step
        tp.grad = torch.tensor(gs)
        opt.step()
        pp, m, v = M.adam(pp, gs, m, v, step, 1e-3)
    assert np.allclose(pp, tp.detach().numpy(), rtol=0, atol=1e-12)


def test_bf16_rounding_vs_torch():
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(100000) * 10.0 ** rng.integers(-6, 6, 100000)).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def test_route_and_stats():
    preds = np.array([[0.0, 1.0, 0.5], [0.0, 1.0, 0.5], [0.0, 1.2, 0.5]])
    mean, std = M.ensemble_stats(preds)
    assert np.allclose(mean, [0.0, 1.0666666666666667, 0.5])
    assert list(M.route(std, 0.05)) == [1]
