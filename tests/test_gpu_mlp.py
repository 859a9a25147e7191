"""The ensemble MLP surrogate on the GPU (through the C ABI) vs the FP64 numpy oracle.

Forward and gradients are compared at the same BF16-rounded weights (the GPU also
rounds activations to BF16 between layers, so agreement is to BF16 accuracy);
Adam is compared on the oracle's own gradients; routing is checked exactly.
"""
from __future__ import annotations

import numpy as np
import pytest

from helpers import say
from oracle import mlp as M
from paper_1409_4923_amd import bmotor as B
from paper_1409_4923_amd import workloads as W

pytestmark = pytest.mark.gpu

NM = 5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    B.lib()
    yield
    torch.cuda.synchronize()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def cosine(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def surrogate(params):
    return B.Surrogate(NM, params=params)


@pytest.mark.parametrize("batch", [1, 63, 1000, 70000])
def test_forward_matches_oracle(batch):
    import torch
    p = W.mlp_params(NM, seed=1)
    x = W.surrogate_queries(batch, seed=2)
    say("MLP forward, batch %d" % batch)
    s = surrogate(p)
    y = s.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    # the first rows and the ragged tail of the last 128-row work-group
    rows = np.unique(np.concatenate([np.arange(min(batch, 1000)), np.arange(max(0, batch - 1000), batch)]))
    for m in range(NM):
        yo, _ = M.forward(p[m].astype(np.float64), x[rows].astype(np.float64), bf16_weights=True)
        assert rel_l2(y[m, rows], yo) < 2e-2, m
        if len(rows) > 10:
            assert cosine(y[m, rows] - y[m, rows].mean(), yo - yo.mean()) > 0.999


@pytest.mark.parametrize("members,batch", [(1, 129), (B.BM_MLP_MAX_MEMBERS, 300)])
def test_forward_member_counts(members, batch):
    """One member and the largest ensemble the library takes, every row checked."""
    import torch
    p = W.mlp_params(members, seed=5)
    x = W.surrogate_queries(batch, seed=6)
    s = B.Surrogate(members, params=p)
    y = s.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    assert y.shape == (members, batch)
    for m in range(members):
        yo, _ = M.forward(p[m].astype(np.float64), x.astype(np.float64), bf16_weights=True)
        assert rel_l2(y[m], yo) < 2e-2, m


def test_gradients_match_oracle():
    import torch
    p = W.mlp_params(NM, seed=3)
    x = W.surrogate_queries(512, seed=4)
    t = (0.3 * np.sin(x[:, 0]) + 0.5 * x[:, 2]).astype(np.float32)
    s = surrogate(p)
    loss = s.backward(torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")).cpu().numpy()
    g = s.grad.cpu().numpy()
    offs = np.cumsum([0] + [int(np.prod(sh)) for _, sh in M.SIZES])
    for m in range(NM):
        lo, go = M.backward(p[m].astype(np.float64), x.astype(np.float64), t.astype(np.float64),
                            bf16_weights=True)
        assert abs(loss[m] - lo) <= 2e-2 * lo
        for k, (name, _) in enumerate(M.SIZES):
            a, b = g[m, offs[k]:offs[k + 1]], go[offs[k]:offs[k + 1]]
            if name == "b4":
                assert abs(a[0] - b[0]) <= 2e-2 * max(abs(b[0]), 1e-3), (m, name)
                continue
            assert rel_l2(a, b) < 5e-2, (m, name, rel_l2(a, b))
            assert cosine(a, b) > 0.998, (m, name, cosine(a, b))


def test_gradients_with_member_indices():
    """Each member may train on its own minibatch rows."""
    import torch
    p = W.mlp_params(NM, seed=5)
    x = W.surrogate_queries(4096, seed=6)
    t = (0.2 * np.cos(x[:, 1])).astype(np.float32)
    rng = np.random.default_rng(7)
    idx = rng.integers(0, 4096, (NM, 256)).astype(np.int32)
    s = surrogate(p)
    s.backward(torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda"), torch.tensor(idx, device="cuda"))
    g = s.grad.cpu().numpy()
    for m in range(NM):
        _, go = M.backward(p[m].astype(np.float64), x[idx[m]].astype(np.float64), t[idx[m]].astype(np.float64),
                           bf16_weights=True)
        assert cosine(g[m], go) > 0.998


def test_adam_matches_oracle_on_given_gradients():
    import torch
    p = W.mlp_params(NM, seed=8)
    rng = np.random.default_rng(9)
    s = surrogate(p)
    pp = p.astype(np.float64)
    mo = np.zeros_like(pp)
    vo = np.zeros_like(pp)
    for step in range(1, 4):
        g = (rng.standard_normal(p.shape) * 1e-2).astype(np.float32)
        s.grad.copy_(torch.tensor(g))
        s.adam(1e-3)
        for m in range(NM):
            pp[m], mo[m], vo[m] = M.adam(pp[m], g[m].astype(np.float64), mo[m], vo[m], step, 1e-3)
    got = s.params.cpu().numpy()
    assert np.max(np.abs(got - pp)) < 1e-6
    # the BF16 copies follow the updated weights
    wbf = s.wbf.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    w2 = wbf[:, 1280:1280 + 65536].view(np.float32)
    ref = M.bf16_round(got[:, 1536:1536 + 65536]).astype(np.float32)
    assert np.array_equal(w2, ref)


def test_training_lowers_loss():
    import torch
    x = W.surrogate_queries(8192, seed=10)
    t = (0.4 * np.sin(x[:, 0]) * np.cos(0.5 * x[:, 1]) + 0.3 * x[:, 2]).astype(np.float32)
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    s = B.Surrogate(NM, seed=11)
    rng = np.random.default_rng(12)
    first = None
    for step in range(300):
        idx = torch.tensor(rng.integers(0, 8192, (NM, 256)).astype(np.int32), device="cuda")
        loss = s.backward(xd, td, idx)
        s.adam(2e-3)
        if first is None:
            first = loss.cpu().numpy()
    last = s.backward(xd[:4096], td[:4096]).cpu().numpy()
    say("  loss %s -> %s" % (first, last))
    assert np.all(last < 0.1 * first)


def test_query_statistics_and_routing():
    import torch
    p = W.mlp_params(NM, seed=13)
    x = W.surrogate_queries(100_003, seed=14)
    s = surrogate(p)
    xd = torch.tensor(x, device="cuda")
    y = s.forward(xd).cpu().numpy().astype(np.float64)
    thr = float(np.median(y.std(axis=0)))
    mean, std, fidx, fcnt = s.query(xd, thr)
    mean, std = mean.cpu().numpy(), std.cpu().numpy()
    n = int(fcnt.cpu().numpy()[0])
    assert np.allclose(mean, y.mean(axis=0), rtol=0, atol=1e-6)
    assert np.allclose(std, y.std(axis=0), rtol=0, atol=1e-6)
    assert np.array_equal(fidx.cpu().numpy()[:n].astype(np.uint32), M.route(std, thr))
    # against the oracle's ensemble statistics at BF16 weights (first rows)
    preds = np.stack([M.forward(p[m].astype(np.float64), x[:500].astype(np.float64), bf16_weights=True)[0]
                      for m in range(NM)])
    mo, so = M.ensemble_stats(preds)
    assert rel_l2(mean[:500], mo) < 2e-2


def test_init_distribution():
    import torch
    s = B.Surrogate(NM, seed=15)
    p = s.params.cpu().numpy()
    assert np.all(np.abs(p[:, :1280]) <= 1 / np.sqrt(5) + 1e-7)
    assert np.all(np.abs(p[:, 1536:]) <= 1 / 16 + 1e-7)
    assert abs(np.mean(p[:, 1536:1536 + 65536] * 16)) < 0.01
    assert abs(np.var(p[:, 1536:1536 + 65536] * 16) - 1 / 3) < 0.01
    assert not np.array_equal(p[0], p[1])
