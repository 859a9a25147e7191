"""What the learned surrogate gains over plain Monte Carlo (GPU).

Labels come from one batched scan; the 5-member ensemble is trained on the GPU by
the library's own backward / Adam kernels; held-out truth comes from a scan with
4x the paths.  Plain-MC cost of a point at |d<v>| <= 0.01 is the path-steps needed
for 3 SE <= 0.01 at the measured scan throughput; the surrogate's cost is its
query time plus that MC cost for the routed queries.  The sub-domain (D >= 10^-1.5,
a <= 1) is one where <v> is smooth, so the ensemble agrees and is right.
"""
from __future__ import annotations

import numpy as np
import pytest

from helpers import say
from paper_1409_4923_amd import bmotor as B
from paper_1409_4923_amd import surrogate as S
from paper_1409_4923_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    B.lib()
    yield


def smooth_queries(n, seed):
    x = W.surrogate_queries(n, seed=seed)
    rng = np.random.default_rng(seed + 1)
    x[:, 0] = rng.uniform(0.0, 1.0, n)
    x[:, 3] = 10.0 ** rng.uniform(-1.5, -1.0, n)
    return x.astype(np.float32)


def test_surrogate_gain_over_monte_carlo():
    import torch
    tol, thr = 0.01, 0.005
    xl = smooth_queries(20000, 5)
    lab = S.monte_carlo(xl, 1024, 100, seed=1)
    say("labels: 20000 points in %.2f s, median SE %.4f" % (lab.seconds, np.median(lab.se)))
    sur = B.Surrogate(5, seed=3)
    hist = S.train(sur, xl, lab.mean, epochs=30, batch=1024, lr=2e-3, seed=4)
    say("train loss %.3g -> %.3g" % (hist[0], hist[-1]))
    assert hist[-1] < 0.1 * hist[0]
    xh = smooth_queries(1000, 9)
    truth = S.monte_carlo(xh, 4096, 100, seed=2, first_point=1 << 24)
    mean, std, fidx, fcnt = sur.query(torch.tensor(xh, device="cuda"), thr)
    mean, std = mean.cpu().numpy(), std.cpu().numpy()
    keep = std <= thr
    err = np.abs(mean - truth.mean)
    say("answered %d of 1000, p95 |err| %.4f (truth SE median %.4f)"
        % (keep.sum(), np.percentile(err[keep], 95) if keep.any() else -1, np.median(truth.se)))
    assert keep.mean() > 0.5
    assert np.percentile(err[keep], 95) <= tol
    # points/s at |d<v>| <= tol
    rate = truth.path_steps / truth.seconds
    need = np.maximum(64.0, np.ceil((3.0 * truth.std / tol) ** 2))
    mc_cost = float(np.mean(need) * 100 * S.SPP / rate)
    q = S.query(sur, smooth_queries(100_000, 11), thr, n_paths=4096, periods=100, seed=3)
    f = len(q.fallback) / 100_000
    sur_rate = 100_000 / (q.t_query + f * 100_000 * mc_cost)
    say("MC %.1f points/s, surrogate %.1f points/s (fallback %.3f), gain %.1f"
        % (1 / mc_cost, sur_rate, f, sur_rate * mc_cost))
    assert sur_rate * mc_cost > 10.0


def test_surrogate_on_the_configured_domain_is_tracked():
    """The whole configured domain (multistable regions included), with a small label
    budget and one round of labels where the ensemble disagrees most: the answered
    held-out points stay within 0.01 of the Monte Carlo truth (p95), the ensemble
    answers a fair share of the queries itself, and the fallback fraction and gain over
    plain MC are reported (the benchmark tracks them at full size)."""
    import torch
    tol, thr = 0.01, 0.005
    xl = W.surrogate_queries(60000, seed=21)
    lab = S.monte_carlo(xl, 256, 100, seed=1)
    sur = B.Surrogate(5, seed=3)
    S.train(sur, xl, lab.mean, epochs=60, batch=1024, lr=2e-3, seed=4)
    xc = W.surrogate_queries(300_000, seed=22)
    pick = S.uncertain_points(sur, xc, 30000, thr)
    assert 0 < len(pick) <= 30000
    _, sd, _, _ = sur.query(torch.tensor(xc, device="cuda"), thr)
    sd = sd.cpu().numpy()
    # the picked points are the largest spreads above the threshold
    rest = np.setdiff1d(np.nonzero(sd > thr)[0], pick)
    assert np.all(sd[pick] > thr)
    assert len(rest) == 0 or np.min(sd[pick]) >= np.max(sd[rest])
    lab_a = S.monte_carlo(xc[pick], 256, 100, seed=1, first_point=1 << 22)
    xa, ya = np.concatenate([xl, xc[pick]]), np.concatenate([lab.mean, lab_a.mean])
    S.train(sur, xa, ya, epochs=40, batch=1024, lr=1e-3, seed=5)
    xh = W.surrogate_queries(1000, seed=23)
    truth = S.monte_carlo(xh, 4096, 100, seed=2, first_point=1 << 24)
    mean, std, _, _ = sur.query(torch.tensor(xh, device="cuda"), thr)
    mean, std = mean.cpu().numpy(), std.cpu().numpy()
    keep = std <= thr
    err = np.abs(mean - truth.mean)
    rate = truth.path_steps / truth.seconds
    need = np.maximum(64.0, np.ceil((3.0 * np.nan_to_num(truth.std, nan=1.0) / tol) ** 2))
    cost = need * 100 * S.SPP / rate
    f = 1.0 - keep.mean()
    gain = float(np.mean(cost)) / (f * float(np.mean(cost[~keep])) if f > 0 else 1e-9)
    say("full domain: %d + %d labels, answered %.3f of held-out, p95 |err| %.4f, fallback %.3f, "
        "routed points cost %.2fx the mean, gain %.2f"
        % (len(xl), len(pick), keep.mean(), np.percentile(err[keep], 95) if keep.any() else -1, f,
           float(np.mean(cost[~keep])) / float(np.mean(cost)) if f > 0 else 0.0, gain))
    assert keep.mean() > 0.3
    assert np.percentile(err[keep], 95) <= tol


def test_adaptive_monte_carlo_meets_its_tolerance():
    """The fallback's sequential budget: every point gets at least the pilot's paths and
    at most the cap, the path-steps charged are the paths run, the pooled standard
    errors meet 3 SE <= tol (up to the spread the last round misjudged), and the means
    agree with an independent scan of 16384 paths per point."""
    tol, periods, pilot, cap = 0.02, 50, 64, 1 << 15
    x = W.surrogate_queries(64, seed=31)
    ad = S.adaptive_monte_carlo(x, tol, periods, pilot=pilot, max_paths=cap, seed=3, first_point=1 << 26)
    assert np.all(ad.n_paths >= pilot) and np.all(ad.n_paths <= cap)
    assert ad.path_steps == int(np.sum(ad.n_paths)) * periods * S.SPP
    free = ad.n_paths < cap
    say("adaptive: paths per point %d .. %d (median %d), %d capped, 3 SE / tol max %.2f, %.3f s"
        % (ad.n_paths.min(), ad.n_paths.max(), np.median(ad.n_paths), (~free).sum(),
           np.max(3 * ad.se[free] / tol) if free.any() else 0.0, ad.seconds))
    assert np.mean(3 * ad.se[free] <= tol) >= 0.9
    assert np.all(3 * ad.se[free] <= 1.5 * tol)
    truth = S.monte_carlo(x, 1 << 14, periods, seed=9, first_point=1 << 26)
    z = np.abs(ad.mean - truth.mean) / np.sqrt(ad.se ** 2 + truth.se ** 2)
    say("adaptive vs truth: max z %.2f, fraction within 3 combined SE %.3f" % (z.max(), np.mean(z <= 3)))
    assert np.mean(z <= 3) >= 0.95
    # the budget follows the spread: a uniform count at the largest need costs more
    assert np.sum(ad.n_paths) < len(x) * np.max(ad.n_paths)


def test_query_with_sequential_fallback():
    """query(tol=...) answers the rows the ensemble routes with the sequential Monte Carlo
    budget and leaves the others at the ensemble mean; the routed rows agree with an
    independent 16384-path scan within 3 combined SE (95% of them)."""
    import torch
    tol, periods = 0.02, 50
    sur = B.Surrogate(5, seed=3)                   # untrained: the spreads are wide
    x = W.surrogate_queries(96, seed=41)
    _, sd0, _, _ = sur.query(torch.tensor(x, device="cuda"), 1.0)
    thr = float(np.median(sd0.cpu().numpy()))      # about half of the rows routed
    q = S.query(sur, x, thr, None, periods, seed=7, mc_first_point=1 << 27, tol=tol)
    mean, std, _, fcnt = sur.query(torch.tensor(x, device="cuda"), thr)
    mean, std = mean.cpu().numpy().astype(np.float64), std.cpu().numpy()
    routed = np.nonzero(~(std <= thr))[0]
    assert np.array_equal(np.sort(q.fallback), routed) and len(routed) == int(fcnt.item())
    kept = np.setdiff1d(np.arange(len(x)), routed)
    assert np.array_equal(q.value[kept], mean[kept])
    assert 0 < len(routed) < len(x)
    ad = S.adaptive_monte_carlo(x[routed], tol, periods, seed=7, first_point=1 << 27)
    assert np.array_equal(q.value[routed], ad.mean)      # the same streams, the same budget
    truth = S.monte_carlo(x[routed], 1 << 14, periods, seed=19, first_point=1 << 27)
    z = np.abs(ad.mean - truth.mean) / np.sqrt(ad.se ** 2 + truth.se ** 2)
    say("query with sequential fallback: %d of %d routed, %.3f within 3 combined SE"
        % (len(routed), len(x), np.mean(z <= 3)))
    assert np.mean(z <= 3) >= 0.95
