"""The batched scan (persistent work-stealing launch in a hipGraph) through the C ABI.

Each scan point must equal, bit for bit, bm_integrate + bm_reduce on an ensemble
of that point (which is itself checked against the FP64 oracle), whatever the
launch shape; FP64 scan points are also compared with the oracle directly.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

import oracle
from helpers import ORACLE_THREADS, say, to_oracle
from paper_1409_4923_amd import bmotor as B
from paper_1409_4923_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    B.lib()
    yield
    torch.cuda.synchronize()


def stats_bytes(s: B.bm_stats) -> bytes:
    return bytes(memoryview(s))


def ensemble_stats(w: W.Workload) -> B.bm_stats:
    m, r = W.to_c(w)
    e = B.Ensemble(m, r)
    e.integrate(w.n_steps)
    return e.stats()


def run_scan(ws, tune=None):
    mr = [W.to_c(w) for w in ws]
    sc = B.Scan([m for m, _ in mr], [r for _, r in mr], tune=tune)
    sc.launch()
    return sc.stats()


def mixed_points(prec, noise=W.GAUSS | W.POISSON, dyn=W.INERTIAL, pot=W.POT_SIN):
    base = W.C2.with_(prec=prec, noise=noise, dyn=dyn, pot=pot, Fa=0.5, Fb=1.0, mua=1.0, mub=2.0)
    shapes = [(1, 480, 240), (63, 1000, 500), (65, 777, 100), (200, 2000, 1000), (1000, 1500, 1499),
              (4097, 600, 0), (128, 3000, 1500)]
    out = []
    for i, (n, steps, win) in enumerate(shapes):
        out.append(base.with_(name="p%d" % i, n_paths=n, n_steps=steps, n_window=win, point=100 + i,
                              a=1.0 + 0.5 * i, F=0.05 * i - 0.1, D=1e-3 * (i + 1), seed=7))
    return out


@pytest.mark.parametrize("prec", [W.F32, W.F64])
def test_scan_equals_ensembles_bitwise(prec):
    pts = mixed_points(prec)
    say("scan of %d mixed points, prec=%d" % (len(pts), prec))
    got = run_scan(pts)
    for w, g in zip(pts, got):
        ref = ensemble_stats(w)
        assert stats_bytes(g) == stats_bytes(ref), (w.name, g.mean, ref.mean)
        assert g.n == w.n_paths


def test_scan_busy_jumps_bitwise():
    """Kick queues that fill up (lambda dt = 0.5, flips with probability ~0.2 per step) end
    windows early inside the scan's persistent loop as well."""
    pts = [w.with_(lam=156.0, mua=60.0, mub=80.0)
           for w in mixed_points(W.F32, noise=W.GAUSS | W.POISSON | W.DICH)]
    got = run_scan(pts)
    for w, g in zip(pts, got):
        assert stats_bytes(g) == stats_bytes(ensemble_stats(w)), w.name


@pytest.mark.parametrize("noise,dyn,pot", [(W.GAUSS | W.DICH, W.OVERDAMPED, W.POT_RATCHET),
                                           (W.POISSON | W.DICH, W.OVERDAMPED, W.POT_TENT)])
def test_scan_other_models_bitwise(noise, dyn, pot):
    pts = [w.with_(spp=0, dt=2e-3, a=0.0) for w in mixed_points(W.F32, noise=noise, dyn=dyn, pot=pot)]
    got = run_scan(pts)
    for w, g in zip(pts, got):
        assert stats_bytes(g) == stats_bytes(ensemble_stats(w)), w.name


def test_scan_fp64_matches_oracle():
    pts = [w.with_(n_paths=min(w.n_paths, 300)) for w in mixed_points(W.F64)]
    got = run_scan(pts)
    for w, g in zip(pts, got):
        P = to_oracle(w)
        st = oracle.run(P, 0, w.n_paths, w.n_steps, threads=ORACLE_THREADS)
        so = oracle.stats(oracle.velocity(P, st, w.n_steps))
        assert g.n == so.n
        assert abs(g.mean - so.mean) <= 1e-8 * max(1.0, abs(so.mean)), (w.name, g.mean, so.mean)
        if so.n > 1:
            assert abs(g.var - so.var) <= 1e-7 * max(1.0, so.var)


@pytest.mark.parametrize("ppl,block,gpc", [(1, 64, 0), (1, 512, 1), (2, 128, 2), (2, 256, 0)])
def test_scan_launch_shape_invariance(ppl, block, gpc):
    pts = mixed_points(W.F32)
    a = run_scan(pts)
    b = run_scan(pts, tune=B.make_tune(ppl, block, gpc))
    assert [stats_bytes(x) for x in a] == [stats_bytes(x) for x in b]


def test_scan_graph_replays_with_eager_work_between():
    import torch
    pts = mixed_points(W.F32)
    mr = [W.to_c(w) for w in pts]
    sc = B.Scan([m for m, _ in mr], [r for _, r in mr])
    first = None
    for rep in range(3):
        sc.launch()
        res = [stats_bytes(x) for x in sc.stats()]
        if first is None:
            first = res
        assert res == first, rep
        # unrelated eager work on the same stream between replays
        ensemble_stats(pts[2])
        torch.cuda.synchronize()


def test_full_scan_workload_sampled_points():
    pts = W.c4_points()
    total = sum(w.path_steps() for w in pts)
    say("full scan: %d points, %.3g path-steps" % (len(pts), total))
    got = run_scan(pts)
    assert all(g.n + g.n_nonfinite == w.n_paths for w, g in zip(pts, got))
    assert all(g.n_nonfinite == 0 and math.isfinite(g.mean) for g in got)
    rng = np.random.default_rng(11)
    for i in rng.choice(len(pts), 6, replace=False):
        w = pts[int(i)]
        say("  point %d: %d paths x %d steps" % (i, w.n_paths, w.n_steps))
        assert stats_bytes(got[int(i)]) == stats_bytes(ensemble_stats(w)), int(i)


def test_autotune_sets_default():
    import torch
    pts = mixed_points(W.F32)
    mr = [W.to_c(w) for w in pts]
    models, runs = [m for m, _ in mr], [r for _, r in mr]
    nb = B.bm_scan_workspace_size(models, runs)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    res = torch.empty(len(pts) * B.STATS_BYTES, dtype=torch.uint8, device="cuda")
    t, ms = B.bm_scan_autotune(models, runs, 400, ws.data_ptr(), nb, res.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
    assert t.paths_per_lane in (1, 2) and t.block in (64, 128, 256, 512) and ms > 0
    d = B.bm_tune_get_default(pts[0].dyn, pts[0].pot, pts[0].noise, pts[0].prec)
    assert (d.paths_per_lane, d.block) == (t.paths_per_lane, t.block)
    # results under the tuned default are still bit-identical to the ensembles
    got = run_scan(pts)
    for w, g in zip(pts, got):
        assert stats_bytes(g) == stats_bytes(ensemble_stats(w))
    B.bm_tune_set_default(pts[0].dyn, pts[0].pot, pts[0].noise, pts[0].prec, B.make_tune())


def test_tune_cache_reused_by_a_second_process(tmp_path):
    """The tuned shape is written to a JSON cache keyed by device and model family; a
    second process loads it and gets the same shape without timing anything."""
    import json
    import subprocess
    import sys

    import torch
    pts = mixed_points(W.F32)
    mr = [W.to_c(w) for w in pts]
    models, runs = [m for m, _ in mr], [r for _, r in mr]
    nb = B.bm_scan_workspace_size(models, runs)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    res = torch.empty(len(pts) * B.STATS_BYTES, dtype=torch.uint8, device="cuda")
    cache = str(tmp_path / "tune.json")
    stream = torch.cuda.current_stream().cuda_stream
    t, ms = B.autotune_cached(models, runs, 400, ws.data_ptr(), nb, res.data_ptr(), stream, cache)
    assert ms is not None and ms > 0                               # timed: no cache yet
    doc = json.load(open(cache))
    key = dict(dyn=pts[0].dyn, pot=pts[0].pot, noise=pts[0].noise, prec=pts[0].prec)
    mine = [e for e in doc["entries"] if all(e[k] == v for k, v in key.items())]
    assert len(mine) == 1 and mine[0]["arch"].startswith("gfx950")
    assert (mine[0]["paths_per_lane"], mine[0]["block"]) == (t.paths_per_lane, t.block)
    code = (
        "import sys, json, time; sys.path.insert(0, %r)\n"
        "from paper_1409_4923_amd import bmotor as B, workloads as W\n"
        "import test_gpu_scan as T\n"
        "pts = T.mixed_points(W.F32)\n"
        "mr = [W.to_c(w) for w in pts]\n"
        "assert B.bm_tune_lookup(pts[0].dyn, pts[0].pot, pts[0].noise, pts[0].prec) is None\n"
        "t0 = time.perf_counter()\n"
        "t, ms = B.autotune_cached([m for m, _ in mr], [r for _, r in mr], 400, 0, 0, 0, 0, %r)\n"
        "print(json.dumps([t.paths_per_lane, t.block, t.groups_per_cu, ms, time.perf_counter() - t0]))\n"
    ) % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))), cache)
    env = dict(os.environ)
    env["PYTHONPATH"] = os.path.dirname(os.path.abspath(__file__)) + os.pathsep + env.get("PYTHONPATH", "")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stderr[-2000:]
    ppl, block, gpc, ms2, secs = json.loads(out.stdout.strip().splitlines()[-1])
    assert (ppl, block, gpc) == (t.paths_per_lane, t.block, t.groups_per_cu)
    assert ms2 is None                                             # taken from the cache, no timing
    B.bm_tune_set_default(pts[0].dyn, pts[0].pot, pts[0].noise, pts[0].prec, B.make_tune())
