"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 paths: per-path states within 1e-9 relative, integer noise state
bit-exact.  FP32 paths: integer noise decisions (taken in FP64 on both sides)
bit-exact, ensemble <v> within 3 standard errors.  Reductions match exactly
rounded sums.  Results are invariant to chunking, launch shape and ensemble size.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from helpers import ORACLE_THREADS, oracle_paths, say, to_oracle
from paper_1409_4923_amd import bmotor as B
from paper_1409_4923_amd import workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    B.lib()
    yield
    torch.cuda.synchronize()


def gpu_run(w: W.Workload, chunks, tune=None, first=0, count=None):
    m, r = W.to_c(w)
    e = B.Ensemble(m, r, tune=tune)
    for c in chunks:
        e.integrate(c)
    ps = e.read(first, count)
    return e, ps


def assert_close(a, b, rel=REL, what=""):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    err = np.abs(a - b) / np.maximum(1.0, np.abs(b))
    i = int(np.argmax(err))
    assert err[i] <= rel, "%s: max rel err %.3e at %d (gpu %r, oracle %r)" % (what, err[i], i, a[i], b[i])


# ---------------------------------------------------------------------------
# FP64 per-path parity
# ---------------------------------------------------------------------------
def test_c1_per_path_fp64_1000_steps():
    w = W.C1
    say("C1 FP64 per-path parity: 1024 paths x 1000 steps")
    _, ps = gpu_run(w, [1000])
    xu, v, nz, _ = oracle_paths(w, 0, w.n_paths, 1000)
    assert_close(ps.x.numpy(), xu, what="x")
    assert_close(ps.v.numpy(), v, what="v")


def _model_matrix():
    cases = []
    for dyn in (W.OVERDAMPED, W.INERTIAL):
        for pot in (W.POT_SIN, W.POT_RATCHET, W.POT_TENT, W.POT_FREE):
            jg = W.POISSON | W.JUMP_GRID
            for noise in list(range(8)) + [W.NORMAL, W.NORMAL | W.POISSON, W.NORMAL | W.DICH,
                                            W.NORMAL | W.POISSON | W.DICH,
                                            jg, jg | W.GAUSS, jg | W.DICH, jg | W.GAUSS | W.DICH,
                                            jg | W.NORMAL, jg | W.NORMAL | W.DICH]:
                cases.append((dyn, pot, noise))
    return cases


@pytest.mark.parametrize("dyn,pot,noise", _model_matrix())
def test_fp64_per_path_model_matrix(dyn, pot, noise):
    """Every (dynamics, potential, noise) kernel: ragged N, unaligned chunks."""
    spp = 64 if pot != W.POT_TENT else 0
    w = W.Workload(name="matrix", dyn=dyn, pot=pot, noise=noise, prec=W.F64, n_paths=333,
                   n_steps=777, n_window=300, gamma=1.3, a=(1.7 if spp else 0.0), omega=2.5,
                   F=0.2, D=0.05, lam=7.0, zeta=0.1, Fa=0.8, Fb=1.2, mua=3.0, mub=2.0, spp=spp,
                   dt=(0.0 if spp else 0.01), seed=12345, point=3, x0_lo=-0.5, x0_hi=1.5,
                   v0_lo=-1.0, v0_hi=1.0)
    say("FP64 matrix case dyn=%d pot=%d noise=%d" % (dyn, pot, noise))
    _, ps = gpu_run(w, [5, 100, 672])
    xu, v, nz, _ = oracle_paths(w, 0, w.n_paths, 777)
    assert np.array_equal(ps.noise.numpy(), nz)
    assert_close(ps.x.numpy(), xu, what="x")
    if dyn == W.INERTIAL:
        assert_close(ps.v.numpy(), v, what="v")


@pytest.mark.parametrize("dyn", [W.OVERDAMPED, W.INERTIAL])
@pytest.mark.parametrize("noise", [W.POISSON, W.DICH, W.GAUSS | W.POISSON | W.DICH,
                                   W.POISSON | W.JUMP_GRID, W.GAUSS | W.POISSON | W.DICH | W.JUMP_GRID])
@pytest.mark.parametrize("scale", [1.0, 4.0])
def test_fp64_per_path_high_jump_rates(dyn, noise, scale):
    """High jump rates (lambda dt = 0.25 or 1, flip probability ~0.2 or ~0.6 per step): the
    jump window shrinks to 16 steps, and at the higher rates lanes exceed its queue, so
    later jumps are drawn at their steps."""
    w = W.Workload(name="high-rate", dyn=dyn, pot=W.POT_SIN, noise=noise, prec=W.F64, n_paths=500,
                   n_steps=1000, n_window=100, gamma=1.0, D=0.01, lam=25.0 * scale, zeta=0.02,
                   Fa=0.5, Fb=0.5, mua=20.0 * scale, mub=25.0 * scale, dt=0.01, seed=5, x0_lo=0.0,
                   x0_hi=1.0, v0_lo=-1.0, v0_hi=1.0)
    say("FP64 high jump rates dyn=%d noise=%d" % (dyn, noise))
    _, ps = gpu_run(w, [131, 869])
    xu, v, nz, _ = oracle_paths(w, 0, w.n_paths, 1000)
    assert np.array_equal(ps.noise.numpy(), nz)
    assert_close(ps.x.numpy(), xu, what="x")
    if dyn == W.INERTIAL:
        assert_close(ps.v.numpy(), v, what="v")


@pytest.mark.parametrize("noise", [W.POISSON, W.DICH])
def test_fp32_jump_decisions_equal_fp64_kernel(noise):
    """The FP32 kernels decide countdowns from an FP32 estimate with an FP64 fallback near
    integer boundaries; over ~3e7 draws the integer jump state equals the FP64 kernel's."""
    base = W.Workload(name="decisions", dyn=W.OVERDAMPED, pot=W.POT_FREE, noise=noise, prec=W.F64,
                      n_paths=1 << 16, n_steps=2000, n_window=0, lam=25.0, zeta=0.02,
                      Fa=0.5, Fb=0.5, mua=20.0, mub=25.0, dt=0.01, seed=99)
    say("FP32 vs FP64 kernel jump decisions, noise=%d, 65536 paths x 2000 steps" % noise)
    _, a = gpu_run(base, [2000])
    _, b = gpu_run(base.with_(prec=W.F32), [2000])
    assert np.array_equal(a.noise.numpy(), b.noise.numpy())


@pytest.mark.parametrize("w", [W.C2, W.C3, W.C2.with_(noise=W.GAUSS | W.POISSON | W.JUMP_GRID)],
                         ids=["c2-model", "c3-model", "c2-jump-grid"])
def test_fp64_per_path_jump_models(w):
    w = w.with_(prec=W.F64, n_paths=4096)
    n = 1000
    say("FP64 per-path parity of %s: 4096 paths x %d steps" % (w.name, n))
    _, ps = gpu_run(w, [n])
    xu, v, nz, _ = oracle_paths(w, 0, w.n_paths, n)
    assert np.array_equal(ps.noise.numpy(), nz)
    assert_close(ps.x.numpy(), xu, what="x")
    assert_close(ps.v.numpy(), v, what="v")


# ---------------------------------------------------------------------------
# FP32 paths
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("w", [W.C1, W.C2, W.C3, W.C1.with_(noise=W.NORMAL),
                               W.C2.with_(noise=W.NORMAL | W.POISSON),
                               W.C2.with_(noise=W.GAUSS | W.POISSON | W.JUMP_GRID)],
                         ids=["c1-model", "c2-model", "c3-model", "c1-normal", "c2-normal", "c2-jump-grid"])
def test_fp32_noise_decisions_exact_and_states_close(w):
    w = w.with_(prec=W.F32, n_paths=2048)
    n = 300
    say("FP32 short-horizon parity of %s: 2048 paths x %d steps" % (w.name, n))
    _, ps = gpu_run(w, [n])
    xu, v, nz, _ = oracle_paths(w, 0, w.n_paths, n)
    assert np.array_equal(ps.noise.numpy(), nz)
    # FP32 rounding (and the hardware cos / log / sqrt) grown over a short horizon.
    # The driven inertial model is chaotic: a path near a separatrix amplifies its
    # rounding more than the bulk, so the bound holds for 99.5% of the paths and a
    # 25x looser one for every path (a systematic error would move them all).
    def bulk_close(a, b, what):
        err = np.abs(np.asarray(a, np.float64) - b) / np.maximum(1.0, np.abs(b))
        assert np.quantile(err, 0.995) <= 2e-3, "%s: 99.5%% quantile %.3e" % (what, np.quantile(err, 0.995))
        assert err.max() <= 5e-2, "%s: max %.3e at %d" % (what, err.max(), int(np.argmax(err)))
    bulk_close(ps.x.numpy(), xu, "x")
    if w.dyn == W.INERTIAL:
        bulk_close(ps.v.numpy(), v, "v")


def _ensemble_case(w, n_steps, n_window):
    return w.with_(n_paths=4096, n_steps=n_steps, n_window=n_window)


@pytest.mark.parametrize("w", [
    _ensemble_case(W.C1.with_(prec=W.F32), 20000, 10000),
    _ensemble_case(W.C2, 40000, 20000),
    _ensemble_case(W.C3, 100000, 10000),
    _ensemble_case(W.C1.with_(prec=W.F32, noise=W.NORMAL), 20000, 10000),
    _ensemble_case(W.C2.with_(noise=W.GAUSS | W.POISSON | W.JUMP_GRID), 40000, 20000),
    _ensemble_case(W.C3.with_(noise=W.NORMAL | W.DICH), 100000, 10000),
], ids=["c1-f32", "c2-f32", "c3-f32", "c1-normal-f32", "c2-jump-grid-f32", "c3-normal-f32"])
def test_fp32_mean_velocity_within_3se(w):
    say("FP32 <v> vs FP64 oracle: %s, %d paths x %d steps" % (w.name, w.n_paths, w.n_steps))
    e, ps = gpu_run(w, [w.n_steps])
    s = e.stats()
    P = to_oracle(w)
    st = oracle.run(P, 0, w.n_paths, w.n_steps, threads=ORACLE_THREADS)
    vo = oracle.velocity(P, st, w.n_steps)
    so = oracle.stats(vo)
    vg = ps.vp.numpy()
    say("  gpu %.6f +- %.6f   oracle %.6f +- %.6f" % (s.mean, s.se, so.mean, so.se))
    assert s.n == w.n_paths and s.n_nonfinite == 0
    assert abs(s.mean - so.mean) <= 3.0 * math.hypot(s.se, so.se)
    d = oracle.stats(vg - vo)                          # paired: same random streams
    assert abs(d.mean) <= 3.0 * d.se + 1e-12


# ---------------------------------------------------------------------------
# Reduction
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_paths", [1, 63, 64, 65, 1000, 70001])
def test_reduction_matches_exact_sums(n_paths):
    w = W.C2.with_(n_paths=n_paths, n_steps=600, n_window=200)
    say("reduction, N=%d" % n_paths)
    e, ps = gpu_run(w, [600])
    s = e.stats()
    ref = oracle.stats(ps.vp.numpy())
    assert s.n == ref.n and s.n_nonfinite == 0
    assert abs(s.t_window - 400 * w.step()) <= 1e-15 * s.t_window
    assert abs(s.mean - ref.mean) <= 2e-15 * max(1.0, abs(ref.mean))
    if n_paths > 1:
        assert abs(s.var - ref.var) <= 1e-12 * ref.var
        assert abs(s.se - ref.se) <= 1e-12 * ref.se
    else:
        assert math.isnan(s.var)


def test_fp64_vp_and_stats_match_oracle():
    w = W.C1.with_(n_steps=1500, n_window=500)
    e, ps = gpu_run(w, [1500])
    P = to_oracle(w)
    st = oracle.run(P, 0, w.n_paths, 1500, threads=ORACLE_THREADS)
    vo = oracle.velocity(P, st, 1500)
    assert_close(ps.vp.numpy(), vo, rel=1e-8, what="vp")
    s = e.stats()
    so = oracle.stats(vo)
    assert abs(s.mean - so.mean) <= 1e-8 * max(1.0, abs(so.mean))


# ---------------------------------------------------------------------------
# Invariances
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [W.F32, W.F64])
def test_chunking_invariance(prec):
    w = W.C2.with_(prec=prec, n_paths=5000, noise=W.GAUSS | W.POISSON)
    _, a = gpu_run(w, [1000])
    _, b = gpu_run(w, [3, 500, 16, 481])
    for f in ("x", "v", "noise"):
        assert np.array_equal(getattr(a, f).numpy(), getattr(b, f).numpy()), f


@pytest.mark.parametrize("ppl,block", [(1, 64), (1, 512), (2, 128), (2, 256)])
def test_launch_shape_invariance(ppl, block):
    # busy jumps (lambda dt = 0.5): kick queues fill up, so windows end early at
    # wave-dependent steps and give back the kicks and flips queued past their end
    # (with flips the queues of 512 lanes exceed the LDS limit)
    busy = W.C2.with_(name="busy-jumps", n_paths=5003, noise=W.GAUSS | W.POISSON, lam=156.0)
    ws = [W.C2.with_(n_paths=5003), W.C3.with_(n_paths=5003), busy]
    if ppl * block <= 256:
        ws.append(busy.with_(name="busy-jumps-flips", noise=W.GAUSS | W.POISSON | W.DICH, Fa=0.5, Fb=0.5,
                             mua=60.0, mub=80.0))
    for w in ws:
        _, a = gpu_run(w, [700])
        _, b = gpu_run(w, [700], tune=B.make_tune(ppl, block))
        for f in ("x", "v", "noise"):
            assert np.array_equal(getattr(a, f).numpy(), getattr(b, f).numpy()), (w.name, f)


def test_ensemble_size_invariance():
    w = W.C3.with_(n_paths=10000)
    _, a = gpu_run(w, [500], first=2000, count=300)
    _, b = gpu_run(w.with_(n_paths=2300), [500], first=2000, count=300)
    assert np.array_equal(a.x.numpy(), b.x.numpy())


# ---------------------------------------------------------------------------
# Full-size launch configuration: sampled paths, one by one
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("w", [W.C2, W.C3], ids=["c2", "c3"])
def test_full_size_sampled_paths(w):
    """Full ensemble in the benchmark's launch shape, 256 sampled paths checked one by one:
    positions after 300 steps (before FP32 and FP64 trajectories of the chaotic dynamics
    separate), and the integer noise state bit-exact after 4000 steps."""
    n_short, n = 300, 4000
    say("full-size %s: %d paths x %d steps, 256 sampled paths" % (w.name, w.n_paths, n))
    m, r = W.to_c(w)
    e = B.Ensemble(m, r)
    e.integrate(n_short)
    short = e.read()
    e.integrate(n - n_short)
    ps = e.read()
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(w.n_paths, 256, replace=False))
    P = to_oracle(w)
    for i in idx:
        st = oracle.run(P, int(i), 1, n_short)
        xu = oracle.unwrapped(P, st)[0]
        assert abs(short.x[i].item() - xu) <= 2e-3 * max(1.0, abs(xu)), (i, short.x[i].item(), xu)
        oracle.advance(P, st, int(i), n_short, n)
        nz = [st["sP"][0], st["kP"][0], st["sD"][0], st["mD"][0], st["d"][0]]
        if not (w.noise & W.POISSON):
            nz[0:2] = [0, 0]
        if not (w.noise & W.DICH):
            nz[2:5] = [0, 0, 0]
        assert list(ps.noise[i].numpy()) == [int(t) for t in nz], i


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------
def test_single_path_and_zero_steps():
    w = W.C1.with_(n_paths=1)
    e, ps0 = gpu_run(w, [0])
    xu, v, _, _ = oracle_paths(w, 0, 1, 0)
    assert_close(ps0.x.numpy(), xu)
    e.integrate(0)
    assert e.steps == 0
    e.integrate(37)
    xu, v, _, _ = oracle_paths(w, 0, 1, 37)
    assert_close(e.read().x.numpy(), xu)


def test_reduce_before_window_is_state_error():
    w = W.C1.with_(n_paths=100, n_window=50)
    e, _ = gpu_run(w, [50])
    with pytest.raises(B.BMError) as ex:
        e.reduce()
    assert ex.value.code == B.BM_ERR_STATE
    e.integrate(1)
    assert e.stats().n == 100


def test_window_at_zero():
    w = W.C3.with_(n_paths=256, n_window=0, prec=W.F64)
    e, ps = gpu_run(w, [200])
    P = to_oracle(w)
    st = oracle.run(P, 0, 256, 200)
    assert_close(ps.vp.numpy(), oracle.velocity(P, st, 200), rel=1e-8)


def test_nonfinite_paths_are_counted():
    # a tilt that overflows FP32 within one step drives every path to NaN
    w = W.Workload(name="overflow", dyn=W.OVERDAMPED, pot=W.POT_FREE, noise=0, prec=W.F32,
                   n_paths=100, n_steps=10, n_window=5, F=3e38, dt=10.0)
    e, _ = gpu_run(w, [10])
    s = e.stats()
    assert s.n == 0 and s.n_nonfinite == 100


def test_read_range_checked():
    w = W.C1.with_(n_paths=10)
    e, _ = gpu_run(w, [1])
    with pytest.raises(B.BMError) as ex:
        e.read(5, 6)
    assert ex.value.code == B.BM_ERR_INVALID_ARG


# ---------------------------------------------------------------------------
# eq. (19): density of the folded positions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [W.F64, W.F32])
def test_density_histogram(prec):
    import torch
    w = W.C3.with_(prec=prec, n_paths=20000, n_steps=3000, n_window=100)
    m, r = W.to_c(w)
    e = B.Ensemble(m, r)
    counts = torch.zeros(50, dtype=torch.int64, device="cuda")
    P = to_oracle(w)
    st = oracle.init(P, 0, w.n_paths)
    ref = np.zeros(50, dtype=np.int64)
    n = 0
    for chunk in (1000, 1000, 1000):
        e.integrate(chunk)
        e.density(counts)
        oracle.advance(P, st, 0, n, n + chunk, threads=ORACLE_THREADS)
        n += chunk
        ref += oracle.density(P, st, 50)
    got = counts.cpu().numpy()
    assert got.sum() == 3 * w.n_paths
    if prec == W.F64:
        assert np.array_equal(got, ref)
    else:
        assert np.max(np.abs(got - ref)) <= 0.02 * ref.max() + 20


@pytest.mark.parametrize("w", [W.C2.with_(n_paths=3000, n_steps=5000, n_window=2000),
                               W.C3.with_(n_paths=3000, n_steps=5000, n_window=1000, prec=W.F64),
                               W.C2.with_(n_paths=3000, n_steps=5000, n_window=2000,
                                          noise=W.GAUSS | W.POISSON | W.JUMP_GRID)],
                         ids=["c2-f32", "c3-f64", "c2-jump-grid"])
def test_checkpoint_resume_bit_identical(w):
    """A checkpoint (host copy of the workspace + step count) resumed by bm_ensemble_attach,
    before and after the window start, gives what an uninterrupted run gives, bit for bit."""
    m, r = W.to_c(w)
    ref = B.Ensemble(m, r)
    ref.integrate(w.n_steps)
    a = ref.read()
    for cut in (1500, 3333):
        e = B.Ensemble(m, r)
        e.integrate(cut)
        ck = e.checkpoint()
        e.close()
        del e
        f = B.Ensemble(m, r, checkpoint=ck)
        assert f.steps == cut
        f.integrate(w.n_steps - cut)
        b = f.read()
        assert np.array_equal(a.x.numpy(), b.x.numpy()) and np.array_equal(a.v.numpy(), b.v.numpy())
        assert np.array_equal(a.noise.numpy(), b.noise.numpy())
        assert np.array_equal(a.vp.numpy(), b.vp.numpy(), equal_nan=True)
        sa, sb = ref.stats(), f.stats()
        assert (sa.mean, sa.se, sa.n) == (sb.mean, sb.se, sb.n)
