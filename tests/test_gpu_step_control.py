"""Step-size control on chi (the paragraph after Algorithm 1) on the GPU, through the
C ABI, against the FP64 oracle: per-path parity with the control active (levels and
step counts bit-exact, positions and velocities within 1e-9), FP32 <v> within 3 SE,
invariance under chunking and work-group size, and the state records."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from helpers import ORACLE_THREADS, oracle_paths, say, to_oracle
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


TENT = W.Workload(name="tent-gauss", dyn=W.OVERDAMPED, pot=W.POT_TENT, noise=W.GAUSS, prec=W.F64, F=0.5, D=0.2,
                  dt=0.05, n_paths=200, n_steps=600, n_window=200, x0_lo=0.0, x0_hi=2.0)
CASES = {
    "inertial-gauss": W.C1.with_(n_paths=200, n_steps=600, n_window=200, step_tol=3e-6, max_halvings=3),
    "inertial-poisson": W.C2.with_(prec=W.F64, n_paths=200, n_steps=600, n_window=200, step_tol=3e-6,
                                   max_halvings=3),
    "ratchet-dich": W.C3.with_(prec=W.F64, n_paths=200, n_steps=600, n_window=200, step_tol=1e-7,
                               max_halvings=4),
    "tent-gauss": TENT.with_(step_tol=1e-3, max_halvings=4),
    "tent-poisson-dich": TENT.with_(noise=W.GAUSS | W.POISSON | W.DICH, lam=3.0, zeta=0.2, Fa=0.5, Fb=1.0,
                                    mua=1.0, mub=2.0, step_tol=1e-3, max_halvings=3),
}


def _records(w, chunks, tune=None):
    m, r = W.to_c(w)
    e = B.Ensemble(m, r, tune=tune)
    for c in chunks:
        e.integrate(c)
    return e, B.records(e.read_state())


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_per_path_parity_with_step_control(name):
    w = CASES[name]
    say("step control FP64 parity:", name)
    e, rec = _records(w, [250, 350])
    ps = e.read()
    xu, v, noise, st = oracle_paths(w, 0, w.n_paths, w.n_steps)
    assert np.array_equal(rec["step_level"], st["lev"].astype(np.int64))
    assert np.array_equal(rec["steps_taken"], st["kA"].astype(np.int64))
    assert rec["steps_taken"].max() > 1.2 * w.n_steps             # the control refined
    assert np.array_equal(ps.noise.numpy(), noise)
    err = np.abs(ps.x.numpy() - xu) / np.maximum(1.0, np.abs(xu))
    assert err.max() <= 1e-9, err.max()
    if w.dyn == W.INERTIAL:
        errv = np.abs(ps.v.numpy() - v) / np.maximum(1.0, np.abs(v))
        assert errv.max() <= 1e-9, errv.max()
    vo = oracle.velocity(to_oracle(w), st, w.n_steps)
    assert np.allclose(ps.vp.numpy(), vo, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("name", ["inertial-gauss", "tent-gauss"])
def test_fp32_mean_velocity_within_3se(name):
    w = CASES[name].with_(prec=W.F32, n_paths=4096, n_steps=4000, n_window=1000)
    m, r = W.to_c(w)
    e = B.Ensemble(m, r)
    e.integrate(w.n_steps)
    s = e.stats()
    ps = e.read()
    P = to_oracle(w)
    st = oracle.run(P, 0, w.n_paths, w.n_steps, threads=ORACLE_THREADS, n_paths=w.n_paths)
    vo = oracle.velocity(P, st, w.n_steps)
    so = oracle.stats(vo)
    d = oracle.stats(ps.vp.numpy() - vo)
    say("step control FP32 %s: gpu %.6f +- %.6f, oracle %.6f +- %.6f, steps/dt %.2f"
        % (name, s.mean, s.se, so.mean, so.se, st["kA"].mean() / w.n_steps))
    assert s.n == w.n_paths and s.n_nonfinite == 0
    assert abs(s.mean - so.mean) <= 3.0 * math.hypot(s.se, so.se)
    assert abs(d.mean) <= 3.0 * d.se + 1e-12


@pytest.mark.parametrize("prec", [W.F32, W.F64])
def test_chunks_and_launch_shape_do_not_change_results(prec):
    w = CASES["tent-poisson-dich"].with_(prec=prec, n_paths=1000)
    _, a = _records(w, [600])
    _, b = _records(w, [1, 199, 17, 383])
    assert a.tobytes() == b.tobytes()
    for block in (64, 128, 512):
        _, c = _records(w, [600], tune=B.make_tune(1, block))
        assert a.tobytes() == c.tobytes(), block


def test_records_resume_bit_identical_under_step_control():
    w = CASES["ratchet-dich"].with_(prec=W.F32, n_paths=777)
    m, r = W.to_c(w)
    _, ref = _records(w, [600])
    e, rec = _records(w, [333])
    f = B.Ensemble.resume(m, r, 333)
    f.write_state(rec)
    f.integrate(267)
    assert B.records(f.read_state()).tobytes() == ref.tobytes()


def test_step_control_arguments_checked():
    m, r = W.to_c(CASES["inertial-gauss"])
    e = B.Ensemble(m, r)
    with pytest.raises(B.BMError):
        e.set_tune(B.make_tune(2, 128))
