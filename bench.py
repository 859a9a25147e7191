#!/usr/bin/env python3
"""Benchmark of the Monte Carlo path on one MI355X.

One "step" = one full pass of the hot path over one synthetic batch: create the
ensemble (initial conditions), integrate the whole horizon with Algorithms 1-4,
and reduce <v> (eq. 31) in FP64 on the device.  Default workload: the inertial
Brownian motor with Gaussian + white Poissonian noise, 2^20 FP32 paths, 10^3
drive periods of 400 steps (4.19e11 path-steps per step).

Prints one JSON line with path-steps/s, the roofline of the integration kernel
(measured with HIP events on the stream it runs on) and the FP64 oracle timed on
the host's cores over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published figures: 256 CUs, 2.4 GHz.  Each CU has 4 SIMDs of 16 lanes,
# so the main VALU pipe retires 64 lane-instructions per CU per clock (one wave64
# instruction per CU-clock); transcendental instructions (cos, log, exp, sqrt, rcp)
# go to a separate unit that runs alongside it.  The published FP32 vector peak
# (157.3 TFLOP/s) needs packed FP32 FMAs (2 elements x 2 flops per lane-clock),
# which this library does not emit; FP64 FMAs run at the same lane rate.
N_CU, CLOCK_HZ, LANES_PER_CU = 256, 2.4e9, 64
VALU_LANE_OPS_PEAK = N_CU * LANES_PER_CU * CLOCK_HZ          # 3.93e13 lane-instr/s
FP32_PEAK_FLOPS = 157.3e12                                   # packed FP32 vector
FP64_PEAK_FLOPS = 78.6e12

# HBM traffic of k_advance on the default workload from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE), averaged over the two launches of one step and
# scaled by what the same counters read for a 1 GiB device copy (FETCH_SIZE
# reads 0.5 GiB for it: factor 2.0; WRITE_SIZE reads 1 GiB: factor 1.0).  Valid
# only while the integration kernel's sources hash to KERNEL_SOURCES_SHA256.
TRAFFIC_WORKLOAD = "inertial-poisson-f32-2^20"
TRAFFIC_BYTES_PER_LAUNCH = ((10528.0625 + 10335.0) / 2 * 2.0 + (28672.0 + 20480.0) / 2 * 1.0) * 1024
KERNEL_SOURCES = ("common.hpp", "paths.hpp", "paths_kernels.hpp", "paths_tu.inc", "paths_f32_in.hip",
                  "launch.hpp")
KERNEL_SOURCES_SHA256 = "d6fbeecabe7d6e2b68fcf7361058bc72e5508394e0aa8650ead8592aa18b704f"


def algorithmic_work(w):
    """(main-pipe VALU lane-ops, transcendental lane-ops, flops) per path-step.

    The cheapest direct form of Algorithms 1-4 (one op per add, multiply, FMA,
    compare, select or conversion; transcendentals -- cos, log, sqrt, sin -- apart,
    as they issue to their own unit; flops count an FMA as 2):
      drift evaluation (3 per step): V = sin 2 pi x: cos, 1 FMA; ratchet: cos, 2 FMA;
        tent: mul, floor, FMA, compare, select, add; inertial: + 1 FMA (-gamma v);
      Algorithm 1: inertial 8 FMA + 1 add, overdamped 4 FMA + 1 add (the noise
        increment is added once, and the predictor's and corrector's trapezoids
        share the base y + F1 dt/2), + 1 add for a kick;
      dichotomous level: 1 select + 2 adds; fold: 4 ops per 16 steps;
      Algorithm 2 (three-point): 2 compares + 2 selects + 2 shifts for the next
        base-6 digit + Philox4x32-10 (10 rounds x (2 wide products + 2 three-way
        xors) = 40 ops) per 16 steps;  normal increments: Philox per 4 steps,
        Box-Muller (8 ops + log, sqrt, cos, sin per pair) and the scale;
      Algorithm 3: 1 compare per step; per kick half a Philox block (20), the FP32
        countdown (8), the amplitude (4 + log), queue write and read (4);
      Algorithm 4: 1 compare per step; per flip a quarter block (10), countdown (8 +
        log), state flip (1), queue write and read (3).
    The jump-adapted grid adds, per kick, a Philox block for the piece increment (40 /
    16 or 40 / 4), the FP64 kick time (log, divide: ~30), the drive inside the step
    (3 + cos) and a second Algorithm 1 piece.
    """
    from paper_1409_4923_amd import workloads as W
    ops = trans = flops = 0.0
    inertial = w.dyn == W.INERTIAL
    if w.pot == W.POT_SIN:
        e_ops, e_tr, e_fl = 1, 1, 3
    elif w.pot == W.POT_RATCHET:
        e_ops, e_tr, e_fl = 2, 1, 5
    elif w.pot == W.POT_TENT:
        e_ops, e_tr, e_fl = 6, 0, 4
    else:
        e_ops, e_tr, e_fl = 0, 0, 0
    if inertial:
        e_ops, e_fl = e_ops + 1, e_fl + 2
    ops += 3 * e_ops
    trans += 3 * e_tr
    flops += 3 * e_fl + 3 * e_tr
    kick = (w.noise & W.POISSON) != 0
    if inertial:
        ops += 9 + (1 if kick else 0)
        flops += 17 + (1 if kick else 0)
    else:
        ops += 5 + (1 if kick else 0)
        flops += 9 + (1 if kick else 0)
    ops += 4.0 / 16.0
    flops += 2.0 / 16.0
    if w.noise & W.GAUSS:
        ops += 6 + 40.0 / 16.0
    if w.noise & W.NORMAL:
        ops += 40.0 / 4.0 + 4 + 1
        trans += 2
        flops += 4
    h = w.step()
    if kick:
        p_kick = -math.expm1(-w.lam * h)
        ops += 1 + p_kick * (20 + 8 + 4 + 4)
        trans += p_kick * 2
        flops += p_kick * 6
        if w.noise & W.JUMP_GRID:
            piece = 40.0 / 16.0 + 6 if (w.noise & W.GAUSS) else (40.0 / 4.0 + 5 if (w.noise & W.NORMAL) else 0)
            ops += p_kick * (piece + 30 + 3 + (9 if inertial else 5) + 3 * e_ops)
            trans += p_kick * (1 + 3 * e_tr)
            flops += p_kick * (20 + (17 if inertial else 9) + 3 * e_fl)
    if w.noise & W.DICH:
        p_flip = max(-math.expm1(-w.mua * h), -math.expm1(-w.mub * h))
        ops += 3 + 1 + p_flip * (10 + 8 + 1 + 3)
        trans += p_flip
        flops += 2 + p_flip
    return ops, trans, flops


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1409_4923_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


ORACLE_SUBSET = 4096


def _c2_jump_grid():
    from paper_1409_4923_amd import workloads as W
    return W.C2.with_(name="inertial-poisson-jump-grid-f32-2^20", noise=W.GAUSS | W.POISSON | W.JUMP_GRID)


def host_threads() -> int:
    """Host threads this process may run on (its CPU affinity set)."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def oracle_baseline(w, seconds: float | None, threads: int):
    """Time the FP64 oracle on paths 0..S-1 of the workload over its full horizon:
    S = the 4096-path comparison subset (seconds None), or S sized from a short pilot
    so that the run takes about `seconds`."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import to_oracle
    oracle.build(force=False)
    P = to_oracle(w)
    if seconds is None:
        S = min(ORACLE_SUBSET, w.n_paths)
    else:
        pilot_paths, pilot_steps = 4 * threads, min(2000, w.n_steps)
        t = time.perf_counter()
        oracle.run(P, 0, pilot_paths, pilot_steps, threads=threads)
        rate = pilot_paths * pilot_steps / (time.perf_counter() - t)
        S = int(rate * seconds / w.n_steps) // threads * threads
        S = max(threads, min(S, ORACLE_SUBSET, w.n_paths))
    t = time.perf_counter()
    st = oracle.run(P, 0, S, w.n_steps, threads=threads)
    el = time.perf_counter() - t
    vp = oracle.velocity(P, st, w.n_steps)
    s = oracle.stats(vp)
    return dict(value=S * w.n_steps / el, unit="path-steps/s", cores=threads, kind="oracle",
                sample="paths 0..%d of the workload over its full %d-step horizon (%.3g path-steps, %.1f s)"
                       % (S - 1, w.n_steps, S * w.n_steps, el),
                mean_v=s.mean, se=s.se, n_paths=S, vp=vp)


def oracle_check(gpu_vp, gpu_stats, ob):
    """<v> of the GPU against the FP64 oracle on the same paths (same random streams):
    unpaired (subset means), paired (per-path differences) and full ensemble against the
    oracle subset, each at 3 standard errors."""
    import numpy as np
    import oracle
    S = ob["n_paths"]
    g = oracle.stats(gpu_vp[:S])
    d = oracle.stats(gpu_vp[:S] - ob["vp"])
    return {"oracle_paths": S, "oracle_mean_v": ob["mean_v"], "oracle_se_v": ob["se"],
            "gpu_subset_mean_v": g.mean, "gpu_subset_se_v": g.se,
            "paired_mean_diff": d.mean, "paired_se": d.se,
            "unpaired_within_3se": abs(g.mean - ob["mean_v"]) <= 3 * math.hypot(g.se, ob["se"]),
            "paired_within_3se": abs(d.mean) <= 3 * d.se + 1e-12,
            "ensemble_within_3se": abs(gpu_stats.mean - ob["mean_v"]) <= 3 * math.hypot(gpu_stats.se, ob["se"]),
            "paths_within_1e-3": float(np.mean(np.abs(gpu_vp[:S] - ob["vp"])
                                               <= 1e-3 * np.maximum(1.0, np.abs(ob["vp"]))))}


def time_ensemble(w, steps: int, warmup: int, tune=None):
    """Run `warmup` + `steps` passes of the hot path (create with initial conditions,
    integrate the horizon, reduce eq. 31) on torch's current stream.  Returns (wall
    seconds of the timed passes, integration seconds per pass from HIP events on that
    stream, bm_stats of the last pass, per-path velocities of paths 0..4095)."""
    import torch
    from paper_1409_4923_amd import bmotor as B
    from paper_1409_4923_amd import workloads as W
    dev = torch.device("cuda:0")
    m, r = W.to_c(w)
    ws_bytes = B.bm_ensemble_workspace_size(m, r)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    out = torch.empty(B.STATS_BYTES, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    n_sub = min(ORACLE_SUBSET, w.n_paths)
    vp = torch.empty(n_sub, dtype=torch.float64, device=dev)
    events = []

    def one_pass(timed: bool, last: bool):
        h = B.bm_ensemble_create(m, r, ws.data_ptr(), ws_bytes, stream.cuda_stream)
        try:
            if tune is not None:
                B.bm_ensemble_set_tune(h, tune)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            B.bm_integrate(h, w.n_steps)
            e1.record(stream)
            B.bm_reduce(h, out.data_ptr())
            if last:
                B.bm_read_paths(h, 0, n_sub, None, None, None, vp.data_ptr())
        finally:
            B.bm_ensemble_destroy(h)
        if timed:
            events.append((e0, e1))

    for i in range(warmup):
        one_pass(False, False)
        print("%s: warmup pass %d done" % (w.name, i), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        one_pass(True, False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print("%s: timed %d passes in %.3f s" % (w.name, steps, wall), file=sys.stderr, flush=True)
    int_s = sum(a.elapsed_time(b) for a, b in events) / 1e3 / steps
    one_pass(False, True)          # untimed: the per-path velocities for the oracle comparison
    torch.cuda.synchronize()
    st = B.stats_from_bytes(out.cpu().numpy().tobytes())
    return wall, int_s, st, vp.cpu().numpy()


def roofline_of(w, int_s: float):
    from paper_1409_4923_amd import workloads as W
    ops, trans, flops = algorithmic_work(w)
    ps = w.path_steps()
    launches = 2 if 0 < w.n_window < w.n_steps else 1
    peak_flops = FP32_PEAK_FLOPS if w.prec == W.F32 else FP64_PEAK_FLOPS
    achieved = ops * ps / int_s
    return {"bound": "alu", "kernel": "k_advance (integration loop)",
            "achieved": achieved / 1e12, "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "TOP/s (VALU lane-ops)",
            "frac": achieved / VALU_LANE_OPS_PEAK, "traffic": None,
            "ops_per_path_step": ops, "trans_ops_per_path_step": trans,
            "path_steps_per_launch": ps / launches, "kernel_ms_per_launch": int_s * 1e3 / launches,
            "launches_per_step": launches,
            "fp32_flops" if w.prec == W.F32 else "fp64_flops": {
                "flops_per_path_step": flops, "achieved_tflops": flops * ps / int_s / 1e12,
                "peak_tflops": peak_flops / 1e12, "frac": flops * ps / int_s / peak_flops}}


def ensemble_leg(w, steps: int, warmup: int, threads: int, with_oracle: bool):
    """A timed pass of another workload: path-steps/s, the roofline of its
    integration kernel and its <v> against the FP64 oracle on paths 0..4095."""
    wall, int_s, st, vp = time_ensemble(w, steps, warmup)
    res = {"workload": w.name, "n_paths": w.n_paths, "n_steps": w.n_steps, "n_window": w.n_window,
           "noise_mask": w.noise, "dtype": "f32" if w.prec == 1 else "f64", "steps": steps,
           "path_steps_per_s": w.path_steps() * steps / wall, "ms_per_step": 1e3 * wall / steps,
           "mean_v": st.mean, "se_v": st.se, "n_nonfinite": st.n_nonfinite, "roofline": roofline_of(w, int_s)}
    if with_oracle:
        ob = oracle_baseline(w, None, threads)
        res["oracle"] = oracle_check(vp, st, ob)
        res["oracle"]["path_steps_per_s"] = ob["value"]
        res["oracle"]["cores"] = threads
    return res


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


FP64_SAMPLE_STEPS = 20000


def fp64_rate(w) -> float:
    """Path-steps/s of the workload with FP64 paths (all paths, FP64_SAMPLE_STEPS steps,
    timed with HIP events after a 256-step warm-up)."""
    import torch
    from paper_1409_4923_amd import bmotor as B
    from paper_1409_4923_amd import workloads as W
    w64 = w.with_(prec=W.F64, n_steps=FP64_SAMPLE_STEPS, n_window=0)
    m, r = W.to_c(w64)
    e = B.Ensemble(m, r)
    e.integrate(256)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    e.integrate(FP64_SAMPLE_STEPS)
    e1.record()
    torch.cuda.synchronize()
    return w64.n_paths * FP64_SAMPLE_STEPS / (e0.elapsed_time(e1) / 1e3)


def scan_leg(args):
    """Batched scan of the 4096-point inertial workload: autotune on scaled-down horizons,
    then one graph launch timed with HIP events on the plan's stream."""
    import torch
    from paper_1409_4923_amd import bmotor as B
    from paper_1409_4923_amd import workloads as W
    pts = W.c4_points()
    mr = [W.to_c(w) for w in pts]
    models, runs = [m for m, _ in mr], [r for _, r in mr]
    nb = B.bm_scan_workspace_size(models, runs)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    res = torch.empty(len(pts) * B.STATS_BYTES, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    tune, tune_ms = B.bm_scan_autotune(models, runs, 20000, ws.data_ptr(), nb, res.data_ptr(), stream.cuda_stream)
    t_tune = time.perf_counter() - t0
    h = B.bm_scan_plan_create(models, runs, None, ws.data_ptr(), nb, res.data_ptr(), stream.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    B.bm_scan_plan_launch(h)
    e1.record(stream)
    torch.cuda.synchronize()
    B.bm_scan_plan_destroy(h)
    sec = e0.elapsed_time(e1) / 1e3
    st = B.stats_array_from_bytes(res.cpu().numpy().tobytes(), len(pts))
    total = sum(w.path_steps() for w in pts)
    ops, _, _ = algorithmic_work(pts[0])
    print("scan leg: %.3g path-steps in %.3f s" % (total, sec), file=sys.stderr, flush=True)
    return {"workload": "inertial-scan-4096-points", "n_points": len(pts), "path_steps": total,
            "seconds": sec, "path_steps_per_s": total / sec, "points_per_s": len(pts) / sec,
            "tune": {"paths_per_lane": tune.paths_per_lane, "block": tune.block,
                     "groups_per_cu": tune.groups_per_cu, "autotune_s": t_tune},
            "valu_frac": ops * total / sec / VALU_LANE_OPS_PEAK,
            "n_nonfinite_points": int(sum(1 for x in st if not math.isfinite(x.mean)))}


def scheme_leg(args):
    """Simplified (three-point increments, eq. 25) against non-simplified (normal
    increments by Box-Muller) predictor-corrector on the inertial Gaussian model with
    its own horizon (2 x 10^4 steps, <v> over the last half), 2^20 paths, FP32 and
    FP64: path-steps/s of each, and <v> of each next to a normal-increment run at a
    quarter of the step as the small-dt reference."""
    import torch
    from paper_1409_4923_amd import bmotor as B
    from paper_1409_4923_amd import workloads as W
    base = W.C1.with_(n_paths=1 << 20)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = torch.empty(B.STATS_BYTES, dtype=torch.uint8, device=dev)

    def run(w, reps=5):
        m, r = W.to_c(w)
        nb = B.bm_ensemble_workspace_size(m, r)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        best = None
        for _ in range(reps):
            h = B.bm_ensemble_create(m, r, ws.data_ptr(), nb, stream.cuda_stream)
            try:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                B.bm_integrate(h, w.n_steps)
                e1.record(stream)
                B.bm_reduce(h, out.data_ptr())
            finally:
                B.bm_ensemble_destroy(h)
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / 1e3
            best = sec if best is None else min(best, sec)
        st = B.stats_from_bytes(out.cpu().numpy().tobytes())
        return {"path_steps_per_s": w.path_steps() / best, "mean_v": st.mean, "se_v": st.se}

    res = {"workload": "inertial-gauss-2^20-paths-2e4-steps"}
    for prec, name in ((W.F32, "f32"), (W.F64, "f64")):
        a = run(base.with_(prec=prec, noise=W.GAUSS))
        b = run(base.with_(prec=prec, noise=W.NORMAL))
        res[name] = {"three_point": a, "normal": b, "speedup": a["path_steps_per_s"] / b["path_steps_per_s"]}
    ref = run(base.with_(prec=W.F32, noise=W.NORMAL, spp=4 * base.spp, n_steps=4 * base.n_steps,
                         n_window=4 * base.n_window), reps=1)
    # best of five launches per variant: each lasts only some 20 ms
    res["reference_quarter_dt"] = {"mean_v": ref["mean_v"], "se_v": ref["se_v"]}
    for k in ("three_point", "normal"):
        d = res["f32"][k]["mean_v"] - ref["mean_v"]
        res["f32"][k]["rel_dev_from_reference"] = d / abs(ref["mean_v"]) if ref["mean_v"] else None
        res["f32"][k]["dev_in_se"] = d / math.hypot(res["f32"][k]["se_v"], ref["se_v"])
    print("scheme leg: three-point / normal speed %.2fx (f32), %.2fx (f64)"
          % (res["f32"]["speedup"], res["f64"]["speedup"]), file=sys.stderr, flush=True)
    return res


def infer_leg(args):
    """Inference alone: a 5-member ensemble (initial weights) on args.queries queries:
    30 untimed forwards (the clocks settle), then 20 back to back between two HIP
    events (the mean per forward); the MFMA figure the surrogate leg also reports,
    without training first."""
    import torch
    from paper_1409_4923_amd import bmotor as B
    from paper_1409_4923_amd import workloads as W
    sur = B.Surrogate(5, seed=11)
    xq = torch.tensor(W.surrogate_queries(args.queries, seed=303), device="cuda")
    for _ in range(30):
        sur.forward(xq)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        sur.forward(xq)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    flops = args.queries * 5 * 2 * (5 * 256 + 2 * 256 * 256 + 256)
    return {"queries": args.queries, "members": 5, "forward_ms": ms, "timed_forwards": 20,
            "achieved": flops / ms / 1e9, "peak": 2500.0, "unit": "TFLOP/s (BF16 MFMA)",
            "frac": flops / ms / 1e9 / 2500.0}


def train_leg(args):
    """One training step of the 5-member ensemble (backward of the MSE + Adam) on
    minibatches of 1024 and 4096 rows drawn from 10^5 rows: 10 untimed steps, then 200
    timed with HIP events (ms per step)."""
    import numpy as np
    import torch
    from paper_1409_4923_amd import bmotor as B
    from paper_1409_4923_amd import workloads as W
    sur = B.Surrogate(5, seed=7)
    n = 100_000
    x = torch.tensor(W.surrogate_queries(n, seed=1), device="cuda")
    y = torch.tensor(np.random.default_rng(2).normal(0.0, 0.01, n).astype(np.float32), device="cuda")
    rng = np.random.default_rng(0)
    out = {}
    for batch in (1024, 4096):
        idx = torch.tensor(rng.integers(0, n, (210, 5, batch)).astype(np.int32), device="cuda")
        for s in range(10):
            sur.backward(x, y, idx[s])
            sur.adam(1e-3)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for s in range(10, 210):
            sur.backward(x, y, idx[s])
            sur.adam(1e-3)
        e1.record()
        torch.cuda.synchronize()
        out["ms_per_step_batch_%d" % batch] = e0.elapsed_time(e1) / 200
    out["members"] = 5
    return out


def surrogate_leg(args):
    """Learned surrogate of <v>(a, omega, F, D, gamma) with Monte Carlo fallback.

    Labels: args.labels points (gamma ~ U[0.5, 2]) by one batched scan at
    args.label_paths paths x args.label_periods periods.  Truth: args.heldout points
    at args.truth_paths x args.label_periods.  Plain-MC cost of point i at
    |d<v>| <= 0.01 (3 SE <= 0.01): N_i = (3 sigma_i / 0.01)^2 paths (at least 64) of
    the same horizon at the measured scan throughput.  Surrogate+fallback: the
    10^6-query routing time plus, for the routed fraction, the mean MC cost of the
    held-out points the ensemble routes (they are the costly, multi-attractor ones).
    A point counts as delivered at tolerance if MC computed it or if the ensemble
    answered it within 0.01 of the truth (measured on the held-out points).  The
    amortised figure also charges label generation and training to the 10^6 queries.
    A second baseline gives plain MC (and the fallback) one path count for all points,
    the largest any held-out point needs, as MC must without knowing sigma_i.  The
    "adaptive_fallback" figures price both sides as they would run without knowing
    sigma_i: sequential MC (pilot, then top-ups from the spread so far) on every
    held-out point, and the same on the routed ones for the fallback."""
    import numpy as np
    import torch
    from paper_1409_4923_amd import bmotor as B
    from paper_1409_4923_amd import surrogate as S
    from paper_1409_4923_amd import workloads as W
    thr, tol = 0.005, 0.01
    xl = W.surrogate_queries(args.labels, seed=101)
    lab = S.monte_carlo(xl, args.label_paths, args.label_periods, seed=1, first_point=0)
    t_label = lab.seconds
    yl = lab.mean
    print("surrogate: %d labels in %.1f s" % (args.labels, lab.seconds), file=sys.stderr, flush=True)
    sur = B.Surrogate(5, seed=7)
    t0 = time.perf_counter()
    hist = S.train(sur, xl, yl, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print("surrogate: trained in %.1f s, loss %.4g -> %.4g" % (t_train, hist[0], hist[-1]), file=sys.stderr,
          flush=True)
    # active learning: label the candidates the ensemble disagrees on most, retrain on all
    rounds = []
    for rd in range(args.active_rounds):
        xc = W.surrogate_queries(args.active_candidates, seed=500 + rd)
        t0 = time.perf_counter()
        pick = S.uncertain_points(sur, xc, args.active_labels, thr)
        t_pick = time.perf_counter() - t0
        if len(pick) == 0:
            break
        lab_a = S.monte_carlo(xc[pick], args.label_paths, args.label_periods, seed=1,
                              first_point=(1 << 22) + rd * args.active_candidates)
        xl = np.concatenate([xl, xc[pick]])
        yl = np.concatenate([yl, lab_a.mean])
        t0 = time.perf_counter()
        h = S.train(sur, xl, yl, epochs=args.active_epochs, batch=args.batch, lr=args.lr / 2, seed=4 + rd)
        torch.cuda.synchronize()
        t_tr = time.perf_counter() - t0
        t_label += lab_a.seconds + t_pick
        t_train += t_tr
        rounds.append({"labels_added": int(len(pick)), "label_seconds": lab_a.seconds, "train_seconds": t_tr,
                       "train_loss": [h[0], h[-1]]})
        print("surrogate: active round %d: %d labels (%.1f s), retrained in %.1f s" %
              (rd, len(pick), lab_a.seconds, t_tr), file=sys.stderr, flush=True)
    xh = W.surrogate_queries(args.heldout, seed=202)
    truth = S.monte_carlo(xh, args.truth_paths, args.label_periods, seed=2, first_point=1 << 24)
    rate = truth.path_steps / truth.seconds                              # MC path-steps/s on this workload
    n_steps = args.label_periods * S.SPP
    need = np.maximum(64.0, np.ceil((3.0 * np.nan_to_num(truth.std, nan=1.0) / tol) ** 2))
    cost = need * n_steps / rate                                         # seconds per point at |d| <= tol
    mc_cost = float(np.mean(cost))
    # surrogate accuracy on the held-out points it answers itself
    xd = torch.tensor(xh, device="cuda")
    mean, std, fidx, fcnt = sur.query(xd, thr)
    mean, std = mean.cpu().numpy(), std.cpu().numpy()
    keep = std <= thr
    err = np.abs(mean - truth.mean)
    good = float(np.mean(err[keep] <= tol)) if keep.any() else 0.0
    fb_cost = float(np.mean(cost[~keep])) if (~keep).any() else mc_cost
    # routing 10^6 queries
    xq = torch.tensor(W.surrogate_queries(args.queries, seed=303), device="cuda")
    sur.query(xq, thr)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, _, _, qcnt = sur.query(xq, thr)
    e1.record()
    torch.cuda.synchronize()
    t_query = e0.elapsed_time(e1) / 1e3
    n_q = args.queries
    f = int(qcnt.item()) / n_q
    delivered = n_q * ((1.0 - f) * good + f)
    t_sur = t_query + f * n_q * fb_cost
    sur_rate = delivered / t_sur
    sur_rate_amortised = delivered / (t_sur + t_label + t_train)
    mc_rate = 1.0 / mc_cost
    # Plain MC that does not know sigma_i in advance: one path count for every point,
    # the largest the held-out points need; the fallback then pays the same.
    fixed_cost = float(np.max(need)) * n_steps / rate
    sur_rate_fixed = delivered / (t_query + f * n_q * fixed_cost)
    # A threshold calibrated on held-out data instead of fixed: on the even-indexed
    # held-out points, the largest threshold on a grid whose answered points keep a p95
    # error <= tol and 95% within tol; judged on the odd-indexed points (fallback cost
    # and accuracy) and on the 10^6 queries (fallback fraction).
    cal_a, cal_b = np.arange(0, len(xh), 2), np.arange(1, len(xh), 2)
    thr_cal, sweep = S.calibrate_threshold(std[cal_a], err[cal_a], tol, [thr * 2.0 ** (k / 4.0) for k in range(17)])
    thr_cal = thr if thr_cal is None else thr_cal
    kb = std[cal_b] <= thr_cal
    good_b = float(np.mean(err[cal_b][kb] <= tol)) if kb.any() else 0.0
    fb_cost_b = float(np.mean(cost[cal_b][~kb])) if (~kb).any() else mc_cost
    _, _, _, qc = sur.query(xq, thr_cal)
    f_cal = int(qc.item()) / n_q
    deliv_cal = n_q * ((1.0 - f_cal) * good_b + f_cal)
    t_sur_cal = t_query + f_cal * n_q * fb_cost_b
    calibrated = {"threshold": thr_cal, "sweep_even_half": sweep, "fallback_fraction": f_cal,
                  "answered_odd_half": float(kb.mean()),
                  "abs_err_answered_p95_odd_half": float(np.percentile(err[cal_b][kb], 95)) if kb.any() else None,
                  "within_tol_answered_odd_half": good_b,
                  "gain": deliv_cal / t_sur_cal * mc_cost,
                  "gain_amortised": deliv_cal / (t_sur_cal + t_label + t_train) * mc_cost}
    print("surrogate: calibrated threshold %.4f: fallback %.3f, gain %.3f" % (thr_cal, f_cal, calibrated["gain"]),
          file=sys.stderr, flush=True)
    # Both sides as run, without knowing sigma_i: sequential MC (a 64-path pilot, then
    # up to three top-ups sized from the spread so far) on every held-out point gives
    # plain MC's cost per point; the same runs on the points the ensemble routes give
    # the fallback's.  Costs are the path-steps run at the measured throughput; the
    # means are checked against the truth scan.
    ad = S.adaptive_monte_carlo(xh, tol, args.label_periods, seed=5, first_point=1 << 25)
    ad_cost = ad.n_paths * n_steps / rate
    z = np.abs(ad.mean - truth.mean) / np.sqrt(ad.se ** 2 + truth.se ** 2)
    mc_cost_seq = float(np.mean(ad_cost))
    fb_cost_seq = float(np.mean(ad_cost[~keep])) if (~keep).any() else mc_cost_seq
    sur_rate_seq = delivered / (t_query + f * n_q * fb_cost_seq)
    adaptive = {"paths_per_point_mean": float(np.mean(ad.n_paths)),
                "paths_per_point_routed_mean": float(np.mean(ad.n_paths[~keep])) if (~keep).any() else None,
                "paths_per_point_max": int(np.max(ad.n_paths)), "scan_seconds": ad.seconds,
                "mc_seconds_per_point": mc_cost_seq, "fallback_mc_seconds_per_point": fb_cost_seq,
                "three_se_within_tol": float(np.mean(3.0 * ad.se <= tol)),
                "within_3_combined_se_of_truth": float(np.mean(z <= 3.0)),
                "gain": sur_rate_seq * mc_cost_seq,
                "gain_amortised": delivered / (t_query + f * n_q * fb_cost_seq + t_label + t_train) * mc_cost_seq}
    print("surrogate: sequential MC on %d held-out points: %.0f paths each (%.0f where routed), gain %.3f"
          % (len(xh), np.mean(ad.n_paths), adaptive["paths_per_point_routed_mean"] or 0.0, adaptive["gain"]),
          file=sys.stderr, flush=True)
    flops = n_q * 5 * 2 * (5 * 256 + 2 * 256 * 256 + 256)
    return {"labels": int(len(xl)), "labels_uniform": args.labels, "active_rounds": rounds,
            "label_budget": [args.label_paths, args.label_periods],
            "label_seconds": t_label, "train_seconds": t_train, "epochs": args.epochs, "batch": args.batch,
            "train_loss": [hist[0], hist[-1]],
            "heldout": args.heldout, "truth_paths": args.truth_paths, "truth_se_median": float(np.median(truth.se)),
            "queries": n_q, "threshold": thr, "query_seconds": t_query,
            "fallback_fraction": f, "answered_heldout": int(keep.sum()),
            "abs_err_answered_p50": float(np.percentile(err[keep], 50)) if keep.any() else None,
            "abs_err_answered_p95": float(np.percentile(err[keep], 95)) if keep.any() else None,
            "within_tol_answered": good,
            "mc_seconds_per_point": mc_cost, "fallback_mc_seconds_per_point": fb_cost,
            "mc_points_per_s_at_tol": mc_rate, "surrogate_points_per_s_at_tol": sur_rate,
            "gain": sur_rate / mc_rate, "gain_amortised": sur_rate_amortised / mc_rate,
            "fixed_n_paths": float(np.max(need)), "mc_points_per_s_fixed_n": 1.0 / fixed_cost,
            "gain_vs_fixed_n": sur_rate_fixed * fixed_cost,
            "adaptive_fallback": adaptive,
            "calibrated_threshold": calibrated,
            "mlp_inference": {"achieved": flops / t_query / 1e12, "peak": 2500.0, "unit": "TFLOP/s (BF16 MFMA)",
                              "frac": flops / t_query / 2.5e15}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c2jump", "c3"],
                    help="main workload: c2 = inertial Poisson (fixed grid), c2jump = the same on the "
                         "jump-adapted grid, c3 = overdamped dichotomous, c1 = inertial Gaussian FP64")
    ap.add_argument("--ppl", type=int, default=0, help="paths per lane (0: library default)")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="c3,c2jump,scan,scheme,train,infer,surrogate",
                    help="extra legs: c3, c2jump, scan, scheme, train, infer, surrogate (or none)")
    ap.add_argument("--labels", type=int, default=60_000, help="uniform labels before active learning")
    ap.add_argument("--active-rounds", type=int, default=0,
                    help="rounds of labels where the ensemble disagrees most (measured to raise the fallback "
                         "fraction on this domain, so off by default)")
    ap.add_argument("--active-labels", type=int, default=100_000, help="labels added per active round")
    ap.add_argument("--active-candidates", type=int, default=1_000_000)
    ap.add_argument("--active-epochs", type=int, default=100)
    ap.add_argument("--label-paths", type=int, default=256)
    ap.add_argument("--label-periods", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=1024, help="surrogate training minibatch")
    ap.add_argument("--lr", type=float, default=2e-3, help="surrogate training learning rate (start)")
    ap.add_argument("--heldout", type=int, default=10_000)
    ap.add_argument("--truth-paths", type=int, default=4096)
    ap.add_argument("--queries", type=int, default=1_000_000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (for scaling HBM counters) and exit")
    ap.add_argument("--calibrate-valu", action="store_true",
                    help="only measure the device's vector-ALU issue rate (FMA chains; FMA + compare + select; "
                         "FMA + exp2) "
                         "against the roofline peak and exit")
    args = ap.parse_args()
    if args.calibrate_valu:
        import torch
        from paper_1409_4923_amd import probe as PR
        n = 256 * 32 * 256                        # 32 work-groups of 256 lanes per CU
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        rec = {"peak_lane_ops_per_s": VALU_LANE_OPS_PEAK}
        for mix, name in ((0, "fma"), (1, "fma_cmp_select"), (2, "fma_exp2")):
            r = PR.valu_probe(mix, 20000, out.data_ptr(), n, stream)
            rec[name] = {"lane_ops_per_s": r, "frac_of_peak": r / VALU_LANE_OPS_PEAK}
        print(json.dumps({"valu_probe": rec}), flush=True)
        return
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "read_bytes": n, "write_bytes": n}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(paths and parameter points would shard across GPUs by index range).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1409_4923_amd import bmotor as B
    from paper_1409_4923_amd import workloads as W

    C2_JUMP_GRID = _c2_jump_grid()
    w = {"c1": W.C1, "c2": W.C2, "c2jump": C2_JUMP_GRID, "c3": W.C3}[args.config]
    torch.cuda.set_device(torch.device("cuda:0"))
    tune = B.make_tune(args.ppl, args.block) if args.ppl else None
    wall, int_s, st, vp = time_ensemble(w, args.steps, args.warmup, tune)
    value = w.path_steps() * args.steps / wall
    roof = roofline_of(w, int_s)
    if w.name == TRAFFIC_WORKLOAD and kernel_sources_sha256() == KERNEL_SOURCES_SHA256:
        roof["traffic"] = TRAFFIC_BYTES_PER_LAUNCH
    rec = {
        "metric": "path-steps/s",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.prec == W.F32 else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_paths": w.n_paths, "n_steps": w.n_steps,
                   "n_window": w.n_window, "dt": w.step(), "noise_mask": w.noise,
                   "parallelism": "single-gpu", "paths_per_lane": args.ppl or 1, "block": args.block},
        "mean_v": st.mean, "se_v": st.se, "n_nonfinite": st.n_nonfinite,
        "roofline": roof,
        "cpu_baseline": None,
    }
    threads = host_threads()
    if not args.no_cpu_baseline:
        # the oracle on the 4096-path comparison subset, on every host thread this
        # process may use, timed in the same run
        cb = oracle_baseline(w, None, threads)
        rec["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        rec["cpu_baseline"]["host_cpus"] = os.cpu_count()
        rec["cpu_baseline"]["host_cpu"] = host_cpu_model()
        rec["oracle"] = oracle_check(vp, st, cb)
        rec["mean_v_within_3se"] = rec["oracle"]["ensemble_within_3se"]
        rec["speedup_vs_oracle"] = value / cb["value"]
        # the paper's GPU/CPU figure is against one CPU core
        one = oracle_baseline(w, args.cpu_seconds / 2, 1)
        rec["cpu_baseline"]["single_core"] = {"value": one["value"], "sample": one["sample"]}
        rec["speedup_vs_one_core"] = value / one["value"]
        # the same workload with FP64 paths, against the same (FP64) oracle core
        f64 = fp64_rate(w)
        rec["fp64_paths"] = {"path_steps_per_s": f64, "speedup_vs_one_core": f64 / one["value"],
                             "sample": "all %d paths, %d steps" % (w.n_paths, FP64_SAMPLE_STEPS)}
        # the paper's figures (Sec. 7): GPU over the same program on one CPU core
        rec["paper_speedup"] = {"fp32": 3000, "fp64": [700, 400],
                                "hardware": "NVIDIA GeForce GTX TITAN Black vs one core of an "
                                            "Intel Core i7-3930K at 3.2 GHz"}
    legs = [l for l in args.legs.split(",") if l and l != "none"]
    if "c3" in legs and w.name != W.C3.name:
        rec["c3"] = ensemble_leg(W.C3, 2, 1, threads, not args.no_cpu_baseline)
    if "c2jump" in legs and w.name != C2_JUMP_GRID.name:
        rec["c2_jump_adapted_grid"] = ensemble_leg(C2_JUMP_GRID, 2, 1, threads, not args.no_cpu_baseline)
    if "scan" in legs:
        rec["scan"] = scan_leg(args)
    if "scheme" in legs:
        rec["scheme"] = scheme_leg(args)
    if "train" in legs:
        rec["train"] = train_leg(args)
    if "infer" in legs:
        rec["infer"] = infer_leg(args)
    if "surrogate" in legs:
        rec["surrogate"] = surrogate_leg(args)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
