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

# MI355X published figures: 256 CUs, 2.4 GHz; 64 VALU lanes per CU per clock.
N_CU, CLOCK_HZ, LANES_PER_CU = 256, 2.4e9, 64
VALU_LANE_OPS_PEAK = N_CU * LANES_PER_CU * CLOCK_HZ          # 3.93e13 lane-ops/s
FP32_PEAK_FLOPS = 157.3e12                                   # packed FP32 vector
FP64_PEAK_FLOPS = 78.6e12


def algorithmic_work(w):
    """(VALU lane-ops, FP32/FP64 flops) the method needs per path-step.

    Counted from Algorithms 1-4 in their cheapest direct form, one op per add,
    multiply, FMA, compare, select, conversion or transcendental; flops count an
    FMA as 2 and a transcendental as 1.  Philox4x32-10 = 10 rounds x (2 wide
    products + 2 three-way xors) = 40 ops, amortised over 16 steps (Algorithm 2)
    or 2 kicks / 4 flips (Algorithms 3 / 4).
    """
    from paper_1409_4923_amd import workloads as W
    ops = flops = 0.0
    inertial = w.dyn == W.INERTIAL
    # drift evaluations (3 per step): potential force + drive + friction
    if w.pot == W.POT_SIN:
        per_eval_ops, per_eval_flops = 2, 3            # cos, fma(-2 pi, c, A')
    elif w.pot == W.POT_RATCHET:
        per_eval_ops, per_eval_flops = 4, 5            # cos, add, mul, fma
    elif w.pot == W.POT_TENT:
        per_eval_ops, per_eval_flops = 4, 2            # mul, floor, fma, cmp/select
    else:
        per_eval_ops, per_eval_flops = 0, 0
    if inertial:
        per_eval_ops += 1                             # fma(-gamma, v, f)
        per_eval_flops += 2
    ops += 3 * per_eval_ops
    flops += 3 * per_eval_flops
    # constant-within-step forcing A' = A(t) + level - bias at t_n and t_{n+1}
    if w.noise & (W.POISSON | W.DICH):
        ops += 2
        flops += 2
    # predictor / corrector updates
    if inertial:
        ops += 14                                     # 6 fma + 8 add
        flops += 20
    else:
        ops += 9                                      # 3 fma + 6 add
        flops += 12
    # fold: floor, sub, convert, integer add
    ops += 4
    flops += 2
    if w.noise & W.GAUSS:
        ops += 5 + 40.0 / 16.0                        # 2 compares, 2 selects, digit shift
    p_kick = -math.expm1(-w.lam * w.step()) if (w.noise & W.POISSON) else 0.0
    if w.noise & W.POISSON:
        ops += 2 + p_kick * (40.0 / 2.0 + 10.0)       # countdown; kick: draws, 2 logs, floor
    if w.noise & W.DICH:
        p_flip = max(-math.expm1(-w.mua * w.step()), -math.expm1(-w.mub * w.step()))
        ops += 3 + p_flip * (40.0 / 4.0 + 6.0)        # countdown + level select; flip draw
    return ops, flops


def oracle_baseline(w, seconds: float, threads: int):
    """Time the FP64 oracle on paths 0..S-1 of the workload (full horizon), S sized
    from a short pilot so that the run takes about `seconds`."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import to_oracle
    oracle.build(force=False)
    P = to_oracle(w)
    pilot_paths, pilot_steps = 4 * threads, min(2000, w.n_steps)
    t = time.perf_counter()
    oracle.run(P, 0, pilot_paths, pilot_steps, threads=threads)
    rate = pilot_paths * pilot_steps / (time.perf_counter() - t)
    S = int(rate * seconds / w.n_steps) // threads * threads
    S = max(threads, min(S, 4096, w.n_paths))
    t = time.perf_counter()
    st = oracle.run(P, 0, S, w.n_steps, threads=threads)
    el = time.perf_counter() - t
    s = oracle.stats(oracle.velocity(P, st, w.n_steps))
    return dict(value=S * w.n_steps / el, unit="path-steps/s", cores=threads, kind="oracle",
                sample="paths 0..%d of the workload over its full %d-step horizon (%.3g path-steps, %.1f s)"
                       % (S - 1, w.n_steps, S * w.n_steps, el),
                mean_v=s.mean, se=s.se, n_paths=S)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--ppl", type=int, default=0, help="paths per lane (0: library default)")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(paths and parameter points shard trivially; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1409_4923_amd import bmotor as B
    from paper_1409_4923_amd import workloads as W

    w = {"c1": W.C1, "c2": W.C2, "c3": W.C3}[args.config]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    m, r = W.to_c(w)
    ws_bytes = B.bm_ensemble_workspace_size(m, r)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    out = torch.empty(B.STATS_BYTES, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    tune = B.make_tune(args.ppl, args.block) if args.ppl else None

    kernel_ms = []

    def one_step(timed: bool):
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
        finally:
            B.bm_ensemble_destroy(h)
        if timed:
            kernel_ms.append((e0, e1))

    for i in range(args.warmup):
        one_step(False)
        print("warmup step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print("timed %d steps in %.3f s" % (args.steps, t1 - t0), file=sys.stderr, flush=True)

    st = B.stats_from_bytes(out.cpu().numpy().tobytes())
    int_s = sum(a.elapsed_time(b) for a, b in kernel_ms) / 1e3 / args.steps
    launches = 2 if 0 < w.n_window < w.n_steps else 1
    ps_per_step = w.path_steps()
    value = ps_per_step * args.steps / (t1 - t0)
    ops, flops = algorithmic_work(w)
    achieved = ops * ps_per_step / int_s
    peak_flops = FP32_PEAK_FLOPS if w.prec == W.F32 else FP64_PEAK_FLOPS
    rec = {
        "metric": "path-steps/s",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * (t1 - t0) / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.prec == W.F32 else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_paths": w.n_paths, "n_steps": w.n_steps,
                   "n_window": w.n_window, "dt": w.step(), "noise_mask": w.noise,
                   "parallelism": "single-gpu", "paths_per_lane": args.ppl or 1, "block": args.block},
        "mean_v": st.mean, "se_v": st.se, "n_nonfinite": st.n_nonfinite,
        "roofline": {
            "bound": "alu",
            "kernel": "k_advance (integration loop)",
            "achieved": achieved / 1e12,
            "peak": VALU_LANE_OPS_PEAK / 1e12,
            "unit": "TOP/s (VALU lane-ops)",
            "frac": achieved / VALU_LANE_OPS_PEAK,
            "traffic": None,
            "ops_per_path_step": ops,
            "kernel_ms_per_launch": int_s * 1e3 / launches,
            "launches_per_step": launches,
            "fp32_flops": {"achieved_tflops": flops * ps_per_step / int_s / 1e12,
                           "peak_tflops": peak_flops / 1e12,
                           "frac": flops * ps_per_step / int_s / peak_flops},
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        cb = oracle_baseline(w, args.cpu_seconds, threads)
        rec["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        rec["oracle_mean_v"] = cb["mean_v"]
        rec["oracle_se_v"] = cb["se"]
        rec["mean_v_within_3se"] = abs(st.mean - cb["mean_v"]) <= 3 * math.hypot(st.se, cb["se"])
        rec["speedup_vs_oracle"] = value / cb["value"]
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
