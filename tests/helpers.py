"""Test helpers: convert a workload to the oracle's parameters, run both sides."""
from __future__ import annotations

import os
import sys

import numpy as np

import oracle
from paper_1409_4923_amd import workloads as W

ORACLE_THREADS = min(16, os.cpu_count() or 1)


def to_oracle(w: W.Workload) -> "oracle.Params":
    return oracle.Params(dyn=w.dyn, pot=w.pot, noise=w.noise, gamma=w.gamma, a=w.a, omega=w.omega,
                         F=w.F, D=w.D, lam=w.lam, zeta=w.zeta, Fa=w.Fa, Fb=w.Fb, mua=w.mua, mub=w.mub,
                         dt=(0.0 if w.spp > 0 else w.dt), spp=w.spp, n_window=w.n_window, seed=w.seed,
                         point=w.point, x0_lo=w.x0_lo, x0_hi=w.x0_hi, v0_lo=w.v0_lo, v0_hi=w.v0_hi,
                         step_tol=w.step_tol, max_halvings=w.max_halvings)


def oracle_paths(w: W.Workload, first: int, count: int, n_steps: int):
    """(unwrapped x, v, noise[count,5], state) of paths [first, first+count) after n_steps."""
    P = to_oracle(w)
    st = oracle.run(P, first, count, n_steps, threads=ORACLE_THREADS, n_paths=w.n_paths)
    xu = oracle.unwrapped(P, st)
    noise = np.stack([st["sP"], st["kP"].astype(np.int64), st["sD"], st["mD"].astype(np.int64),
                      st["d"].astype(np.int64)], axis=1)
    if not (w.noise & W.POISSON):
        noise[:, 0:2] = 0
    if not (w.noise & W.DICH):
        noise[:, 2:5] = 0
    return xu, st["v"].copy(), noise, st


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
