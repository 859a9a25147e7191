"""Seeded synthetic workloads: parameter sets only, no arithmetic of the method.

A ``Workload`` is a neutral description of one Monte Carlo run in the paper's
notation (eq. 24 / inertial form, Algorithms 1-4, eq. 31).  It is converted to
the C structs by ``to_c`` and, in the tests, to the oracle's parameters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

OVERDAMPED, INERTIAL = 0, 1
POT_SIN, POT_RATCHET, POT_TENT, POT_FREE = 0, 1, 2, 3
GAUSS, POISSON, DICH, NORMAL, JUMP_GRID = 1, 2, 4, 8, 16   # NORMAL: normal increments, not eq. (25);
# JUMP_GRID (with POISSON): kicks at their exact times
F64, F32 = 0, 1


@dataclass(frozen=True)
class Workload:
    name: str
    dyn: int
    pot: int
    noise: int
    n_paths: int
    n_steps: int
    n_window: int
    prec: int = F32
    gamma: float = 1.0
    a: float = 0.0
    omega: float = 1.0
    F: float = 0.0
    D: float = 0.0
    lam: float = 1.0
    zeta: float = 0.0
    Fa: float = 0.0
    Fb: float = 0.0
    mua: float = 1.0
    mub: float = 1.0
    spp: int = 0
    dt: float = 0.0
    seed: int = 0
    point: int = 0
    x0_lo: float = 0.0
    x0_hi: float = 1.0
    v0_lo: float = 0.0
    v0_hi: float = 0.0
    step_tol: float = 0.0        # step-size control on chi (0: fixed step)
    max_halvings: int = 0

    def step(self) -> float:
        return (2.0 * math.pi / self.omega) / self.spp if self.spp > 0 else self.dt

    def path_steps(self) -> int:
        return self.n_paths * self.n_steps

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# Inertial Brownian motor, Gaussian noise only, FP64 paths: 1024 paths, 100 drive
# periods of 200 steps, <v> over the last 50 periods.
C1 = Workload(name="inertial-gauss-f64-1024", dyn=INERTIAL, pot=POT_SIN, noise=GAUSS, prec=F64,
              gamma=0.9, a=4.2, omega=4.9, F=0.1, D=0.001, spp=200,
              n_paths=1024, n_steps=20000, n_window=10000, seed=0, x0_lo=0.0, x0_hi=1.0,
              v0_lo=-2.0, v0_hi=2.0)

# Same model plus white Poissonian noise, FP32 paths: 2^20 paths, 10^3 periods of
# 400 steps, window = last half.
C2 = Workload(name="inertial-poisson-f32-2^20", dyn=INERTIAL, pot=POT_SIN, noise=GAUSS | POISSON,
              prec=F32, gamma=0.9, a=4.2, omega=4.9, F=0.1, D=1e-4, lam=5.0, zeta=0.05, spp=400,
              n_paths=1 << 20, n_steps=400_000, n_window=200_000, seed=0, x0_lo=0.0, x0_hi=1.0,
              v0_lo=-2.0, v0_hi=2.0)

# Overdamped ratchet with dichotomous noise, FP32 paths: eta in {+1.0, -0.5} with
# leaving rates 2.0 / 1.0 (paper notation: Fb = 1.0, mu_b = 2.0, Fa = 0.5, mu_a = 1.0),
# D = 0.01, dt = 1e-3, t_end = 10^3, window from t_f / 10.
C3 = Workload(name="overdamped-ratchet-dich-f32-2^20", dyn=OVERDAMPED, pot=POT_RATCHET,
              noise=GAUSS | DICH, prec=F32, D=0.01, Fa=0.5, Fb=1.0, mua=1.0, mub=2.0, dt=1e-3,
              n_paths=1 << 20, n_steps=1_000_000, n_window=100_000, seed=0, x0_lo=0.0, x0_hi=1.0)


def c4_points(n_points: int = 4096, seed: int = 0, gamma_range=None):
    """Batched-scan points of the inertial model (configuration of C1, FP32 paths).

    a ~ U[0,8], omega ~ U[1,10], F ~ U[-0.5,0.5], D log-uniform in [1e-4, 1e-1],
    gamma = 0.9 (or U[gamma_range]); path counts log-uniform in [256, 16384];
    run lengths log-uniform in [10^2, 10^4] periods of 200 steps; window = last half.
    """
    rng = np.random.default_rng(seed)
    u = rng.random((n_points, 6))
    a = 8.0 * u[:, 0]
    omega = 1.0 + 9.0 * u[:, 1]
    F = u[:, 2] - 0.5
    D = 10.0 ** (-4.0 + 3.0 * u[:, 3])
    n_paths = np.rint(256.0 * 64.0 ** u[:, 4]).astype(np.int64)
    periods = np.rint(100.0 * 100.0 ** u[:, 5]).astype(np.int64)
    if gamma_range is None:
        gamma = np.full(n_points, 0.9)
    else:
        gamma = gamma_range[0] + (gamma_range[1] - gamma_range[0]) * rng.random(n_points)
    out = []
    for i in range(n_points):
        n_steps = int(periods[i]) * 200
        out.append(Workload(name="scan-point-%d" % i, dyn=INERTIAL, pot=POT_SIN, noise=GAUSS, prec=F32,
                            gamma=float(gamma[i]), a=float(a[i]), omega=float(omega[i]), F=float(F[i]),
                            D=float(D[i]), spp=200, n_paths=int(n_paths[i]), n_steps=n_steps,
                            n_window=n_steps // 2, seed=0, point=i, x0_lo=0.0, x0_hi=1.0,
                            v0_lo=-2.0, v0_hi=2.0))
    return out


def to_c(w: Workload):
    """(bm_model, bm_run) for a workload."""
    from . import bmotor as B
    m = B.make_model(dyn=w.dyn, pot=w.pot, noise=w.noise, gamma=w.gamma, drive_amp=w.a,
                     drive_omega=w.omega, force=w.F, D=w.D, shot_rate=w.lam, shot_mean=w.zeta,
                     dich_Fa=w.Fa, dich_Fb=w.Fb, dich_mua=w.mua, dich_mub=w.mub)
    r = B.make_run(prec=w.prec, steps_per_period=w.spp, point_id=w.point,
                   dt=(0.0 if w.spp > 0 else w.dt), n_steps=w.n_steps, window_start=w.n_window,
                   n_paths=w.n_paths, seed=w.seed, x0_lo=w.x0_lo, x0_hi=w.x0_hi,
                   v0_lo=w.v0_lo, v0_hi=w.v0_hi, step_tol=w.step_tol, max_halvings=w.max_halvings)
    return m, r


# ---------------------------------------------------------------------------
# Surrogate inputs
# ---------------------------------------------------------------------------
MLP_IN, MLP_H = 5, 256
MLP_NPARAM = MLP_H * MLP_IN + MLP_H + 2 * (MLP_H * MLP_H + MLP_H) + MLP_H + 1   # 133377


def mlp_params(n_members: int, seed: int = 0) -> np.ndarray:
    """Initial parameters [n_members, 133377] (float32): every weight and bias of a layer
    with fan-in f drawn from U(-1/sqrt(f), 1/sqrt(f)), packed W1|b1|W2|b2|W3|b3|W4|b4."""
    rng = np.random.default_rng(seed)
    out = np.empty((n_members, MLP_NPARAM), dtype=np.float32)
    fans = [(MLP_H * MLP_IN, MLP_IN), (MLP_H, MLP_IN), (MLP_H * MLP_H, MLP_H), (MLP_H, MLP_H),
            (MLP_H * MLP_H, MLP_H), (MLP_H, MLP_H), (MLP_H, MLP_H), (1, MLP_H)]
    for m in range(n_members):
        parts = [rng.uniform(-1.0, 1.0, n) / np.sqrt(f) for n, f in fans]
        out[m] = np.concatenate(parts).astype(np.float32)
    return out


def surrogate_queries(n: int, seed: int = 0, gamma_range=(0.5, 2.0)) -> np.ndarray:
    """Query points [n, 5] = (a, omega, F, D, gamma) over the surrogate's domain:
    a ~ U[0,8], omega ~ U[1,10], F ~ U[-0.5,0.5], D log-uniform in [1e-4, 1e-1],
    gamma ~ U[gamma_range] (float32)."""
    rng = np.random.default_rng(seed)
    u = rng.random((n, 5))
    x = np.empty((n, 5))
    x[:, 0] = 8.0 * u[:, 0]
    x[:, 1] = 1.0 + 9.0 * u[:, 1]
    x[:, 2] = u[:, 2] - 0.5
    x[:, 3] = 10.0 ** (-4.0 + 3.0 * u[:, 3])
    x[:, 4] = gamma_range[0] + (gamma_range[1] - gamma_range[0]) * u[:, 4]
    return x.astype(np.float32)
