"""Surrogate pipeline: labels from batched Monte Carlo scans, ensemble training,
and queries answered by the surrogate or, where the members disagree, by Monte
Carlo.  Orchestration only: every computation runs in libbmotor (bm_scan,
bm_mlp_backward, bm_mlp_adam_step, bm_surrogate_query).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import bmotor as B
from . import workloads as W

SPP = 200      # steps per drive period of the inertial model


def point_workloads(x: np.ndarray, n_paths, periods: int, seed: int = 0, first_point: int = 0):
    """Inertial-model workloads (Gaussian noise, FP32 paths) for rows x = (a, omega, F, D, gamma);
    n_paths is one count for every row or one per row."""
    out = []
    n_steps = periods * SPP
    counts = np.broadcast_to(np.asarray(n_paths, dtype=np.int64), (len(x),))
    for i, r in enumerate(np.asarray(x, dtype=np.float64)):
        out.append(W.Workload(name="q%d" % i, dyn=W.INERTIAL, pot=W.POT_SIN, noise=W.GAUSS, prec=W.F32,
                              a=float(r[0]), omega=float(r[1]), F=float(r[2]), D=float(r[3]),
                              gamma=float(r[4]), spp=SPP, n_paths=int(counts[i]), n_steps=n_steps,
                              n_window=n_steps // 2, seed=seed, point=first_point + i, x0_lo=0.0, x0_hi=1.0,
                              v0_lo=-2.0, v0_hi=2.0))
    return out


def point_records(x: np.ndarray, n_paths, periods: int, seed: int = 0, first_point: int = 0):
    """The records of point_workloads built column-wise: (numpy models, numpy runs,
    ctypes models, ctypes runs) over the same memory, for a scan over many points."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    mo, ru, M, R = B.record_arrays(n)
    n_steps = periods * SPP
    mo["dyn"], mo["pot"], mo["noise"] = W.INERTIAL, W.POT_SIN, W.GAUSS
    mo["drive_amp"], mo["drive_omega"], mo["force"], mo["D"], mo["gamma"] = x[:, 0], x[:, 1], x[:, 2], x[:, 3], x[:, 4]
    mo["shot_mean"] = 0.0
    ru["prec"], ru["steps_per_period"] = W.F32, SPP
    ru["point_id"] = first_point + np.arange(n, dtype=np.uint64)
    ru["n_steps"], ru["window_start"] = n_steps, n_steps // 2
    ru["n_paths"] = np.broadcast_to(np.asarray(n_paths, dtype=np.int64), (n,))
    ru["seed"] = seed
    ru["x0_lo"], ru["x0_hi"], ru["v0_lo"], ru["v0_hi"] = 0.0, 1.0, -2.0, 2.0
    return mo, ru, M, R


@dataclass
class MCResult:
    mean: np.ndarray
    se: np.ndarray
    std: np.ndarray
    seconds: float
    path_steps: int
    n_paths: np.ndarray | None = None


def pool(n1, m1, s1, n2, m2, s2):
    """Count, mean and sample standard deviation of two samples taken together, from
    each one's count, mean and sample standard deviation (arrays, elementwise)."""
    n1, n2 = np.asarray(n1, dtype=np.float64), np.asarray(n2, dtype=np.float64)
    n = n1 + n2
    mean = (n1 * m1 + n2 * m2) / n
    ss = (n1 - 1.0) * np.square(s1) + (n2 - 1.0) * np.square(s2) + n1 * n2 / n * np.square(m1 - m2)
    return n, mean, np.sqrt(ss / (n - 1.0))


def monte_carlo(x: np.ndarray, n_paths, periods: int, seed: int = 0, first_point: int = 0,
                tune=None) -> MCResult:
    """<v> of every row by one batched scan (plan + one graph launch); n_paths is one
    count for every row or one per row.  Seconds run from building the records to the
    statistics on the host."""
    import torch
    t0 = time.perf_counter()
    _, ru, M, R = point_records(x, n_paths, periods, seed, first_point)
    sc = B.Scan(M, R, tune=tune)
    sc.launch()
    st = sc.stats_records()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sc.close()
    mean = st["mean"].astype(np.float64)
    se = st["se"].astype(np.float64)
    std = np.where(st["n"] > 1, np.sqrt(np.maximum(st["var"], 0.0)), np.nan)
    counts = ru["n_paths"].astype(np.int64)
    return MCResult(mean, se, std, el, int(np.sum(counts)) * periods * SPP, counts)


def adaptive_monte_carlo(x: np.ndarray, tol: float, periods: int, pilot: int = 64, max_paths: int = 1 << 16,
                         rounds: int = 4, seed: int = 0, first_point: int = 0, tune=None) -> MCResult:
    """<v> of every row at 3 SE <= tol by sequential sampling: a pilot scan of `pilot`
    paths per row, then up to rounds - 1 top-up scans.  Before each top-up, row i's
    spread s_i (of all its paths so far) sets its total N_i = ceil((3 s_i / tol)^2),
    at most max_paths (a row without a finite spread takes max_paths); rows short of
    N_i run the difference on streams of their own (seed + round, so the call uses
    seeds seed .. seed + rounds - 1 at these point ids), and the samples are pooled.
    Seconds and path-steps count every scan."""
    x = np.asarray(x)
    res = monte_carlo(x, pilot, periods, seed, first_point, tune)
    n = res.n_paths.astype(np.float64)
    mean, std = res.mean.copy(), res.std.copy()
    seconds, path_steps = res.seconds, res.path_steps
    for rd in range(1, rounds):
        sd = np.where(np.isfinite(std), std, np.inf)
        need = np.ceil(np.square(3.0 * sd / tol))
        need = np.minimum(np.nan_to_num(need, nan=float(max_paths), posinf=float(max_paths)), max_paths)
        more = np.nonzero(need > n)[0]
        if not len(more):
            break
        top = monte_carlo(x[more], (need[more] - n[more]).astype(np.int64), periods, seed + rd, first_point, tune)
        n2, m2, s2 = pool(n[more], mean[more], std[more], top.n_paths, top.mean, top.std)
        n[more], mean[more], std[more] = n2, m2, s2
        seconds += top.seconds
        path_steps += top.path_steps
    se = std / np.sqrt(n)
    return MCResult(mean, se, std, seconds, path_steps, n.astype(np.int64))


def train(sur: "B.Surrogate", x: np.ndarray, y: np.ndarray, epochs: int, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0, lr_final: float = 1e-4):
    """Minibatch Adam on the mean squared error; member m trains on its own bootstrap
    sample of the rows (n rows drawn with replacement), visited in a fresh order every
    epoch.  One permutation of the positions per epoch serves all members: member m's
    rows at those positions are independent of the other members' because the
    bootstrap draws are.  Returns the per-epoch mean member loss."""
    import torch
    rng = np.random.default_rng(seed)
    n = len(x)
    xd = torch.tensor(np.asarray(x, dtype=np.float32), device=sur.device)
    yd = torch.tensor(np.asarray(y, dtype=np.float32), device=sur.device)
    boot = rng.integers(0, n, (sur.n, n)).astype(np.int32)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    last = []
    k = 0
    for ep in range(epochs):
        pos = rng.permutation(n)[:steps_per_epoch * batch]
        # one upload per epoch, laid out [step][member][row] so each step's slice is
        # contiguous; from pinned memory without waiting, so the host prepares the next
        # epoch while the device runs this one (nothing synchronises until the end)
        perm = boot[:, pos].reshape(sur.n, steps_per_epoch, batch).transpose(1, 0, 2)
        perm_d = torch.from_numpy(np.ascontiguousarray(perm)).pin_memory().to(sur.device, non_blocking=True)
        for s in range(steps_per_epoch):
            loss = sur.backward(xd, yd, perm_d[s])
            frac = k / max(1, total - 1)
            sur.adam(lr * (lr_final / lr) ** frac)        # exponential decay to lr_final
            k += 1
        last.append(loss)                                 # the epoch's last step, per member
    return [float(v) for v in torch.stack(last).mean(dim=1).cpu()] if last else []


def uncertain_points(sur: "B.Surrogate", x: np.ndarray, n_pick: int, threshold: float) -> np.ndarray:
    """Rows of candidate points x where the ensemble disagrees most: the n_pick largest
    ensemble spreads among those above `threshold` (fewer if fewer exceed it), for the
    next round of Monte Carlo labels (active learning)."""
    import torch
    xd = torch.tensor(np.asarray(x, dtype=np.float32), device=sur.device)
    _, std, _, _ = sur.query(xd, threshold)
    sd = std.cpu().numpy()
    over = np.nonzero(~(sd <= threshold))[0]
    if len(over) > n_pick:
        over = over[np.argsort(-np.nan_to_num(sd[over], nan=np.inf), kind="stable")[:n_pick]]
    return np.sort(over)


def calibrate_threshold(std: np.ndarray, err: np.ndarray, tol: float, grid, within: float = 0.95):
    """Largest routing threshold t of `grid` (ascending) at which the points the
    ensemble would answer (spread std <= t) keep a 95th-percentile error <= tol and a
    fraction `within` of them within tol, judged on calibration points with known
    errors err = |surrogate - truth|; None if no t qualifies.  Also returns the sweep
    (threshold, answered fraction, p95, fraction within tol) for every t."""
    std, err = np.asarray(std), np.asarray(err)
    best, sweep = None, []
    for t in grid:
        k = std <= t
        p95 = float(np.percentile(err[k], 95)) if k.any() else None
        w = float(np.mean(err[k] <= tol)) if k.any() else None
        sweep.append({"threshold": float(t), "answered": float(k.mean()), "p95": p95, "within_tol": w})
        if p95 is not None and p95 <= tol and w >= within:
            best = float(t)
    return best, sweep


@dataclass
class QueryResult:
    value: np.ndarray          # surrogate mean, replaced by Monte Carlo where routed
    std: np.ndarray            # ensemble spread
    fallback: np.ndarray       # indices answered by Monte Carlo
    t_query: float
    t_fallback: float


def query(sur: "B.Surrogate", x: np.ndarray, threshold: float, n_paths: int | None, periods: int,
          seed: int = 0, mc_first_point: int = 1 << 30, tol: float | None = None) -> QueryResult:
    """Surrogate mean for every row; rows whose ensemble spread exceeds `threshold` are
    answered by Monte Carlo instead: n_paths paths each, or, with tol, the sequential
    budget of adaptive_monte_carlo (3 SE <= tol)."""
    import torch
    xd = torch.tensor(np.asarray(x, dtype=np.float32), device=sur.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mean, std, fidx, fcnt = sur.query(xd, threshold)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_fb = int(fcnt.item())
    fb = fidx[:n_fb].cpu().numpy().astype(np.int64)
    value = mean.cpu().numpy().astype(np.float64)
    t_fb = 0.0
    if n_fb:
        if tol is not None:
            mc = adaptive_monte_carlo(np.asarray(x)[fb], tol, periods, seed=seed, first_point=mc_first_point)
        else:
            mc = monte_carlo(np.asarray(x)[fb], n_paths, periods, seed, mc_first_point)
        value[fb] = mc.mean
        t_fb = mc.seconds
    return QueryResult(value, std.cpu().numpy(), fb, t1 - t0, t_fb)
