"""TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle.

A plain, slow, obviously-correct CPU implementation of the Monte Carlo
integration of the Brownian-motor Langevin equation (24) with the jump-adapted
simplified weak order 2.0 predictor-corrector scheme (Algorithms 1-4) and the
ensemble estimator of eq. (31).  The arithmetic lives in ``bm_oracle.c`` (FP64,
``-ffp-contract=off``); this module only marshals arguments and computes the
ensemble statistics with exactly rounded sums (``math.fsum``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library and never
imports it.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OVERDAMPED, INERTIAL = 0, 1
POT_SIN, POT_RATCHET, POT_TENT, POT_FREE, POT_HARMONIC = 0, 1, 2, 3, 4
GAUSS, POISSON, DICH, NORMAL, JUMP_GRID = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("dyn", ctypes.c_int32), ("pot", ctypes.c_int32), ("noise", ctypes.c_int32),
        ("literal_alg1", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("a", ctypes.c_double), ("omega", ctypes.c_double),
        ("F", ctypes.c_double), ("k_harm", ctypes.c_double), ("D", ctypes.c_double),
        ("lam", ctypes.c_double), ("zeta", ctypes.c_double),
        ("Fa", ctypes.c_double), ("Fb", ctypes.c_double), ("mua", ctypes.c_double),
        ("mub", ctypes.c_double), ("dt", ctypes.c_double),
        ("spp", ctypes.c_int64), ("n_window", ctypes.c_int64),
        ("seed", ctypes.c_uint64), ("point", ctypes.c_uint32), ("pad", ctypes.c_uint32),
        ("x0_lo", ctypes.c_double), ("x0_hi", ctypes.c_double),
        ("v0_lo", ctypes.c_double), ("v0_hi", ctypes.c_double),
        ("step_tol", ctypes.c_double), ("max_halvings", ctypes.c_int32), ("pad2", ctypes.c_int32),
    ]


PATH_DTYPE = np.dtype([("x", "<f8"), ("w", "<i8"), ("v", "<f8"), ("xi", "<f8"), ("wi", "<i8"),
                       ("sP", "<i8"), ("thP", "<f8"), ("kP", "<u8"), ("sD", "<i8"), ("mD", "<u8"),
                       ("d", "<i4"), ("lev", "<i4"), ("kA", "<u8")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.or_three_point.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_int64]
        L.or_three_point.restype = ctypes.c_int
        L.or_normal.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_int64]
        L.or_normal.restype = ctypes.c_double
        L.or_init.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
        L.or_advance.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        L.or_advance_adaptive.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        L.or_advance_adaptive.restype = ctypes.c_int
        L.or_velocity.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_void_p,
                                  ctypes.c_int64, ctypes.c_void_p]
        L.or_unwrapped.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_void_p,
                                   ctypes.c_void_p]
        L.or_sizeof_path.restype = ctypes.c_uint32
        L.or_sizeof_params.restype = ctypes.c_uint32
        assert L.or_sizeof_path() == PATH_DTYPE.itemsize
        assert L.or_sizeof_params() == ctypes.sizeof(_Params)
        _lib = L
    return _lib


@dataclass
class Params:
    """Model + run description in the paper's notation.

    dyn: OVERDAMPED (eq. 24) or INERTIAL (x'' + gamma x' = ...).
    pot: POT_SIN (V = sin 2 pi x), POT_RATCHET (V = -sin 2 pi x - sin(4 pi x)/4),
         POT_TENT (eq. 2, L = 2), POT_FREE, POT_HARMONIC (V = k x^2 / 2).
    noise: bit mask of GAUSS | POISSON | DICH (NORMAL: Gaussian noise with normal
           increments instead of the three-point ones; JUMP_GRID with POISSON: kicks
           at their exact times, the step split around them).
    Poisson (eqs. 3-6): lam, zeta.  Dichotomous (eqs. 13-14): levels -Fa / +Fb,
    leaving rates mua (of -Fa) and mub (of +Fb).
    spp > 0: dt = (2 pi / omega) / spp unless dt is given; drive phase = n mod spp.
    step_tol > 0: step-size control on chi with steps dt / 2^j, j <= max_halvings, one
    controller per group of 64 consecutive paths (Gaussian noise only).
    """
    dyn: int = OVERDAMPED
    pot: int = POT_SIN
    noise: int = GAUSS
    gamma: float = 1.0
    a: float = 0.0
    omega: float = 1.0
    F: float = 0.0
    k_harm: float = 0.0
    D: float = 0.0
    lam: float = 1.0
    zeta: float = 0.0
    Fa: float = 0.0
    Fb: float = 0.0
    mua: float = 1.0
    mub: float = 1.0
    dt: float = 0.0
    spp: int = 0
    n_window: int = 0
    seed: int = 0
    point: int = 0
    x0_lo: float = 0.0
    x0_hi: float = 1.0
    v0_lo: float = 0.0
    v0_hi: float = 0.0
    literal_alg1: bool = False
    step_tol: float = 0.0
    max_halvings: int = 0

    def period(self) -> float:
        return 2.0 if self.pot == POT_TENT else 1.0

    def step(self) -> float:
        if self.dt > 0:
            return self.dt
        if self.spp <= 0:
            raise ValueError("need dt > 0 or spp > 0")
        return (2.0 * math.pi / self.omega) / self.spp

    def c(self) -> _Params:
        p = _Params()
        p.dyn, p.pot, p.noise, p.literal_alg1 = self.dyn, self.pot, self.noise, int(self.literal_alg1)
        p.gamma, p.a, p.omega, p.F, p.k_harm, p.D = self.gamma, self.a, self.omega, self.F, self.k_harm, self.D
        p.lam, p.zeta, p.Fa, p.Fb, p.mua, p.mub = self.lam, self.zeta, self.Fa, self.Fb, self.mua, self.mub
        p.dt = self.step()
        p.spp, p.n_window, p.seed, p.point = self.spp, self.n_window, self.seed, self.point
        p.x0_lo, p.x0_hi, p.v0_lo, p.v0_hi = self.x0_lo, self.x0_hi, self.v0_lo, self.v0_hi
        p.step_tol, p.max_halvings = self.step_tol, self.max_halvings
        return p


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def philox4x64_10(ctr, key):
    m = (1 << 64) - 1
    c = (ctypes.c_uint64 * 4)(*[int(v) & m for v in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(v) & m for v in key])
    o = (ctypes.c_uint64 * 4)()
    lib().or_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def three_point(params: Params, path: int, n: int) -> int:
    """Sign (-1, +1, 0) of the Algorithm 2 increment of `path` at step n."""
    cp = params.c()
    return int(lib().or_three_point(ctypes.byref(cp), path, n))


def normal(params: Params, path: int, n: int) -> float:
    """Standard normal variate of `path` at step n (non-simplified scheme)."""
    cp = params.c()
    return float(lib().or_normal(ctypes.byref(cp), path, n))


def init(params: Params, first_path: int, count: int) -> np.ndarray:
    st = np.zeros(count, dtype=PATH_DTYPE)
    cp = params.c()
    lib().or_init(ctypes.byref(cp), first_path, count, st.ctypes.data)
    return st


def _split(count: int, threads: int):
    threads = max(1, min(threads, count))
    edges = np.linspace(0, count, threads + 1).astype(np.int64)
    return [(int(edges[i]), int(edges[i + 1])) for i in range(threads) if edges[i + 1] > edges[i]]


def advance(params: Params, st: np.ndarray, first_path: int, n_from: int, n_to: int,
            threads: int = 1) -> np.ndarray:
    """Advance the paths in `st` (paths first_path ..) from step n_from to n_to, in place.

    ``threads`` > 1 splits the paths over host threads (ctypes releases the GIL).
    """
    assert st.dtype == PATH_DTYPE and st.flags.c_contiguous
    cp = params.c()
    L = lib()

    def run(lo, hi):
        L.or_advance(ctypes.byref(cp), first_path + lo, hi - lo, n_from, n_to,
                     st.ctypes.data + lo * PATH_DTYPE.itemsize)

    parts = _split(len(st), threads)
    if len(parts) == 1:
        run(*parts[0])
    else:
        ts = [threading.Thread(target=run, args=pr) for pr in parts]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    return st


def advance_adaptive(params: Params, st: np.ndarray, first_path: int, n_paths: int, n_from: int, n_to: int,
                     threads: int = 1) -> np.ndarray:
    """Step-controlled advance (params.step_tol > 0) of paths first_path .. (whole
    groups of 64 of an ensemble of n_paths) from step n_from to n_to, in place."""
    assert st.dtype == PATH_DTYPE and st.flags.c_contiguous
    cp = params.c()
    L = lib()
    groups = (len(st) + 63) // 64

    def run_groups(g0, g1):
        lo, hi = 64 * g0, min(64 * g1, len(st))
        rc = L.or_advance_adaptive(ctypes.byref(cp), first_path + lo, hi - lo, n_paths, n_from, n_to,
                                   st.ctypes.data + lo * PATH_DTYPE.itemsize)
        if rc != 0:
            raise ValueError("step control needs whole groups of 64 paths starting at a multiple of 64")

    parts = _split(groups, threads)
    if len(parts) == 1:
        run_groups(*parts[0])
    else:
        ts = [threading.Thread(target=run_groups, args=pr) for pr in parts]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    return st


def run(params: Params, first_path: int, count: int, n_steps: int, threads: int = 1,
        n_paths: int | None = None) -> np.ndarray:
    """Paths first_path .. first_path + count - 1 after n_steps steps of dt.  With step
    control, n_paths (default first_path + count) is the ensemble size that closes the
    last group."""
    st = init(params, first_path, count)
    if params.step_tol > 0:
        return advance_adaptive(params, st, first_path, n_paths or first_path + count, 0, n_steps, threads)
    return advance(params, st, first_path, 0, n_steps, threads)


def velocity(params: Params, st: np.ndarray, n_now: int) -> np.ndarray:
    """eq. (31) per path: ((w - w_i) L + (x - x_i)) / ((n_now - n_window) dt)."""
    vp = np.zeros(len(st), dtype=np.float64)
    cp = params.c()
    lib().or_velocity(ctypes.byref(cp), len(st), st.ctypes.data, n_now, vp.ctypes.data)
    return vp


def unwrapped(params: Params, st: np.ndarray) -> np.ndarray:
    xu = np.zeros(len(st), dtype=np.float64)
    cp = params.c()
    lib().or_unwrapped(ctypes.byref(cp), len(st), st.ctypes.data, xu.ctypes.data)
    return xu


@dataclass
class Stats:
    n: int
    n_nonfinite: int
    mean: float
    var: float
    se: float


def stats(vp: np.ndarray) -> Stats:
    """Ensemble mean, unbiased variance and standard error with exactly rounded sums."""
    vp = np.asarray(vp, dtype=np.float64)
    fin = vp[np.isfinite(vp)]
    n = len(fin)
    mean = math.fsum(fin.tolist()) / n if n else float("nan")
    var = math.fsum(((fin - mean) ** 2).tolist()) / (n - 1) if n > 1 else float("nan")
    se = math.sqrt(var / n) if n > 1 else float("nan")
    return Stats(n=n, n_nonfinite=len(vp) - n, mean=mean, var=var, se=se)


def density(params: Params, st: np.ndarray, n_bins: int) -> np.ndarray:
    """eq. (19): counts of the folded positions y = x mod L in n_bins equal bins of [0, L)."""
    L = params.period()
    x = unwrapped(params, st)
    y = x - L * np.floor(x / L)
    t = y * n_bins / L
    ok = np.isfinite(t)
    b = np.minimum(np.floor(t[ok]).astype(np.int64), n_bins - 1)
    return np.bincount(b, minlength=n_bins).astype(np.int64)
