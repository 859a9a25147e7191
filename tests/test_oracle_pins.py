"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test compares the oracle with something other than itself: an independent
Philox implementation (ATen, numpy), exact counting, closed-form recurrences of
Algorithm 1 for linear drifts, an adaptive ODE solver, the exact law of the
discretised jump processes, the Stratonovich stationary current and eqs. (21)-(23).
"""
from __future__ import annotations

import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats as sps

import closed_forms as cf

TWO_PI = 2.0 * math.pi
THREADS = min(8, os.cpu_count() or 1)


# ---------------------------------------------------------------------------
# Philox
# ---------------------------------------------------------------------------
_ATEN_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (k1 << 32) | k0, sub = (c3 << 32) | c2, off = (c1 << 32) | c0;
    at::philox_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


def _aten_philox(cases):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "p.cpp")
        exe = os.path.join(td, "p")
        open(src, "w").write(_ATEN_SRC)
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-I" + inc, src, "-o", exe])
        inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [[int(t) for t in line.split()] for line in out.strip().splitlines()]


def test_philox4x32_matches_aten(orc):
    rng = np.random.default_rng(1)
    cases = [(0, 0, 0, 0, 0, 0), (2**32 - 1,) * 6, (5, 17, 3, 2, 0, 0)]
    cases += [tuple(int(v) for v in rng.integers(0, 2**32, 6)) for _ in range(200)]
    ref = _aten_philox(cases)
    for c, r in zip(cases, ref):
        assert orc.philox4x32_10(c[:4], c[4:]) == r, c


def test_philox4x64_matches_numpy(orc):
    rng = np.random.default_rng(2)
    m = (1 << 64) - 1
    for i in range(100):
        ctr = [int(v) for v in rng.integers(0, 2**63, 4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        bg = np.random.Philox(counter=ctr, key=key)
        raw = [int(v) for v in bg.random_raw(4)]
        # numpy advances the 256-bit counter by one before producing a block
        nxt = list(ctr)
        nxt[0] = (nxt[0] + 1) & m
        assert orc.philox4x64_10(nxt, key) == raw


# ---------------------------------------------------------------------------
# Algorithm 2 / eq. (25)
# ---------------------------------------------------------------------------
def test_three_point_digit_probabilities_exact():
    """Each digit position gives Pr{-} = Pr{+} = 1/6 within one word in 2^32, and every
    4-digit sequence has probability 6^-4 within 3.1e-7 relative."""
    for j in range(4):
        cnt = cf.digit_counts(j)
        assert sum(cnt) == cf.TWO32
        for c in cnt:
            assert abs(c - cf.TWO32 / 6) <= 6 ** j * 2
    m = 6 ** 4
    sizes = [-(-(b + 1) * cf.TWO32 // m) - -(-b * cf.TWO32 // m) for b in range(m)]
    assert max(abs(s / (cf.TWO32 / m) - 1.0) for s in sizes) < 3.1e-7


def test_three_point_matches_base6_digits(orc):
    rng = np.random.default_rng(3)
    P = orc.Params(seed=0x1234_5678_9ABC, point=7, dt=0.01)
    for _ in range(400):
        path = int(rng.integers(0, 2**20))
        n = int(rng.integers(0, 10**6))
        w = orc.philox4x32_10([n // 16, path, 7, 0], [0x5678_9ABC, 0x1234])
        d = cf.digit_direct(w[(n % 16) // 4], n % 4)
        expect = -1 if d == 0 else (1 if d == 1 else 0)
        assert orc.three_point(P, path, n) == expect


def test_three_point_frequencies(orc):
    P = orc.Params(seed=11, dt=0.01)
    draws = np.array([orc.three_point(P, p, n) for p in range(200) for n in range(100)])
    obs = [np.sum(draws == -1), np.sum(draws == 1), np.sum(draws == 0)]
    chi = sps.chisquare(obs, f_exp=np.array([1 / 6, 1 / 6, 2 / 3]) * len(draws))
    assert chi.pvalue > 1e-4


# ---------------------------------------------------------------------------
# Algorithm 1 with linear drifts: exact recurrences
# ---------------------------------------------------------------------------
def test_free_diffusion_is_sum_of_increments(orc):
    """V = 0: x_n - x_0 = sum of the Algorithm 2 increments, path by path (Delta xi enters once)."""
    P = orc.Params(pot=orc.POT_FREE, noise=orc.GAUSS, D=0.3, dt=0.01)
    g3 = math.sqrt(2 * P.D) * math.sqrt(3 * P.dt)
    st0 = orc.init(P, 0, 32)
    x0 = orc.unwrapped(P, st0)
    st = orc.advance(P, st0.copy(), 0, 0, 200)
    x1 = orc.unwrapped(P, st)
    for p in range(32):
        s = sum(orc.three_point(P, p, n) for n in range(200))
        assert abs((x1[p] - x0[p]) - g3 * s) < 1e-11


def test_free_diffusion_mean_square(orc):
    """<(x_n - x_0)^2> = n G^2 dt = 2 D t exactly for the three-point increments."""
    P = orc.Params(pot=orc.POT_FREE, noise=orc.GAUSS, D=0.25, dt=0.02)
    n, N = 400, 8192
    st0 = orc.init(P, 0, N)
    x0 = orc.unwrapped(P, st0)
    st = orc.advance(P, st0.copy(), 0, 0, n, threads=THREADS)
    d2 = (orc.unwrapped(P, st) - x0) ** 2
    expect = 2 * P.D * n * P.dt
    assert abs(d2.mean() - expect) < 4 * d2.std(ddof=1) / math.sqrt(N)


def test_ou_deterministic_equals_R_power(orc):
    """f = -k x, D = 0: x_n = R^n x_0 with R = 1 - h + h^2/2 - h^3/4."""
    P = orc.Params(pot=orc.POT_HARMONIC, k_harm=2.0, noise=0, dt=0.05, x0_lo=1.0, x0_hi=1.0)
    st = orc.run(P, 0, 1, 100)
    R, _ = cf.pc_linear_coeffs(2.0 * 0.05)
    assert abs(st["x"][0] - R ** 100) < 1e-13


def test_ou_per_path_recurrence(orc):
    P = orc.Params(pot=orc.POT_HARMONIC, k_harm=1.5, noise=orc.GAUSS, D=0.4, dt=0.03,
                   x0_lo=-1.0, x0_hi=1.0)
    R, c = cf.pc_linear_coeffs(1.5 * 0.03)
    g3 = math.sqrt(2 * P.D) * math.sqrt(3 * P.dt)
    st0 = orc.init(P, 0, 16)
    st = orc.advance(P, st0.copy(), 0, 0, 300)
    for p in range(16):
        x = st0["x"][p]
        for n in range(300):
            x = R * x + c * g3 * orc.three_point(P, p, n)
        assert abs(st["x"][p] - x) < 1e-12


def test_ou_weak_order_two(orc):
    """The mean of the OU process, x0 e^{-kt}, is reached with error O(dt^2)."""
    k, T, x0 = 1.0, 2.0, 1.0
    errs = []
    for n in (20, 40, 80):
        P = orc.Params(pot=orc.POT_HARMONIC, k_harm=k, noise=0, dt=T / n, x0_lo=x0, x0_hi=x0)
        st = orc.run(P, 0, 1, n)
        errs.append(abs(st["x"][0] - x0 * math.exp(-k * T)))
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.6 < e1 / e2 < 4.4


def test_ou_stationary_variance(orc):
    """Sample variance of x_n vs the discrete law, and vs the continuum D/k within O(dt^2)."""
    k, D, dt, n, N = 1.0, 0.5, 0.05, 400, 8192
    P = orc.Params(pot=orc.POT_HARMONIC, k_harm=k, noise=orc.GAUSS, D=D, dt=dt,
                   x0_lo=0.0, x0_hi=0.0)
    st = orc.run(P, 0, N, n, threads=THREADS)
    mean, var = cf.ou_discrete_moments(0.0, k, math.sqrt(2 * D), dt, n)
    x = st["x"]
    # Var of the sample variance for a near-Gaussian variable ~ 2 var^2 / N
    assert abs(x.var(ddof=1) - var) < 5 * var * math.sqrt(2.0 / N)
    assert abs(x.mean()) < 5 * math.sqrt(var / N)
    assert abs(var - D / k) / (D / k) < 2e-3


def test_inertial_free_recurrence(orc):
    P = orc.Params(dyn=orc.INERTIAL, pot=orc.POT_FREE, noise=orc.GAUSS, gamma=0.7, D=0.2, dt=0.02,
                   x0_lo=0.0, x0_hi=1.0, v0_lo=-1.0, v0_hi=1.0)
    st0 = orc.init(P, 0, 8)
    st = orc.advance(P, st0.copy(), 0, 0, 250)
    G = math.sqrt(2 * P.gamma * P.D)
    g3 = G * math.sqrt(3 * P.dt)
    xu = orc.unwrapped(P, st)
    for p in range(8):
        dxi = [g3 * orc.three_point(P, p, n) for n in range(250)]
        x, v = cf.inertial_free_recurrence(st0["x"][p], st0["v"][p], P.gamma, P.dt, dxi)
        assert abs(xu[p] - x) < 1e-11
        assert abs(st["v"][p] - v) < 1e-12


# ---------------------------------------------------------------------------
# Deterministic part vs an adaptive ODE solver (drive phase at t_n / t_{n+1})
# ---------------------------------------------------------------------------
def _det_error(orc, P, rhs, y0, T, n):
    st = orc.run(P, 0, 1, n)
    ref = cf.solve_deterministic(rhs, y0, T)
    xu = orc.unwrapped(P, st)[0]
    if P.dyn == orc.INERTIAL:
        return max(abs(xu - ref[0]), abs(st["v"][0] - ref[1]))
    return abs(xu - ref[0])


def test_inertial_deterministic_vs_ode(orc):
    g, a, w, F = 0.9, 4.2, 4.9, 0.1
    T = 2 * TWO_PI / w

    def rhs(t, y):
        return [y[1], -g * y[1] - TWO_PI * math.cos(TWO_PI * y[0]) + a * math.cos(w * t) + F]

    errs = []
    for spp in (100, 200, 400):
        P = orc.Params(dyn=orc.INERTIAL, pot=orc.POT_SIN, noise=0, gamma=g, a=a, omega=w, F=F,
                       spp=spp, x0_lo=0.3, x0_hi=0.3, v0_lo=0.5, v0_hi=0.5)
        errs.append(_det_error(orc, P, rhs, [0.3, 0.5], T, 2 * spp))
    assert errs[-1] < 3e-4
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.3 < e1 / e2 < 4.7


def test_overdamped_ratchet_deterministic_vs_ode(orc):
    a, w, F = 0.8, 3.0, 0.3
    T = 3 * TWO_PI / w

    def rhs(t, y):
        x = y[0]
        return [TWO_PI * math.cos(TWO_PI * x) + math.pi * math.cos(2 * TWO_PI * x) + a * math.cos(w * t) + F]

    errs = []
    for spp in (200, 400, 800):
        P = orc.Params(pot=orc.POT_RATCHET, noise=0, a=a, omega=w, F=F, spp=spp,
                       x0_lo=0.1, x0_hi=0.1)
        errs.append(_det_error(orc, P, rhs, [0.1], T, 3 * spp))
    # the drift here is contracting, so the error is at least second order (often better)
    assert errs[-1] < 1e-5
    for e1, e2 in zip(errs, errs[1:]):
        assert e1 / e2 > 3.3


# ---------------------------------------------------------------------------
# Algorithm 3: white Poissonian noise on the grid
# ---------------------------------------------------------------------------
def test_poisson_first_step_kicks_and_amplitudes(orc):
    lam, zeta, dt, N = 5.0, 0.05, 0.01, 40000
    P = orc.Params(pot=orc.POT_FREE, noise=orc.POISSON, lam=lam, zeta=zeta, dt=dt)
    st0 = orc.init(P, 0, N)
    x0 = orc.unwrapped(P, st0)
    st = orc.advance(P, st0.copy(), 0, 0, 1)
    kicked = st["kP"] == 1
    p = cf.kick_probability(lam, dt)
    assert abs(kicked.mean() - p) < 4 * math.sqrt(p * (1 - p) / N)
    z = orc.unwrapped(P, st)[kicked] - x0[kicked] + lam * zeta * dt
    assert np.all(z > 0)
    assert sps.kstest(z / zeta, "expon").pvalue > 1e-3
    # drift-only paths move by exactly -lambda zeta dt (eq. 26)
    dx = orc.unwrapped(P, st)[~kicked] - x0[~kicked]
    assert np.allclose(dx, -lam * zeta * dt, rtol=0, atol=1e-14)


def test_poisson_mean_displacement_and_counts(orc):
    lam, zeta, dt, n, N = 5.0, 0.05, 0.01, 400, 8192
    P = orc.Params(pot=orc.POT_FREE, noise=orc.POISSON, lam=lam, zeta=zeta, dt=dt)
    st0 = orc.init(P, 0, N)
    x0 = orc.unwrapped(P, st0)
    st = orc.advance(P, st0.copy(), 0, 0, n, threads=THREADS)
    p = cf.kick_probability(lam, dt)
    k = st["kP"].astype(float)
    assert abs(k.mean() - n * p) < 4 * math.sqrt(n * p * (1 - p) / N)
    assert abs(k.var(ddof=1) / (n * p * (1 - p)) - 1) < 0.1
    dx = orc.unwrapped(P, st) - x0
    expect = n * (p * zeta - lam * zeta * dt)          # discrete law
    assert abs(dx.mean() - expect) < 4 * dx.std(ddof=1) / math.sqrt(N)


def test_poisson_intervals_geometric(orc):
    lam, zeta, dt = 20.0, 0.1, 0.01
    P = orc.Params(pot=orc.POT_FREE, noise=orc.POISSON, lam=lam, zeta=zeta, dt=dt)
    st = orc.init(P, 0, 64)
    kicks = []
    prev = st["kP"].copy()
    for n in range(3000):
        orc.advance(P, st, 0, n, n + 1)
        kicks.append(st["kP"] != prev)
        prev = st["kP"].copy()
    K = np.array(kicks)                    # steps x paths
    p = cf.kick_probability(lam, dt)
    gaps = []
    for j in range(K.shape[1]):
        idx = np.nonzero(K[:, j])[0]
        gaps.extend(np.diff(idx).tolist())
    gaps = np.array(gaps)
    # gap g >= 1 has Pr = (1 - p)^(g - 1) p
    assert abs(gaps.mean() - 1 / p) < 4 * math.sqrt((1 - p) / p ** 2 / len(gaps))
    assert abs(np.mean(gaps == 1) - p) < 4 * math.sqrt(p * (1 - p) / len(gaps))


# ---------------------------------------------------------------------------
# Algorithm 4: dichotomous noise on the grid
# ---------------------------------------------------------------------------
def test_dichotomous_levels_chain(orc):
    Fa, Fb, mua, mub, dt = 0.5, 1.0, 1.0, 2.0, 0.02
    P = orc.Params(pot=orc.POT_FREE, noise=orc.DICH, Fa=Fa, Fb=Fb, mua=mua, mub=mub, dt=dt)
    N, n = 4000, 400
    st = orc.init(P, 0, N)
    x0 = orc.unwrapped(P, st)
    lev = np.empty((n, N))
    for j in range(n):
        orc.advance(P, st, 0, j, j + 1)
        lev[j] = np.where(st["d"] == 1, Fb, -Fa)
    # displacement is exactly dt * sum of the levels (constant forcing in the drift, R1)
    assert np.allclose(orc.unwrapped(P, st) - x0, dt * lev.sum(axis=0), rtol=0, atol=1e-11)
    # initial stationary law Pr{+Fb} = mua / (mua + mub)
    p1 = np.mean(lev[0] == Fb)
    assert abs(p1 - mua / (mua + mub)) < 4 * math.sqrt(p1 * (1 - p1) / N)
    # mean level vs the exact two-state chain, averaged over blocks of 50 steps
    m = cf.dich_mean_level(Fa, Fb, mua, mub, dt, n)
    for b in range(0, n, 50):
        blk = lev[b:b + 50].mean(axis=0)
        assert abs(blk.mean() - m[b:b + 50].mean()) < 4.5 * blk.std(ddof=1) / math.sqrt(N)
    # autocorrelation of the centred chain = (1 - alpha - beta)^k -> exp(-(mua + mub) t)
    al, be = cf.dich_chain(mua, mub, dt)
    c = lev[100:] - lev[100:].mean()
    var = np.mean(c * c)
    for lag in (1, 10, 40):
        rho = np.mean(c[lag:] * c[:-lag]) / var
        assert abs(rho - (1 - al - be) ** lag) < 0.03
    # the chain's per-step factor tends to exp(-(mua + mub) dt) with error mua mub dt^2
    assert abs((1 - al - be) - math.exp(-(mua + mub) * dt)) < 1.1 * mua * mub * dt * dt


# ---------------------------------------------------------------------------
# Full <v>: Stratonovich closed form and eqs. (21)-(23)
# ---------------------------------------------------------------------------
def _mc_velocity(orc, P, N, n):
    st = orc.run(P, 0, N, n, threads=THREADS)
    return orc.stats(orc.velocity(P, st, n))


@pytest.mark.slow
@pytest.mark.parametrize("pot,F,D", [("sin", 4.0, 1.0), ("ratchet", 1.0, 0.5)])
def test_stratonovich_tilted_washboard(orc, pot, F, D):
    if pot == "sin":
        U = lambda x: np.sin(TWO_PI * x)
        P = orc.Params(pot=orc.POT_SIN, noise=orc.GAUSS, F=F, D=D, dt=2e-3)
    else:
        U = lambda x: -np.sin(TWO_PI * x) - 0.25 * np.sin(2 * TWO_PI * x)
        P = orc.Params(pot=orc.POT_RATCHET, noise=orc.GAUSS, F=F, D=D, dt=2e-3)
    n = 20000
    P.n_window = n // 10
    s = _mc_velocity(orc, P, 4096, n)
    ref = cf.stratonovich_velocity(U, F, D)
    assert abs(s.mean - ref) < 4 * s.se + 2e-3, (s, ref)


@pytest.mark.slow
@pytest.mark.parametrize("a,DP", [(1.5, 0.5), (2.5, 1.0)])
def test_eq21a_poisson_tent(orc, a, DP):
    lam, zeta = a * a / DP, DP / a                  # a = lambda zeta, D_P = lambda zeta^2
    dt = (1.0 / lam) / 400                          # spp = 400 per 1/lambda, as in Sec. 6
    n = int(150 / lam / dt)
    P = orc.Params(pot=orc.POT_TENT, noise=orc.POISSON, lam=lam, zeta=zeta, dt=dt,
                   x0_lo=0.0, x0_hi=2.0, n_window=n // 10)
    s = _mc_velocity(orc, P, 2048, n)
    ref = cf.poisson_tent_velocity(a, DP)
    # grid snapping lowers the kick rate to (1 - e^{-lam dt})/dt: a bias O(lam dt) in <v>
    assert abs(s.mean - ref) < 4 * s.se + 0.01 * abs(ref), (s, ref)


@pytest.mark.slow
@pytest.mark.parametrize("Fb,tau", [(1.6, 1.0), (1.1, 0.5)])
def test_eq21b_dichotomous_tent_sign(orc, Fb, tau):
    """Model II velocities have the magnitude of eq. (21b) but the opposite sign (the
    dynamics of eqs. 12-14 with levels -Fa / +Fb drift towards -Fa)."""
    Fa = 3.0
    mua = Fa / (tau * (Fa + Fb))                     # 1/tau = mua + mub, Fa mub = Fb mua
    mub = Fb / (tau * (Fa + Fb))
    tmin = min(1 / mua, 1 / mub)
    dt = tmin / 200                                  # spp = 200 per shorter waiting time
    n = int(150 * tmin / dt)
    P = orc.Params(pot=orc.POT_TENT, noise=orc.DICH, Fa=Fa, Fb=Fb, mua=mua, mub=mub, dt=dt,
                   x0_lo=0.0, x0_hi=2.0, n_window=n // 10)
    s = _mc_velocity(orc, P, 2048, n)
    printed = cf.dich_tent_velocity_printed(Fa, Fb, tau)
    assert printed > 0 and s.mean < 0
    assert abs(s.mean + printed) < 4 * s.se + 0.02 * abs(printed), (s, printed)


def test_adiabatic_limit_sign(orc):
    """Slow switching: <v> tends to the adiabatic average, negative for Fa=3, Fb=1.6."""
    Fa, Fb, tau = 3.0, 1.6, 50.0
    mua, mub = Fa / (tau * (Fa + Fb)), Fb / (tau * (Fa + Fb))
    dt = 0.01
    n = 60000
    P = orc.Params(pot=orc.POT_TENT, noise=orc.DICH, Fa=Fa, Fb=Fb, mua=mua, mub=mub, dt=dt,
                   x0_lo=0.0, x0_hi=2.0, n_window=0)
    s = _mc_velocity(orc, P, 1024, n)
    ref = cf.dich_tent_adiabatic(Fa, Fb)
    assert ref < 0
    assert abs(s.mean - ref) < 4 * s.se + 0.05 * abs(ref), (s, ref)


# ---------------------------------------------------------------------------
# Invariants of the discrete algorithm
# ---------------------------------------------------------------------------
def _c2_like(orc, **kw):
    base = dict(dyn=orc.INERTIAL, pot=orc.POT_SIN, noise=orc.GAUSS | orc.POISSON, gamma=0.9,
                a=4.2, omega=4.9, F=0.1, D=1e-4, lam=5.0, zeta=0.05, spp=400, n_window=500,
                x0_lo=0.0, x0_hi=1.0, v0_lo=-2.0, v0_hi=2.0, seed=3)
    base.update(kw)
    return orc.Params(**base)


def test_chunked_equals_whole(orc):
    P = _c2_like(orc)
    a = orc.run(P, 100, 64, 1000)
    b = orc.init(P, 100, 64)
    orc.advance(P, b, 100, 0, 377)
    orc.advance(P, b, 100, 377, 1000)
    assert a.tobytes() == b.tobytes()


def test_path_subset_independent(orc):
    """Counter-based streams: a path's trajectory does not depend on which paths run with it."""
    P = _c2_like(orc, noise=orc.GAUSS | orc.POISSON | orc.DICH, Fa=0.5, Fb=1.0, mua=1.0, mub=2.0)
    a = orc.run(P, 0, 32, 600)
    b = orc.run(P, 10, 5, 600)
    assert a[10:15].tobytes() == b.tobytes()


def test_window_velocity(orc):
    P = _c2_like(orc)
    st = orc.init(P, 0, 16)
    orc.advance(P, st, 0, 0, 500)
    xi = orc.unwrapped(P, st)
    orc.advance(P, st, 0, 500, 1300)
    xf = orc.unwrapped(P, st)
    vp = orc.velocity(P, st, 1300)
    assert np.allclose(vp, (xf - xi) / (800 * P.step()), rtol=1e-12, atol=0)


def test_fold_is_exact_for_unit_period(orc):
    P = _c2_like(orc, noise=orc.GAUSS, D=1e-3)
    st = orc.run(P, 0, 64, 2000)
    assert np.all((st["x"] >= 0) & (st["x"] < 1))
    # the harmonic test potential is never folded: compare the folded free particle
    Q = orc.Params(pot=orc.POT_FREE, noise=orc.GAUSS, D=2.0, dt=0.01)
    R = orc.Params(pot=orc.POT_HARMONIC, k_harm=0.0, noise=orc.GAUSS, D=2.0, dt=0.01)
    a = orc.unwrapped(Q, orc.run(Q, 0, 64, 1000))
    b = orc.run(R, 0, 64, 1000)["x"]
    assert np.allclose(a, b, rtol=0, atol=1e-12)


def test_literal_variant(orc):
    """Printed Algorithm 1 (increments only in the corrector) equals the drift reading when
    V'' = 0, and differs from it at first order in dt otherwise."""
    kw = dict(noise=orc.POISSON | orc.DICH, lam=3.0, zeta=0.2, Fa=0.5, Fb=1.0, mua=1.0, mub=2.0,
              dt=0.01, x0_lo=0.0, x0_hi=1.0)
    A = orc.Params(pot=orc.POT_FREE, **kw)
    B = orc.Params(pot=orc.POT_FREE, literal_alg1=True, **kw)
    xa = orc.unwrapped(A, orc.run(A, 0, 32, 500))
    xb = orc.unwrapped(B, orc.run(B, 0, 32, 500))
    assert np.allclose(xa, xb, rtol=0, atol=1e-12)
    # constant dichotomous level (no flips over the horizon) on the sine potential
    diffs = []
    for dt in (0.02, 0.01, 0.005):
        kw2 = dict(pot=orc.POT_SIN, noise=orc.DICH, Fa=0.5, Fb=1.0, mua=1e-12, mub=1e-12, dt=dt,
                   x0_lo=0.1, x0_hi=0.1)
        n = int(round(1.0 / dt))
        a = orc.unwrapped(orc.Params(**kw2), orc.run(orc.Params(**kw2), 0, 4, n))
        b = orc.unwrapped(orc.Params(literal_alg1=True, **kw2),
                          orc.run(orc.Params(literal_alg1=True, **kw2), 0, 4, n))
        diffs.append(np.max(np.abs(a - b)))
    assert diffs[0] > 1e-4
    for d1, d2 in zip(diffs, diffs[1:]):
        assert 1.6 < d1 / d2 < 2.5


def test_initial_conditions(orc):
    N = 20000
    P = _c2_like(orc, noise=orc.GAUSS | orc.POISSON | orc.DICH, Fa=0.5, Fb=1.0, mua=1.0, mub=2.0)
    st = orc.init(P, 0, N)
    assert sps.kstest(st["x"], "uniform").pvalue > 1e-3
    assert sps.kstest((st["v"] + 2.0) / 4.0, "uniform").pvalue > 1e-3
    p = cf.kick_probability(P.lam, P.step())
    # s0 = floor(E/(lambda dt)) is geometric: Pr{s0 >= j} = (1 - p)^j
    assert abs(np.mean(st["sP"] >= 50) - (1 - p) ** 50) < 4 * math.sqrt(0.25 / N)
    # d is set opposite to the stationary draw; Pr{d* = +Fb} = mua/(mua+mub)
    assert abs(np.mean(st["d"] == 0) - 1 / 3) < 4 * math.sqrt(2 / 9 / N)
    assert np.all(st["sD"] == 0)


@pytest.mark.slow
def test_stationary_density_tilted_washboard(orc):
    """eq. (19): the time-averaged histogram of x mod L approaches the stationary
    density of the tilted washboard, p ~ exp(-Phi/D) int_x^{x+L} exp(Phi/D)."""
    F, D, nb = 2.0, 0.5, 20
    P = orc.Params(pot=orc.POT_SIN, noise=orc.GAUSS, F=F, D=D, dt=2e-3)
    st = orc.init(P, 0, 4096)
    orc.advance(P, st, 0, 0, 2000, threads=THREADS)          # burn-in, t = 4
    counts = np.zeros(nb, dtype=np.int64)
    n = 2000
    for k in range(20):
        orc.advance(P, st, 0, n, n + 250, threads=THREADS)
        n += 250
        counts += orc.density(P, st, nb)
    expect = cf.stratonovich_density(lambda x: np.sin(TWO_PI * x), F, D, nb) * counts.sum()
    # samples 0.5 time units apart are correlated: compare with a generous chi-square
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert chi2 / nb < 4.0, (chi2, counts, expect)
    assert np.max(np.abs(counts / expect - 1)) < 0.05


# ---------------------------------------------------------------------------
# Non-simplified scheme: normal increments
# ---------------------------------------------------------------------------
def test_normal_increments_distribution(orc):
    P = orc.Params(seed=21, dt=0.01)
    z = np.array([orc.normal(P, p, n) for p in range(100) for n in range(200)])
    assert sps.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 4 / math.sqrt(len(z))
    # Box-Muller pairs: steps 2j and 2j+1 share the radius
    r2 = np.array([orc.normal(P, 7, 2 * j) ** 2 + orc.normal(P, 7, 2 * j + 1) ** 2 for j in range(2000)])
    assert sps.kstest(r2 / 2.0, "expon").pvalue > 1e-3      # r^2 / 2 ~ Exp(1)


def test_ou_recurrence_with_normal_increments(orc):
    """Same linear recurrence of Algorithm 1, now with Delta xi = G sqrt(dt) z."""
    P = orc.Params(pot=orc.POT_HARMONIC, k_harm=1.5, noise=orc.NORMAL, D=0.4, dt=0.03,
                   x0_lo=-1.0, x0_hi=1.0)
    R, c = cf.pc_linear_coeffs(1.5 * 0.03)
    g = math.sqrt(2 * P.D) * math.sqrt(P.dt)
    st0 = orc.init(P, 0, 8)
    st = orc.advance(P, st0.copy(), 0, 0, 300)
    for p in range(8):
        x = st0["x"][p]
        for n in range(300):
            x = R * x + c * g * orc.normal(P, p, n)
        assert abs(st["x"][p] - x) < 1e-12


def test_free_diffusion_normal_increments(orc):
    P = orc.Params(pot=orc.POT_FREE, noise=orc.NORMAL, D=0.25, dt=0.02)
    n, N = 200, 8192
    st0 = orc.init(P, 0, N)
    x0 = orc.unwrapped(P, st0)
    st = orc.advance(P, st0.copy(), 0, 0, n, threads=THREADS)
    dx = orc.unwrapped(P, st) - x0
    # a sum of normals is normal with variance 2 D t
    assert sps.kstest(dx / math.sqrt(2 * P.D * n * P.dt), "norm").pvalue > 1e-3


# ---------------------------------------------------------------------------
# Jump-adapted grid: Poisson kicks at their exact times (the step is split)
# ---------------------------------------------------------------------------
def _kick_times(orc, P, path, t_end):
    """Kick times and amplitudes of one path written out from the Philox words
    (first waiting time: word 2 of the tag-2 block; kick k: tag-1 block k/2,
    words 2(k mod 2) (next waiting time) and 2(k mod 2)+1 (amplitude))."""
    key = (P.seed & 0xFFFFFFFF, P.seed >> 32)
    E = lambda w: -math.log(1.0 - w * 2.0 ** -32)
    t = E(orc.philox4x32_10((0, path, P.point, 2), key)[2]) / P.lam
    out = []
    k = 0
    while t < t_end:
        J = orc.philox4x32_10((k // 2, path, P.point, 1), key)
        half = k % 2
        out.append((t, P.zeta * E(J[2 * half + 1])))
        t += E(J[2 * half]) / P.lam
        k += 1
    return out


def test_jump_grid_kicks_at_exact_times(orc):
    """V = 0, no Gaussian noise: x(T) - x0 = sum of the kicks up to T - lambda zeta T,
    whatever the step, path by path."""
    for dt in (0.1, 0.013):
        P = orc.Params(pot=orc.POT_FREE, noise=orc.POISSON | orc.JUMP_GRID, lam=3.0, zeta=0.2, dt=dt,
                       seed=77, x0_lo=0.0, x0_hi=1.0)
        n = int(round(4.0 / dt))
        T = n * dt
        st0 = orc.init(P, 0, 40)
        st = orc.advance(P, st0.copy(), 0, 0, n)
        dx = orc.unwrapped(P, st) - orc.unwrapped(P, st0)
        for p in range(40):
            kicks = _kick_times(orc, P, p, T)
            want = sum(z for _, z in kicks) - P.lam * P.zeta * T
            assert abs(dx[p] - want) < 1e-10
            assert st["kP"][p] == len(kicks)


def test_jump_grid_kick_counts_unbiased_at_coarse_step(orc):
    """lambda dt = 0.5: on the fixed grid the kick rate is (1 - e^{-lambda dt})/dt
    (21% low); on the jump-adapted grid the count over [0, T] is Poisson(lambda T)."""
    lam, dt, n, N = 5.0, 0.1, 100, 20000
    T = n * dt
    for mode, rate in ((orc.POISSON | orc.JUMP_GRID, lam), (orc.POISSON, -math.expm1(-lam * dt) / dt)):
        P = orc.Params(pot=orc.POT_FREE, noise=mode, lam=lam, zeta=0.1, dt=dt, seed=5)
        st = orc.run(P, 0, N, n, threads=THREADS)
        k = st["kP"].astype(np.float64)
        if mode & orc.JUMP_GRID:
            # kicks drawn = kicks at times < T (the next one is pending)
            assert abs(k.mean() - lam * T) < 4 * math.sqrt(lam * T / N)
            assert abs(k.var() / (lam * T) - 1.0) < 0.05
        else:
            assert abs(k.mean() - rate * T) < 4 * math.sqrt(lam * T / N) + 1.0
            assert k.mean() < 0.85 * lam * T


def _ou_kicked_exact(orc, P, p, x0, T):
    """dx = -k x dt + dN_z - lambda zeta dt, solved exactly between and across kicks."""
    k = P.k_harm
    x = x0 * math.exp(-k * T) - P.lam * P.zeta * (1.0 - math.exp(-k * T)) / k
    for t, z in _kick_times(orc, P, p, T):
        x += z * math.exp(-k * (T - t))
    return x


def test_jump_grid_second_order_with_kicks(orc):
    """Linear drift with kicks and no Gaussian noise: on the jump-adapted grid the
    global error against the exact solution falls 4x when dt halves; on the fixed
    grid the kicks are moved by up to dt and the error is first order."""
    errs = {}
    for mode in (orc.POISSON | orc.JUMP_GRID, orc.POISSON):
        errs[mode] = []
        for dt in (0.02, 0.01, 0.005):
            P = orc.Params(pot=orc.POT_HARMONIC, k_harm=1.3, noise=mode, lam=2.0, zeta=0.5, dt=dt, seed=9,
                           x0_lo=-1.0, x0_hi=1.0)
            n = int(round(3.0 / dt))
            st0 = orc.init(P, 0, 32)
            st = orc.advance(P, st0.copy(), 0, 0, n)
            e = [abs(st["x"][p] - _ou_kicked_exact(orc, P, p, st0["x"][p], n * dt)) for p in range(32)]
            errs[mode].append(max(e))
    adapted, fixed = errs[orc.POISSON | orc.JUMP_GRID], errs[orc.POISSON]
    assert adapted[0] / adapted[1] > 3.3 and adapted[1] / adapted[2] > 3.3
    assert fixed[1] / fixed[2] < 2.5 and fixed[2] > 10 * adapted[2]


def test_jump_grid_gaussian_pieces_variance(orc):
    """V = 0 with Gaussian noise: every piece of a split step gets its own increment of
    variance G^2 h_piece, so the noise part of x(T) has variance 2 D T exactly."""
    for g in (orc.GAUSS, orc.NORMAL):
        P = orc.Params(pot=orc.POT_FREE, noise=g | orc.POISSON | orc.JUMP_GRID, lam=4.0, zeta=0.0, D=0.3,
                       dt=0.05, seed=13)
        n, N = 60, 20000
        st0 = orc.init(P, 0, N)
        st = orc.advance(P, st0.copy(), 0, 0, n, threads=THREADS)
        dx = orc.unwrapped(P, st) - orc.unwrapped(P, st0)
        var = 2 * P.D * n * P.dt
        assert abs(dx.mean()) < 4 * math.sqrt(var / N)
        assert abs(dx.var() / var - 1.0) < 4 * math.sqrt(2.0 / N) + 0.01


def test_jump_grid_chunked_equals_whole(orc):
    P = _c2_like(orc, noise=orc.GAUSS | orc.POISSON | orc.JUMP_GRID, lam=40.0)
    a = orc.run(P, 100, 64, 1000)
    b = orc.init(P, 100, 64)
    orc.advance(P, b, 100, 0, 377)
    orc.advance(P, b, 100, 377, 1000)
    assert a.tobytes() == b.tobytes()


def _fixed_grid_kick_steps(orc, P, path, n_steps):
    """Steps of the fixed-grid kicks of one path and their amplitudes, written out
    from the Philox words: the countdown starts at floor(E0 / (lambda dt)) and a kick
    at step n (countdown at 0) draws the next countdown from its own words."""
    key = (P.seed & 0xFFFFFFFF, P.seed >> 32)
    E = lambda w: -math.log(1.0 - w * 2.0 ** -32)
    lam_dt = P.lam * P.step()
    n = math.floor(E(orc.philox4x32_10((0, path, P.point, 2), key)[2]) / lam_dt)
    out = []
    k = 0
    while n < n_steps:
        J = orc.philox4x32_10((k // 2, path, P.point, 1), key)
        half = k % 2
        out.append((n, P.zeta * E(J[2 * half + 1])))
        n += 1 + math.floor(E(J[2 * half]) / lam_dt)
        k += 1
    return out


def _harmonic_driven_kicked_exact(P, x0, T, kicks):
    """x' = -k x + a cos(omega t) + F - lambda zeta + sum_i z_i delta(t - t_i), exactly:
    x0 e^{-kT} + c (1 - e^{-kT}) / k + a (k cos wT + w sin wT - k e^{-kT}) / (k^2 + w^2)
    + sum_i z_i e^{-k (T - t_i)}, c = F - lambda zeta."""
    k, w, a = P.k_harm, P.omega, P.a
    c = P.F - P.lam * P.zeta
    e = math.exp(-k * T)
    x = x0 * e + c * (1.0 - e) / k + a * (k * math.cos(w * T) + w * math.sin(w * T) - k * e) / (k * k + w * w)
    for t, z in kicks:
        x += z * math.exp(-k * (T - t))
    return x


def test_jump_grid_drive_inside_split_steps(orc):
    """Linear drift, periodic drive (integer phase, spp > 0) and kicks on the
    jump-adapted grid: a piece that ends at a kick at t_n + theta dt takes the drive at
    that time, a cos(2 pi (n + theta) / spp) + F.  Against the exact solution the
    global error falls about 4x per halving of dt; with the drive taken anywhere else
    inside a split step (a phase error of order one) it would be first order."""
    errs = []
    for spp in (64, 128, 256):
        P = orc.Params(pot=orc.POT_HARMONIC, k_harm=1.1, noise=orc.POISSON | orc.JUMP_GRID, lam=3.0, zeta=0.4,
                       a=2.5, omega=4.0, F=0.3, spp=spp, seed=21, x0_lo=-1.0, x0_hi=1.0)
        n = 3 * spp                                   # three drive periods
        T = n * P.step()
        st0 = orc.init(P, 0, 24)
        st = orc.advance(P, st0.copy(), 0, 0, n)
        e = []
        for p in range(24):
            kicks = _kick_times(orc, P, p, T)
            assert st["kP"][p] == len(kicks)
            e.append(abs(st["x"][p] - _harmonic_driven_kicked_exact(P, st0["x"][p], T, kicks)))
        errs.append(max(e))
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3
    assert errs[2] < 2e-4


def _inertial_free_exact(P, x0, v0, T, kicks):
    """v' = -gamma v + a cos(omega t) + F - lambda zeta + sum_i z_i delta(t - t_i), x' = v,
    exactly (the kicks act on v):
    v(T) = v0 e^{-gT} + a (g cos wT + w sin wT - g e^{-gT}) / (g^2 + w^2) + c (1 - e^{-gT}) / g
           + sum_i z_i e^{-g (T - t_i)},
    x(T) = x0 + v0 (1 - e^{-gT}) / g + a (g sin(wT) / w + (1 - cos wT) - (1 - e^{-gT})) / (g^2 + w^2)
           + c (T - (1 - e^{-gT}) / g) / g + sum_i z_i (1 - e^{-g (T - t_i)}) / g."""
    g, w, a = P.gamma, P.omega, P.a
    c = P.F - P.lam * P.zeta
    e = math.exp(-g * T)
    d2 = g * g + w * w
    v = v0 * e + a * (g * math.cos(w * T) + w * math.sin(w * T) - g * e) / d2 + c * (1.0 - e) / g
    x = (x0 + v0 * (1.0 - e) / g + a * (g * math.sin(w * T) / w + (1.0 - math.cos(w * T)) - (1.0 - e)) / d2
         + c * (T - (1.0 - e) / g) / g)
    for t, z in kicks:
        ek = math.exp(-g * (T - t))
        v += z * ek
        x += z * (1.0 - ek) / g
    return x, v


def test_inertial_kicks_act_on_velocity(orc):
    """Inertial free particle with periodic drive and Poisson kicks, no Gaussian noise.
    The kick of Algorithm 3 jumps v (never x).  Jump-adapted grid: kicks at their exact
    times, x(T) and v(T) converge at second order.  Fixed grid: the kick of step n is
    added at the end of the step, i.e. at t_{n+1}; against the exact solution with the
    kicks at those times the error is second order too."""
    errs = {}
    for mode in (orc.POISSON | orc.JUMP_GRID, orc.POISSON):
        errs[mode] = []
        for spp in (50, 100, 200):
            P = orc.Params(dyn=orc.INERTIAL, pot=orc.POT_FREE, noise=mode, gamma=0.8, lam=2.5, zeta=0.6,
                           a=1.5, omega=3.0, F=0.2, spp=spp, seed=33, x0_lo=0.0, x0_hi=1.0,
                           v0_lo=-1.0, v0_hi=1.0)
            n = 4 * spp
            dt = P.step()
            T = n * dt
            st0 = orc.init(P, 0, 24)
            x0 = orc.unwrapped(P, st0)
            st = orc.advance(P, st0.copy(), 0, 0, n)
            xT = orc.unwrapped(P, st)
            e = []
            for p in range(24):
                if mode & orc.JUMP_GRID:
                    kicks = _kick_times(orc, P, p, T)
                else:
                    kicks = [((m + 1) * dt, z) for m, z in _fixed_grid_kick_steps(orc, P, p, n)]
                assert st["kP"][p] == len(kicks) and len(kicks) > 0
                xe, ve = _inertial_free_exact(P, x0[p], st0["v"][p], T, kicks)
                e.append(max(abs(xT[p] - xe), abs(st["v"][p] - ve)))
            errs[mode].append(max(e))
    for mode, er in errs.items():
        assert er[0] / er[1] > 3.3 and er[1] / er[2] > 3.3, (mode, er)
        assert er[2] < 1e-4, (mode, er)


# ---------------------------------------------------------------------------
# Step-size control on chi = predictor - corrector (the paragraph after
# Algorithm 1): steps dt / 2^j, one controller per group of 64 paths
# ---------------------------------------------------------------------------
def test_step_control_without_halvings_is_the_fixed_step_scheme(orc):
    """max_halvings = 0 leaves only the step dt: every path equals the fixed-step
    scheme bit for bit, for every noise the control supports."""
    import dataclasses
    for noise in (0, orc.GAUSS, orc.GAUSS | orc.POISSON, orc.GAUSS | orc.DICH, orc.POISSON | orc.DICH):
        P = _c2_like(orc, noise=noise, Fa=0.5, Fb=1.0, mua=1.0, mub=2.0, n_window=150)
        a = orc.run(P, 0, 130, 400)
        b = orc.run(dataclasses.replace(P, step_tol=1e-9, max_halvings=0), 0, 130, 400)
        for f in a.dtype.names:
            if f != "kA":
                assert np.array_equal(a[f], b[f]), (noise, f)
        assert (b["kA"] == 400).all() and (b["lev"] == 0).all()


def _pendulum(orc, spp, **kw):
    return orc.Params(dyn=orc.INERTIAL, pot=orc.POT_SIN, noise=0, gamma=0.9, a=4.2, omega=4.9, F=0.1, spp=spp,
                      x0_lo=0.3, x0_hi=0.3, v0_lo=0.5, v0_hi=0.5, **kw)


def test_step_control_deterministic_error_and_step_count(orc):
    """D = 0, the driven inertial pendulum over two drive periods against DOP853.
    chi of a second-order scheme is a local error of order h^3, so holding it below tol
    takes a number of steps growing as tol^(-1/3) (2.15x per decade of tol), and the
    global error falls as tol falls.  A chi of another order (h^2: 3.2x per decade), a
    drive taken at the wrong time inside a sub-step or a sub-step of the wrong length
    breaks one of these."""
    g, a, w, F = 0.9, 4.2, 4.9, 0.1
    T = 2 * TWO_PI / w

    def rhs(t, y):
        return [y[1], -g * y[1] - TWO_PI * math.cos(TWO_PI * y[0]) + a * math.cos(w * t) + F]

    ref = cf.solve_deterministic(rhs, [0.3, 0.5], T)
    steps, errs = [], []
    for tol in (1e-4, 1e-5, 1e-6, 1e-7):
        P = _pendulum(orc, 25, step_tol=tol, max_halvings=8)
        st = orc.run(P, 0, 1, 50)
        assert st["lev"][0] <= 8
        steps.append(int(st["kA"][0]))
        errs.append(max(abs(orc.unwrapped(P, st)[0] - ref[0]), abs(st["v"][0] - ref[1])))
    ratios = [b / a for a, b in zip(steps, steps[1:])]
    assert all(1.8 < r < 2.6 for r in ratios), (steps, ratios)
    assert all(e2 < e1 / 2 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4
    # the fixed step of the same base dt is far worse than the controlled one
    P0 = _pendulum(orc, 25)
    st0 = orc.run(P0, 0, 1, 50)
    e0 = max(abs(orc.unwrapped(P0, st0)[0] - ref[0]), abs(st0["v"][0] - ref[1]))
    assert e0 > 50 * errs[-1]


def test_step_control_overdamped_ratchet_deterministic(orc):
    a, w, F = 0.8, 3.0, 0.3
    T = 3 * TWO_PI / w

    def rhs(t, y):
        x = y[0]
        return [TWO_PI * math.cos(TWO_PI * x) + math.pi * math.cos(2 * TWO_PI * x) + a * math.cos(w * t) + F]

    ref = cf.solve_deterministic(rhs, [0.1], T)
    errs = []
    for tol in (1e-5, 1e-7, 1e-9):
        P = orc.Params(pot=orc.POT_RATCHET, noise=0, a=a, omega=w, F=F, spp=30, x0_lo=0.1, x0_hi=0.1,
                       step_tol=tol, max_halvings=10)
        st = orc.run(P, 0, 1, 90)
        errs.append(abs(orc.unwrapped(P, st)[0] - ref[0]))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6, errs


def test_step_control_ou_moments(orc):
    """Linear drift with Gaussian noise: each sub-step takes its own three-point draw
    of variance G^2 h, so E x(T) and Var x(T) stay within sampling error plus the
    coarsest step's bias of the continuum OU values x0 e^(-kT) and (D/k)(1 - e^(-2kT)).
    Reusing a draw across sub-steps, or scaling a sub-step's draw with dt, would
    multiply the variance."""
    k, D, dt, n = 1.5, 0.4, 0.2, 20
    P = orc.Params(pot=orc.POT_HARMONIC, k_harm=k, noise=orc.GAUSS, D=D, dt=dt, x0_lo=1.0, x0_hi=1.0,
                   step_tol=2e-3, max_halvings=4, seed=17)
    N = 1 << 15
    st = orc.run(P, 0, N, n, threads=THREADS)
    steps_per_dt = st["kA"].mean() / n
    assert 2.0 < steps_per_dt < 16.0                   # the control is active
    x = st["x"]
    T = n * dt
    mean_c, var_c = math.exp(-k * T), D / k * (1.0 - math.exp(-2 * k * T))
    # coarsest step dt: the discrete mean R^n and variance (exact for the fixed step)
    m_coarse, v_coarse = cf.ou_discrete_moments(1.0, k, math.sqrt(2 * D), dt, n)
    se_m, se_v = math.sqrt(var_c / N), var_c * math.sqrt(2.0 / N)
    assert abs(x.mean() - mean_c) <= 4 * se_m + abs(m_coarse - mean_c)
    assert abs(x.var() - var_c) <= 4 * se_v + abs(v_coarse - var_c)
    assert abs(x.var() - var_c) < 0.05 * var_c


def test_step_control_kicks_and_flips_stay_on_the_dt_grid(orc):
    """The jump processes keep their fixed-grid times under step control: an inertial
    free particle with drive and Poisson kicks matches the exact solution with the kick
    of step n at t_{n+1}; an overdamped free particle with dichotomous noise moves by
    exactly dt times the sum of its levels (the sub-steps of a step add up to dt)."""
    errs = []
    for tol in (1e-4, 1e-6):
        P = orc.Params(dyn=orc.INERTIAL, pot=orc.POT_FREE, noise=orc.POISSON, gamma=0.8, lam=2.5, zeta=0.6,
                       a=1.5, omega=3.0, F=0.2, spp=25, seed=33, x0_lo=0.0, x0_hi=1.0, v0_lo=-1.0, v0_hi=1.0,
                       step_tol=tol, max_halvings=8)
        n, dt = 100, P.step()
        st0 = orc.init(P, 0, 64)
        x0 = orc.unwrapped(P, st0)
        st = orc.advance_adaptive(P, st0.copy(), 0, 64, 0, n)
        xT = orc.unwrapped(P, st)
        e = []
        for p in range(64):
            kicks = [((m + 1) * dt, z) for m, z in _fixed_grid_kick_steps(orc, P, p, n)]
            assert st["kP"][p] == len(kicks)
            xe, ve = _inertial_free_exact(P, x0[p], st0["v"][p], n * dt, kicks)
            e.append(max(abs(xT[p] - xe), abs(st["v"][p] - ve)))
        errs.append(max(e))
    assert errs[1] < errs[0] / 5 and errs[1] < 1e-4, errs
    P = orc.Params(pot=orc.POT_FREE, noise=orc.DICH, Fa=0.7, Fb=1.3, mua=3.0, mub=2.0, dt=0.01, seed=3,
                   step_tol=1e-6, max_halvings=3)
    st0 = orc.init(P, 0, 64)
    x0 = orc.unwrapped(P, st0)
    st = orc.advance_adaptive(P, st0.copy(), 0, 64, 0, 300)
    ref = orc.advance(P.__class__(**{**P.__dict__, "step_tol": 0.0, "max_halvings": 0}),
                      orc.init(P, 0, 64), 0, 0, 300)
    assert np.array_equal(st["mD"], ref["mD"]) and np.array_equal(st["d"], ref["d"])
    assert np.allclose(orc.unwrapped(P, st) - x0, orc.unwrapped(P, ref) - x0, rtol=0, atol=1e-12)


def test_step_control_groups_and_chunks(orc):
    """A path depends only on the paths of its group of 64; any split of the horizon
    into calls gives the same bits."""
    P = _c2_like(orc, noise=orc.GAUSS, D=0.01, step_tol=3e-5, max_halvings=5, n_window=100)
    a = orc.run(P, 0, 200, 300, n_paths=200)                 # groups 0-63, 64-127, 128-191, 192-199
    b = orc.run(P, 64, 64, 300, n_paths=200)
    assert a[64:128].tobytes() == b.tobytes()
    c = orc.run(P, 192, 8, 300, n_paths=200)
    assert a[192:].tobytes() == c.tobytes()
    d = orc.init(P, 0, 200)
    orc.advance_adaptive(P, d, 0, 200, 0, 77)
    orc.advance_adaptive(P, d, 0, 200, 77, 300)
    assert a.tobytes() == d.tobytes()
    assert len(set(a["lev"][:64])) == 1 and a["kA"][0] > 300
    with pytest.raises(ValueError):
        orc.advance_adaptive(P, orc.init(P, 10, 64), 10, 200, 0, 5)
