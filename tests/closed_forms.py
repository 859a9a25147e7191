"""Closed forms and exact discrete expectations that pin the oracle.

Each function states the mathematics it encodes; none of them calls the oracle.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

TWO32 = 1 << 32


# ---------------------------------------------------------------------------
# Algorithm 2 / eq. (25) with base-6 digits of a 32-bit word.
# ---------------------------------------------------------------------------
def digit_direct(u: int, j: int) -> int:
    """Base-6 digit j (0 = most significant) of the fraction u / 2^32, by big-integer arithmetic."""
    return (u * 6 ** (j + 1) // TWO32) % 6


def digit_counts(j: int) -> list[int]:
    """Exact number of 32-bit words whose base-6 digit j equals 0..5.

    Digits 0..j of u are the base-6 expansion of floor(6^(j+1) u / 2^32); bucket b of that
    integer holds the words ceil(b 2^32 / 6^(j+1)) .. ceil((b+1) 2^32 / 6^(j+1)) - 1.
    """
    m = 6 ** (j + 1)
    counts = [0] * 6
    for b in range(m):
        lo = -(-b * TWO32 // m)
        hi = -(-(b + 1) * TWO32 // m)
        counts[b % 6] += hi - lo
    return counts


# ---------------------------------------------------------------------------
# Algorithm 1 for a linear drift f = -k x (overdamped Ornstein-Uhlenbeck).
# ---------------------------------------------------------------------------
def pc_linear_coeffs(h: float) -> tuple[float, float]:
    """x_{n+1} = R x_n + c dxi_n for the predictor-corrector with f = -k x, h = k dt.

    F1 = -k x;  xb = x(1-h) + dxi;  predictor xb = x(1 - h + h^2/2) + dxi(1 - h/2);
    corrector x' = x(1 - h/2) - (h/2) xb + dxi.
    """
    R = 1.0 - h + h * h / 2.0 - h ** 3 / 4.0
    c = 1.0 - h / 2.0 + h * h / 4.0
    return R, c


def ou_discrete_moments(x0: float, k: float, G: float, dt: float, n: int) -> tuple[float, float]:
    """Mean and variance of x_n under the linear recurrence with iid three-point noise of
    variance G^2 dt."""
    R, c = pc_linear_coeffs(k * dt)
    mean = R ** n * x0
    var = c * c * G * G * dt * (1.0 - R ** (2 * n)) / (1.0 - R * R)
    return mean, var


# ---------------------------------------------------------------------------
# Inertial model with V = 0, no drive: x' = v, v' = -gamma v + noise.
# ---------------------------------------------------------------------------
def inertial_free_recurrence(x0, v0, gamma, dt, dxi):
    """Exact iterates of the predictor-corrector for F(x, v) = (v, -gamma v).

    With g = gamma dt:  v' = v (1 - g + g^2/2 - g^3/4) + dxi (1 - g/2 + g^2/4)
                        x' = x + dt v (1 - g/2 + g^2/4) + (dt/2)(1 - g/2) dxi
    """
    g = gamma * dt
    R = 1.0 - g + g * g / 2.0 - g ** 3 / 4.0
    c = 1.0 - g / 2.0 + g * g / 4.0
    x, v = x0, v0
    for d in dxi:
        x, v = x + dt * v * c + 0.5 * dt * (1.0 - g / 2.0) * d, v * R + c * d
    return x, v


# ---------------------------------------------------------------------------
# Poisson shot noise on the dt grid (Algorithm 3 with floor).
# ---------------------------------------------------------------------------
def kick_probability(lam: float, dt: float) -> float:
    """Pr{kick at a step} = Pr{floor(E/(lam dt)) >= j} ratio = 1 - exp(-lam dt)."""
    return -math.expm1(-lam * dt)


# ---------------------------------------------------------------------------
# Dichotomous noise on the dt grid (Algorithm 4 with floor): a two-state Markov
# chain with leaving probabilities alpha = 1 - exp(-mu_a dt) (state -Fa) and
# beta = 1 - exp(-mu_b dt) (state +Fb).
# ---------------------------------------------------------------------------
def dich_chain(mua, mub, dt):
    alpha = -math.expm1(-mua * dt)
    beta = -math.expm1(-mub * dt)
    return alpha, beta


def dich_mean_level(Fa, Fb, mua, mub, dt, n):
    """E[Gamma_j], j = 0..n-1, starting from the continuous stationary law at step 0."""
    alpha, beta = dich_chain(mua, mub, dt)
    p1_0 = mua / (mua + mub)
    pd = alpha / (alpha + beta)
    lam2 = 1.0 - alpha - beta
    j = np.arange(n, dtype=np.float64)
    p1 = pd + (p1_0 - pd) * lam2 ** j
    return -Fa * (1.0 - p1) + Fb * p1


# ---------------------------------------------------------------------------
# Stationary velocity of the overdamped tilted periodic potential with Gaussian
# white noise (Stratonovich): x' = -U'(x) + F + sqrt(2D) xi.
#   J = D (1 - exp(-F L / D)) / int_0^L dx int_x^{x+L} dy exp((Phi(y) - Phi(x)) / D),
#   Phi = U - F x,  <v> = L J.
# ---------------------------------------------------------------------------
def stratonovich_velocity(U, F: float, D: float, L: float = 1.0, m: int = 8000) -> float:
    """Nodes x_i = i L/m; the inner integral by cumulative trapezoid (O(1/m^2)) and the outer
    one by the periodic trapezoid rule (its integrand exp(-Phi/D) I(x) has period L)."""
    w = L / m
    y = np.arange(2 * m + 1) * w
    phi_y = U(y) - F * y
    shift = np.max(phi_y) / D
    cum = integrate.cumulative_trapezoid(np.exp(phi_y / D - shift), y, initial=0.0)
    i = np.arange(m)
    inner = cum[i + m] - cum[i]                                  # int_{x_i}^{x_i + L}
    total = np.sum(np.exp(-phi_y[i] / D + shift) * inner) * w
    J = D * (-math.expm1(-F * L / D)) / total
    return L * J


def stratonovich_density(U, F: float, D: float, n_bins: int, L: float = 1.0, m: int = 8000) -> np.ndarray:
    """Stationary density of x mod L (eq. 19) for x' = -U'(x) + F + sqrt(2D) xi:
    p(x) proportional to exp(-Phi(x)/D) int_x^{x+L} exp(Phi(y)/D) dy, Phi = U - F x;
    returned as the probability of each of n_bins equal bins of [0, L)."""
    w = L / m
    y = np.arange(2 * m + 1) * w
    phi = U(y) - F * y
    shift = np.max(phi) / D
    cum = integrate.cumulative_trapezoid(np.exp(phi / D - shift), y, initial=0.0)
    i = np.arange(m + 1)
    p = np.exp(-phi[i] / D + shift) * (cum[i + m] - cum[i])
    xs = y[: m + 1]
    edges = np.linspace(0.0, L, n_bins + 1)
    cp = integrate.cumulative_trapezoid(p, xs, initial=0.0)
    cp /= cp[-1]
    return np.diff(np.interp(edges, xs, cp))


# ---------------------------------------------------------------------------
# Eqs. (21)-(23): currents for the symmetric tent potential (L = 2), D_G = 0.
# ---------------------------------------------------------------------------
def poisson_tent_velocity(a: float, DP: float) -> float:
    """eq. (21a)/(22), <v> = L J_I with L = 2; a = lambda zeta, D_P = lambda zeta^2."""
    ap = math.exp(a / (DP * (a - 1.0)))
    am = math.exp(a / (DP * (a + 1.0)))
    J = (1.0 / (4.0 * DP)) * (ap - am) / ((ap - 1.0) * (am - 1.0))
    return 2.0 * J


def dich_tent_velocity_printed(Fa: float, Fb: float, tau: float) -> float:
    """eq. (21b)/(22) exactly as printed, times L = 2 (D_D = Fa Fb tau)."""
    DD = Fa * Fb * tau
    bp = math.exp(1.0 / ((Fa + 1.0) * (Fb - 1.0) * tau))
    bm = math.exp(1.0 / ((Fa - 1.0) * (Fb + 1.0) * tau))
    J = (1.0 / (4.0 * DD)) * (bp - bm) / ((bp - 1.0) * (bm - 1.0))
    return 2.0 * J


def dich_tent_adiabatic(Fa: float, Fb: float) -> float:
    """Slow-switching limit of Model II with the tent potential (|V'| = 1, L = 2):
    in a level f the particle crosses the two half-periods at speeds f+1 and f-1."""
    def vel(f):
        return 2.0 / (1.0 / abs(f + 1.0) + 1.0 / abs(f - 1.0)) * np.sign(f)
    p_b = Fa / (Fa + Fb)             # zero mean: Fa mub = Fb mua -> Pr{+Fb} = Fa/(Fa+Fb)
    return p_b * vel(Fb) + (1.0 - p_b) * vel(-Fa)


# ---------------------------------------------------------------------------
# Deterministic reference trajectories.
# ---------------------------------------------------------------------------
def solve_deterministic(rhs, y0, t_end):
    sol = integrate.solve_ivp(rhs, (0.0, t_end), y0, method="DOP853", rtol=1e-12, atol=1e-13)
    return sol.y[:, -1]
