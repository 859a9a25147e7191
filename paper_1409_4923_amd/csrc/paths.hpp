// paths.hpp -- the per-path Monte Carlo step (Algorithms 1-4) as device code.
//
// One lane owns PPL paths; the whole path state lives in registers between the
// load at kernel entry and the store at exit (Sec. 4, Memory optimization).
// Instantiated per (precision, dynamics, potential, noise mask, paths per lane)
// so that each kernel contains only the arithmetic of its model.
#pragma once

#include "common.hpp"

namespace bm {

enum : int { DYN_OVERDAMPED = 0, DYN_INERTIAL = 1 };
enum : int { POT_SIN = 0, POT_RATCHET = 1, POT_TENT = 2, POT_FREE = 3 };
enum : int { NZ_GAUSS = 1, NZ_POISSON = 2, NZ_DICH = 4 };

template <typename R> struct Path {
    R x;           // folded position
    int32_t w;     // folded periods
    R v;           // velocity
    int32_t sP;    // Poisson countdown
    uint32_t kP;   // Poisson kicks so far
    int32_t sD;    // dichotomous countdown
    uint32_t mD;   // dichotomous flips so far
    int32_t d;     // dichotomous state
};

// ---------------------------------------------------------------------------
// -V'(x)
// ---------------------------------------------------------------------------
template <int POT> __device__ __forceinline__ float force(float x)
{
    if constexpr (POT == POT_SIN) {
        // V = sin(2 pi x): -V' = -2 pi cos(2 pi x); v_cos_f32 takes its argument in turns
        return -6.28318530717958648f * __builtin_amdgcn_cosf(x);
    } else if constexpr (POT == POT_RATCHET) {
        // V = -sin 2 pi x - sin(4 pi x)/4: -V' = 2 pi c + pi (2 c^2 - 1), c = cos 2 pi x
        const float c = __builtin_amdgcn_cosf(x);
        return 6.28318530717958648f * c + 3.14159265358979324f * (2.0f * c * c - 1.0f);
    } else if constexpr (POT == POT_TENT) {
        // eq. (2), period 2: +1 on [0, 1] (V = 1 - x), -1 on (1, 2) (V = 1 + x shifted)
        const float y = x - 2.0f * floorf(x * 0.5f);
        return y <= 1.0f ? 1.0f : -1.0f;
    } else {
        return 0.0f;
    }
}

template <int POT> __device__ __forceinline__ double force(double x)
{
    constexpr double PI = 3.14159265358979323846;
    if constexpr (POT == POT_SIN) {
        return -2.0 * PI * cos(2.0 * PI * x);
    } else if constexpr (POT == POT_RATCHET) {
        return 2.0 * PI * cos(2.0 * PI * x) + PI * cos(4.0 * PI * x);
    } else if constexpr (POT == POT_TENT) {
        const double y = x - 2.0 * floor(x / 2.0);
        return y <= 1.0 ? 1.0 : -1.0;
    } else {
        return 0.0;
    }
}

template <int POT> constexpr double period() { return POT == POT_TENT ? 2.0 : 1.0; }

// ---------------------------------------------------------------------------
// Folding of x modulo L (Sec. 4, Instruction optimization).
// ---------------------------------------------------------------------------
template <int POT, typename R> __device__ __forceinline__ void fold(Path<R> &s)
{
    if constexpr (POT == POT_TENT) {
        const R k = floor(s.x / R(2));
        s.x = s.x - k * R(2);
        s.w += (int32_t)k;
    } else {
        const R k = floor(s.x);
        s.x = s.x - k;
        s.w += (int32_t)k;
    }
}

// ---------------------------------------------------------------------------
// Algorithm 3 (white Poissonian noise): countdown on the dt grid; on expiry the
// next waiting time s = floor(E_1 / (lambda dt)) and the amplitude z = zeta E_2.
// Kick number k uses words (2(k%2), 2(k%2)+1) of block k/2.  FP64 decisions.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R poisson_update(const KArgs &a, uint32_t path, Path<R> &s)
{
    R z = R(0);
    if (s.sP <= 0) {
        const U4 q = philox4x32_10(s.kP >> 1, path, a.point, TAG_POISSON, a.key0, a.key1);
        const bool second = (s.kP & 1u) != 0u;
        const uint32_t wa = second ? q.z : q.x;
        const uint32_t wb = second ? q.w : q.y;
        s.sP = (int32_t)floor(expo64(wa) / a.lam_dt);
        z = (R)(a.zeta * expo64(wb));
        s.kP += 1u;
    } else {
        s.sP -= 1;
    }
    return z;
}

// ---------------------------------------------------------------------------
// Algorithm 4 (dichotomous noise): on expiry flip the state and draw the dwell
// with the new state's leaving rate.  Flip m uses word m%4 of block m/4.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void dich_update(const KArgs &a, uint32_t path, Path<R> &s)
{
    if (s.sD <= 0) {
        const U4 q = philox4x32_10(s.mD >> 2, path, a.point, TAG_DICH, a.key0, a.key1);
        s.d = 1 - s.d;
        const double mu_dt = s.d ? a.mub_dt : a.mua_dt;
        s.sD = (int32_t)floor(expo64(pick(q, s.mD & 3u)) / mu_dt);
        s.mD += 1u;
    } else {
        s.sD -= 1;
    }
}

// ---------------------------------------------------------------------------
// Algorithm 1: one predictor-corrector step.  A0 / A1 are the drive + tilt at
// t_n / t_{n+1}; cst is the constant-within-step forcing (dichotomous level
// minus the Poisson bias), part of the drift in all three evaluations; z is the
// Poisson kick, added once in the corrector.
// ---------------------------------------------------------------------------
template <int DYN, int POT, typename R>
__device__ __forceinline__ void pc_step(Path<R> &s, R h, R gam, R dxi, R z, R A0, R A1, R cst)
{
    const R half = R(0.5);
    if constexpr (DYN == DYN_INERTIAL) {
        const R x = s.x, v = s.v;
        const R f1 = -gam * v + ((force<POT>(x) + A0) + cst);
        const R xb = x + v * h;
        const R vb = v + f1 * h + dxi;
        R f2 = -gam * vb + ((force<POT>(xb) + A1) + cst);
        const R xp = x + half * (v + vb) * h;                 // predictor
        const R vpr = v + half * (f1 + f2) * h + dxi;
        f2 = -gam * vpr + ((force<POT>(xp) + A1) + cst);
        s.x = x + half * (v + vpr) * h;                      // corrector
        s.v = v + half * (f1 + f2) * h + dxi + z;
    } else {
        const R x = s.x;
        const R f1 = (force<POT>(x) + A0) + cst;
        const R xb = x + f1 * h + dxi;
        R f2 = (force<POT>(xb) + A1) + cst;
        const R xp = x + half * (f1 + f2) * h + dxi;          // predictor
        f2 = (force<POT>(xp) + A1) + cst;
        s.x = x + half * (f1 + f2) * h + dxi + z;            // corrector
    }
}

} // namespace bm
