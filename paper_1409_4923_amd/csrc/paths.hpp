// paths.hpp -- the per-path Monte Carlo step (Algorithms 1-4) as device code.
//
// One lane owns PPL paths; the whole path state lives in registers between the
// load at kernel entry and the store at exit (Sec. 5, Memory optimization).
// Instantiated per (precision, dynamics, potential, noise mask, paths per lane)
// so that each kernel contains only the arithmetic of its model.
#pragma once

#include "common.hpp"

namespace bm {

enum : int { DYN_OVERDAMPED = 0, DYN_INERTIAL = 1 };
enum : int { POT_SIN = 0, POT_RATCHET = 1, POT_TENT = 2, POT_FREE = 3 };
enum : int { NZ_GAUSS = 1, NZ_POISSON = 2, NZ_DICH = 4,
             NZ_NORMAL = 8,     // Gaussian noise with normal increments (non-simplified scheme)
             NZ_JGRID = 16 };   // Poisson kicks at their exact times (jump-adapted grid)

// Poisson kicks pre-drawn per window into the LDS queue (fixed grid only).
template <int NOISE> constexpr bool queued_kicks()
{
    return (NOISE & NZ_POISSON) != 0 && (NOISE & NZ_JGRID) == 0;
}

template <typename R> struct Path {
    R x;           // folded position
    int32_t w;     // folded periods
    R v;           // velocity
    int32_t sP;    // Poisson countdown
    uint32_t kP;   // Poisson kicks so far
    int32_t sD;    // dichotomous countdown
    uint32_t mD;   // dichotomous flips so far
    int32_t d;     // dichotomous state
    double thP;    // jump-adapted grid: fraction of its step at which the next kick falls
};

// ---------------------------------------------------------------------------
// -V'(x) + A, where A is the constant-within-step forcing of the step (drive,
// tilt, Poisson bias, dichotomous level) plus the potential's constant offset
// pot_offset<POT>() (folded into the drive table on the host).
// ---------------------------------------------------------------------------
// The potential's constant factor of the force: -2 pi (sine) or 2 pi (ratchet).
// In FP32 it is held in a vector register the compiler cannot see through: the
// forcing A is wave-uniform and lives in a scalar register, an FMA may read only
// one scalar operand, and with the factor as a literal (a second one) the compiler
// would copy A into a vector register at every use.  Formed once per kernel.
template <int POT, typename R> __device__ __forceinline__ R pot_factor()
{
    constexpr double TWO_PI = 6.28318530717958647692;
    const R c = (R)(POT == POT_SIN ? -TWO_PI : TWO_PI);
    if constexpr (sizeof(R) == 4) {
        R r;
        asm volatile("; pot_factor" : "=v"(r) : "0"(c));
        return r;
    } else {
        return c;
    }
}

// -V'(x) + A, with kp = pot_factor<POT>().
template <int POT> __device__ __forceinline__ float force_plus(float x, float A, float kp)
{
    if constexpr (POT == POT_SIN) {
        // V = sin(2 pi x): -V' = -2 pi cos(2 pi x); v_cos_f32 takes its argument in turns
        return __builtin_fmaf(kp, __builtin_amdgcn_cosf(x), A);
    } else if constexpr (POT == POT_RATCHET) {
        // V = -sin 2 pi x - sin(4 pi x)/4:  -V' = 2 pi c + pi (2 c^2 - 1) = c (2 pi c + 2 pi) - pi
        const float c = __builtin_amdgcn_cosf(x);
        return __builtin_fmaf(c, __builtin_fmaf(kp, c, kp), A);           // A includes -pi
    } else if constexpr (POT == POT_TENT) {
        // eq. (2), period 2: +1 on [0, 1] (V = 1 - x), -1 on (1, 2) (V = 1 + x shifted)
        const float y = x - 2.0f * floorf(x * 0.5f);
        return (y <= 1.0f ? 1.0f : -1.0f) + A;
    } else {
        return A;
    }
}

// cos y in FP64.  Cody-Waite reduction y = k pi/2 + r, k = rint(2y/pi), with pi/2
// split into three doubles (the first two of 33 significant bits, so k times each is
// exact for |k| < 2^20), r in [-pi/4, pi/4]; then the Taylor series of sin r to r^17
// and of cos r to r^16 (remainders below 1e-19 and 3e-18 on that interval), and k
// mod 4 picks cos r, -sin r, -cos r or sin r.  A lane whose argument has |y| >= 2^20
// (or is NaN) takes the library cos instead; the other lanes keep the polynomial, so
// a path's value never depends on the paths that share its wave.
__device__ __noinline__ double cos_library(double y) { return cos(y); }

__device__ __forceinline__ double cos_fp64(double y_in)
{
    const bool big = !(fabs(y_in) < 0x1p20);
    double lib = 0.0;
    if (__builtin_amdgcn_ballot_w64(big) != 0) {
        if (big) lib = cos_library(y_in);
    }
    const double y = big ? 0.0 : y_in;                               // keeps the reduction exact
    const double k = rint(y * 0x1.45f306dc9c883p-1);                 // 2/pi
    double r = fma(-k, 0x1.921fb544p+0, y);                          // pi/2, first 33 bits
    r = fma(-k, 0x1.0b4611a6p-34, r);                                //       next 33 bits
    r = fma(-k, 0x1.3198a2e037073p-69, r);                           //       the rest
    const double r2 = r * r;
    // coefficients (-1)^j / n!, n = 2j + 1 (sin) or 2j (cos), rounded to nearest
    double ps = 0x1.952c77030ad4ap-49;                               //  1/17!
    ps = fma(ps, r2, -0x1.ae7f3e733b81fp-41);                        // -1/15!
    ps = fma(ps, r2, 0x1.6124613a86d09p-33);                         //  1/13!
    ps = fma(ps, r2, -0x1.ae64567f544e4p-26);                        // -1/11!
    ps = fma(ps, r2, 0x1.71de3a556c734p-19);                         //  1/9!
    ps = fma(ps, r2, -0x1.a01a01a01a01ap-13);                        // -1/7!
    ps = fma(ps, r2, 0x1.1111111111111p-7);                          //  1/5!
    ps = fma(ps, r2, -0x1.5555555555555p-3);                         // -1/3!
    const double sn = fma(r * r2, ps, r);
    double pc = 0x1.ae7f3e733b81fp-45;                               //  1/16!
    pc = fma(pc, r2, -0x1.93974a8c07c9dp-37);                        // -1/14!
    pc = fma(pc, r2, 0x1.1eed8eff8d898p-29);                         //  1/12!
    pc = fma(pc, r2, -0x1.27e4fb7789f5cp-22);                        // -1/10!
    pc = fma(pc, r2, 0x1.a01a01a01a01ap-16);                         //  1/8!
    pc = fma(pc, r2, -0x1.6c16c16c16c17p-10);                        // -1/6!
    pc = fma(pc, r2, 0x1.5555555555555p-5);                          //  1/4!
    pc = fma(pc, r2, -0.5);                                          // -1/2!
    const double cs = fma(r2, pc, 1.0);
    const int q = (int)k & 3;                                        // k mod 4 (two's complement)
    const double v = (q & 1) ? sn : cs;
    const double poly = (q == 1 || q == 2) ? -v : v;
    return big ? lib : poly;
}

template <int POT> __device__ __forceinline__ double force_plus(double x, double A, double kp)
{
    constexpr double PI = 3.14159265358979323846;
    if constexpr (POT == POT_SIN) {
        return fma(kp, cos_fp64(2.0 * PI * x), A);
    } else if constexpr (POT == POT_RATCHET) {
        const double c = cos_fp64(2.0 * PI * x);
        return fma(c, fma(kp, c, kp), A);                                 // A includes -pi
    } else if constexpr (POT == POT_TENT) {
        const double y = x - 2.0 * floor(x / 2.0);
        return (y <= 1.0 ? 1.0 : -1.0) + A;
    } else {
        return A;
    }
}

// ---------------------------------------------------------------------------
// Normal increments of the non-simplified scheme: the Box-Muller transform of
// two uniform words, r = sqrt(-2 ln(1 - phi1)), (r cos 2 pi phi2, r sin 2 pi phi2)
// with phi = w 2^-32.  1 - phi1 = (2^32 - w1) 2^-32 is formed from the integer,
// so it is exact before the conversion and never 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void normal_pair(uint32_t w1, uint32_t w2, float &zc, float &zs)
{
    constexpr float NEG_2LN2 = -1.38629436111989061f;            // -2 ln 2
    const float om = w1 ? (float)(0u - w1) * 0x1p-32f : 1.0f;
    const float r = __builtin_amdgcn_sqrtf(NEG_2LN2 * __builtin_amdgcn_logf(om));   // log2, then scale
    const float t = (float)w2 * 0x1p-32f;                        // turns: v_sin/v_cos take 2 pi t
    zc = r * __builtin_amdgcn_cosf(t);
    zs = r * __builtin_amdgcn_sinf(t);
}

__device__ __forceinline__ void normal_pair(uint32_t w1, uint32_t w2, double &zc, double &zs)
{
    constexpr double PI = 3.14159265358979323846;
    const double om = w1 ? (double)(0u - w1) * 0x1p-32 : 1.0;
    const double r = sqrt(-2.0 * log(om));
    const double t = (double)w2 * 0x1p-32;
    zc = r * cos(2.0 * PI * t);
    zs = r * sin(2.0 * PI * t);
}

// Constant part of -V'(x) moved into the drive table.
template <int POT> constexpr double pot_offset()
{
    return POT == POT_RATCHET ? -3.14159265358979323846 : 0.0;
}

template <int POT> constexpr double period() { return POT == POT_TENT ? 2.0 : 1.0; }

// ---------------------------------------------------------------------------
// Folding of x modulo L (Sec. 5, Instruction optimization).
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
// Jump processes on the dt grid.  The times and sizes of the jumps do not depend
// on the path state, so each lane resolves all jumps of a window of steps in
// one wave-uniform loop (the draws are the same as in Algorithms 3 / 4 step by
// step) and queues them in LDS; the step loop then only compares the step
// offset with the next queued offset.  The window (16 2^k steps, at most 1024) is
// chosen per parameter point so that a lane expects about four jumps in it: the
// wave-uniform loop runs as many iterations as the lane with the most jumps, and
// a queue rarely fills up.  On the fixed grid a full queue ends the window early for
// the whole wave (at the first jump it does not hold); on the jump-adapted grid a
// lane with more than JCAP flips in a window queues an "inline" marker and draws
// the rest at their steps.
// ---------------------------------------------------------------------------
constexpr uint32_t JCAP = 11;         // queued jumps per lane and window
constexpr uint32_t INLINE_BIT = 0x80000000u;

// A kick of the jump-adapted grid, drawn ahead: its step offset in the window, the
// fraction of that step at which it falls, its amplitude, and the Gaussian
// increment (times G sqrt(3 dt) or G sqrt(dt)) of the piece that follows it.
template <typename R> struct JGKick {
    uint32_t off;
    R th, z, u;
};
constexpr uint32_t JG_NONE = 0xFFFFFFFFu;
// Queued kicks per lane and window of the jump-adapted grid (more are drawn at their
// steps): 10 in FP32, 6 in FP64, so that the FP64 queues of 256 lanes with the
// dichotomous queue still fit in 64 KiB of LDS.
template <typename R> constexpr uint32_t jg_cap() { return sizeof(R) == 4 ? 10u : 6u; }

template <typename R> struct KickEntry {
    uint32_t off;   // step offset in the window (>= the steps run: none left)
    R z;            // amplitude
};

// Exponential countdown s = floor(E / (rate dt)), E = -ln(1 - phi), phi = w 2^-32,
// decided exactly as in FP64 (the oracle's expression).  FP32 paths first form
// an FP32 estimate X32 with v_log_f32; its error is below
// 3e-7 / (rate dt) + 4.2e-7 X (rounding of 1 - phi, log2 near 1, the scale), and
// the tolerance tol0 + tol1 X is several times that, so floor(X32) is exact
// unless X32 lies within the tolerance of an integer -- then FP64 decides.  The
// FP64 work sits behind a wave-uniform branch taken only when some lane needs it
// (a few per cent of the draws); as a plain per-lane branch the compiler turns it
// into a select and evaluates the FP64 log and divide for every draw.
// The FP64 decision, out of line: inlined, its log and divide would be repeated at
// every draw site of the unrolled step loop although they rarely run.
__device__ __noinline__ uint32_t countdown_fp64(uint32_t w, double rate_dt)
{
    return (uint32_t)floor(expo64(w) / rate_dt);
}

template <typename R>
__device__ __forceinline__ uint32_t countdown(uint32_t w, double rate_dt, float c, float tol0, float tol1)
{
    if constexpr (sizeof(R) == 4) {
        const float one_minus_phi = ((float)(~w) + 1.0f) * 0x1p-32f;   // (2^32 - w) 2^-32
        const float X = -__builtin_amdgcn_logf(one_minus_phi) * c;
        const float fl = floorf(X);
        const float fr = X - fl;
        const float tol = fmaf(tol1, X, tol0);
        const bool sure = fr > tol && fr < 1.0f - tol;
        uint32_t s = (uint32_t)fl;
        if (__builtin_amdgcn_ballot_w64(!sure) != 0) {
            const uint32_t s64 = countdown_fp64(w, rate_dt);
            if (!sure) s = s64;
        }
        return s;
    }
    return countdown_fp64(w, rate_dt);
}

// Kick amplitude z = zeta E (no decision depends on it: FP32 paths use v_log_f32).
template <typename R> __device__ __forceinline__ R amplitude(const PointConst &a, uint32_t w)
{
    if constexpr (sizeof(R) == 4) {
        const float one_minus_phi = ((float)(~w) + 1.0f) * 0x1p-32f;
        return __builtin_amdgcn_logf(one_minus_phi) * a.zeta_ln2;
    } else {
        return a.zeta * expo64(w);
    }
}

// Algorithm 3 draw for kick number k: next waiting time s (steps) and amplitude z.
// Kick k uses words (2(k%2), 2(k%2)+1) of block k/2.
template <typename R>
__device__ __forceinline__ void kick_from(const PointConst &a, uint32_t ws, uint32_t wz, uint32_t &s, R &z)
{
    s = countdown<R>(ws, a.lam_dt, a.c_lam, a.tol0_lam, a.tol1);
    z = amplitude<R>(a, wz);
}

// Algorithm 4 draw for flip number m into state d_new: dwell s (steps).
template <typename R>
__device__ __forceinline__ uint32_t flip_draw(const PointConst &a, uint32_t path, uint32_t m, int32_t d_new)
{
    const U4 q = philox4x32_10(m >> 2, path, a.point, TAG_DICH, a.key0, a.key1);
    const uint32_t w = pick(q, m & 3u);
    return d_new ? countdown<R>(w, a.mub_dt, a.c_mub, a.tol0_mub, a.tol1)
                 : countdown<R>(w, a.mua_dt, a.c_mua, a.tol0_mua, a.tol1);
}

// Queue the kicks of one window.  `off` is the offset of the next kick (the
// Algorithm 3 countdown at the window start).  q[slot * qs] is this lane's queue.
// One Philox block holds two kicks: an iteration uses both halves when it can.
// Returns the number of leading steps of the window whose kicks are all queued:
// wlen, or, when the queue is full, the offset of the first kick it does not hold.
template <typename R>
__device__ __forceinline__ uint32_t kick_window(const PointConst &a, uint32_t path, uint32_t wlen, uint32_t off,
                                                uint32_t &kP, KickEntry<R> *q, uint32_t qs)
{
    uint32_t slot = 0;
    bool active = off < wlen;
    while (__any(active)) {
        if (active) {
            if (slot < JCAP) {
                const U4 b = philox4x32_10(kP >> 1, path, a.point, TAG_POISSON, a.key0, a.key1);
                const bool second = (kP & 1u) != 0u;
                uint32_t sn;
                R z;
                kick_from<R>(a, second ? b.z : b.x, second ? b.w : b.y, sn, z);
                q[slot * qs] = KickEntry<R>{off, z};
                ++slot;
                ++kP;
                off = off + 1u + sn;
                active = off < wlen;
                if (!second && active && slot < JCAP) {      // the block's second kick
                    kick_from<R>(a, b.z, b.w, sn, z);
                    q[slot * qs] = KickEntry<R>{off, z};
                    ++slot;
                    ++kP;
                    off = off + 1u + sn;
                    active = off < wlen;
                }
            } else {
                active = false;      // queue full: the window ends at this kick
            }
        }
    }
    q[slot * qs] = KickEntry<R>{off, R(0)};
    return off < wlen ? off : wlen;
}

// Jumps queued in slots below JCAP at offsets in [from, wlen): drawn for a window
// of wlen steps that ended after `from` steps.  Offsets rise along the queue and
// the entry after the last queued jump lies at or beyond wlen (or at slot JCAP).
template <typename T, typename OffOf>
__device__ __forceinline__ uint32_t queued_beyond(const T *q, uint32_t qs, uint32_t from, uint32_t wlen, OffOf off_of)
{
    uint32_t c = 0;
    for (uint32_t slot = 0; slot < JCAP; ++slot) {
        const uint32_t o = off_of(q[slot * qs]);
        if (o >= wlen) break;
        c += (o >= from) ? 1u : 0u;
    }
    return c;
}

// Queue the flips of one window; bit INLINE_BIT marks "draw inline from here" (only
// the jump-adapted grid runs past it; on the fixed grid a full queue ends the window,
// as for kicks).  Returns the number of leading steps whose flips are all queued.
template <typename R>
__device__ __forceinline__ uint32_t flip_window(const PointConst &a, uint32_t path, uint32_t wlen, uint32_t off,
                                                uint32_t &mD, int32_t d, uint32_t *q, uint32_t qs)
{
    uint32_t slot = 0;
    bool active = off < wlen;
    while (__any(active)) {
        if (active) {
            if (slot < JCAP) {
                d = 1 - d;
                const uint32_t sn = flip_draw<R>(a, path, mD, d);
                q[slot * qs] = off;
                ++slot;
                ++mD;
                off = off + 1u + sn;
                active = off < wlen;
            } else {
                active = false;
            }
        }
    }
    const bool full = slot == JCAP && off < wlen;
    q[slot * qs] = full ? (off | INLINE_BIT) : off;
    return full ? off : wlen;
}

// ---------------------------------------------------------------------------
// Algorithm 1: one predictor-corrector step.  A0 / A1 are the constant-within-
// step forcing at t_n / t_{n+1} (drive, tilt, Poisson bias, dichotomous level:
// part of the drift in all three evaluations); z is the Poisson kick, added once
// in the corrector; hh = dt / 2.
// ---------------------------------------------------------------------------
template <int DYN, int POT, bool KICK, typename R>
__device__ __forceinline__ void pc_step(Path<R> &s, R h, R hh, R ngam, R kp, R dxi, R z, R A0, R A1)
{
    // The noise increment enters all three stages unchanged, so it is added to the
    // noisy component once (vd / xd) instead of after each stage.  The trapezoid
    // of the predictor and of the corrector share the half-step term of F1:
    // y + (F1 + F) dt/2 is formed as (y + F1 dt/2) + F dt/2, one FMA on a common
    // base instead of an add and an FMA each (the same sums in another rounding
    // order).  Inertial: three cosines, six FMAs in the drifts, nine operations in
    // the stages; overdamped: three cosines and five operations in the stages.
    if constexpr (DYN == DYN_INERTIAL) {
        const R x = s.x, v = s.v, vd = v + dxi;
        const R f1 = fma(ngam, v, force_plus<POT>(x, A0, kp));
        const R xb = fma(v, h, x);                             // Euler
        const R vb = fma(f1, h, vd);
        const R f2 = fma(ngam, vb, force_plus<POT>(xb, A1, kp));
        const R xc = fma(v, hh, x), vc = fma(f1, hh, vd);      // y_n + F1 dt/2
        const R xp = fma(vb, hh, xc);                          // predictor
        const R vpr = fma(f2, hh, vc);
        const R f3 = fma(ngam, vpr, force_plus<POT>(xp, A1, kp));
        s.x = fma(vpr, hh, xc);                                // corrector
        R vn = fma(f3, hh, vc);
        if constexpr (KICK) vn = vn + z;
        s.v = vn;
    } else {
        const R x = s.x, xd = x + dxi;
        const R f1 = force_plus<POT>(x, A0, kp);
        const R xb = fma(f1, h, xd);                           // Euler
        const R f2 = force_plus<POT>(xb, A1, kp);
        const R xc = fma(f1, hh, xd);                          // y_n + F1 dt/2
        const R xp = fma(f2, hh, xc);                          // predictor
        const R f3 = force_plus<POT>(xp, A1, kp);
        R xn = fma(f3, hh, xc);                                // corrector
        if constexpr (KICK) xn = xn + z;
        s.x = xn;
    }
}

// Algorithm 1 as pc_step (no kick), also returning the local error estimate of the
// paragraph after the algorithm: chi = predictor - corrector, as max(|chi_x|, |chi_v|)
// for the inertial state (x, v).
template <int DYN, int POT, typename R>
__device__ __forceinline__ R pc_step_chi(Path<R> &s, R h, R hh, R ngam, R kp, R dxi, R A0, R A1)
{
    if constexpr (DYN == DYN_INERTIAL) {
        const R x = s.x, v = s.v, vd = v + dxi;
        const R f1 = fma(ngam, v, force_plus<POT>(x, A0, kp));
        const R xb = fma(v, h, x);                             // Euler
        const R vb = fma(f1, h, vd);
        const R f2 = fma(ngam, vb, force_plus<POT>(xb, A1, kp));
        const R xc = fma(v, hh, x), vc = fma(f1, hh, vd);      // y_n + F1 dt/2
        const R xp = fma(vb, hh, xc);                          // predictor
        const R vpr = fma(f2, hh, vc);
        const R f3 = fma(ngam, vpr, force_plus<POT>(xp, A1, kp));
        const R xn = fma(vpr, hh, xc);                         // corrector
        const R vn = fma(f3, hh, vc);
        s.x = xn;
        s.v = vn;
        return fmax(fabs(xp - xn), fabs(vpr - vn));
    } else {
        const R x = s.x, xd = x + dxi;
        const R f1 = force_plus<POT>(x, A0, kp);
        const R xb = fma(f1, h, xd);                           // Euler
        const R f2 = force_plus<POT>(xb, A1, kp);
        const R xc = fma(f1, hh, xd);                          // y_n + F1 dt/2
        const R xp = fma(f2, hh, xc);                          // predictor
        const R f3 = force_plus<POT>(xp, A1, kp);
        const R xn = fma(f3, hh, xc);                          // corrector
        s.x = xn;
        return fabs(xp - xn);
    }
}

// u * 6 mod 2^32 with two full-rate shifts (the compiler would otherwise emit a
// quarter-rate 32-bit multiply): the next base-6 digit of the fraction u / 2^32.
__device__ __forceinline__ uint32_t times6(uint32_t u)
{
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, 1, %1\n\tv_lshlrev_b32 %0, 1, %0" : "=v"(r) : "v"(u));
    return r;
}

} // namespace bm
