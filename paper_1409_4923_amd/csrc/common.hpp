// common.hpp -- device primitives shared by the libbmotor kernels (gfx950).
//
//  * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw, SC'11):
//    ten rounds of two 32x32->64 products plus xors, key bumped by the Weyl
//    constants between rounds.  One lane evaluates one block; nothing is stored.
//  * Double-double (hi, lo) accumulation for the FP64 ensemble reduction.
//  * Kernel argument block and random-stream tags.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bm {

// ---------------------------------------------------------------------------
// Random-stream layout: counter = (index, path, point, tag), key = seed.
// ---------------------------------------------------------------------------
enum : uint32_t {
    TAG_GAUSS = 0u,    // index = step / 16; word (step % 16) / 4; base-6 digit step % 4
    TAG_POISSON = 1u,  // index = kick / 2; words (2 (kick % 2), 2 (kick % 2) + 1)
    TAG_INIT = 2u,     // index = 0; words: x0, v0, Poisson countdown, dichotomous state
    TAG_DICH = 3u,     // index = flip / 4; word flip % 4
    TAG_KICK_NOISE = 5u, // jump-adapted grid: Gaussian increment of the piece after kick k
                         // (three-point: index k / 16, word (k % 16) / 4, digit k % 4;
                         //  normal: index k / 4, words (2j, 2j+1), j = (k % 4) / 2)
};

// Thresholds of Algorithm 2 on a 32-bit word u (fraction u / 2^32):
// leading base-6 digit 0  <=>  u < ceil(2^32 / 6);  digit <= 1  <=>  u < ceil(2^32 / 3).
constexpr uint32_t T_MINUS = 715827883u;
constexpr uint32_t T_PLUS = 1431655766u;

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
    constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)MA * c0;
        const uint64_t pb = (uint64_t)MB * c2;
        const uint32_t t0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t t2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = t0;
        c2 = t2;
        k0 += WA;
        k1 += WB;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t pick(const U4 &q, uint32_t i)
{
    return i == 0 ? q.x : (i == 1 ? q.y : (i == 2 ? q.z : q.w));
}

// E = -ln(1 - phi), phi = w 2^-32 in [0, 1): an Exp(1) variate (eq. 27), FP64.
__device__ __forceinline__ double expo64(uint32_t w)
{
    const double phi = (double)w * 0x1p-32;
    return -log(1.0 - phi);
}

// ---------------------------------------------------------------------------
// Double-double arithmetic (Knuth two-sum); every sum below is exact-error
// compensated, so the result does not depend on which of two operands is first.
// ---------------------------------------------------------------------------
struct DD { double hi, lo; };

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
#pragma clang fp contract(off)
    const double s = a.hi + b.hi;
    const double bb = s - a.hi;
    const double e = (a.hi - (s - bb)) + (b.hi - bb);
    const double lo = e + (a.lo + b.lo);
    const double hi = s + lo;
    return DD{hi, lo - (hi - s)};
}

__device__ __forceinline__ DD dd_from(double x) { return DD{x, 0.0}; }

// ---------------------------------------------------------------------------
// Per-chunk partial of the ensemble reduction (one wave = 64 consecutive paths).
// ---------------------------------------------------------------------------
struct Partial {
    double s1_hi, s1_lo;   // sum of finite v_p
    double s2_hi, s2_lo;   // sum of finite v_p^2
    uint64_t n, n_bad;     // finite / non-finite counts
};

// ---------------------------------------------------------------------------
// Constants of one parameter point (one ensemble, or one point of a scan).
// ---------------------------------------------------------------------------
constexpr uint32_t JW_LOG2_MAX = 10;  // longest jump window of the path kernels: 1024 steps

struct PointConst {
    const void *tab;      // forcing table, k < spp + 16 (float/double), see drive_at
    uint32_t spp;         // period of the forcing table in steps (1: no periodic drive)
    uint32_t point;       // point index in the random-stream counter
    uint32_t key0, key1;  // Philox key (seed)
    uint32_t n_paths;
    uint32_t jw_log2;     // jump window of 2^jw_log2 steps (>= 16)
    uint64_t n_steps;     // horizon (scan)
    uint64_t n_window;    // eq. (31): step index of t_i
    double dt, gamma;
    double g3;            // G sqrt(3 dt) (three-point), G sqrt(dt) (normal increments)
    double lam_dt;        // lambda dt
    double zeta;
    double Fa, Fb;
    double mua_dt, mub_dt;
    double p_hi;          // stationary Pr{+Fb} = mu_a / (mu_a + mu_b)
    double x0_lo, x0_w, v0_lo, v0_w;
    double drive_a;       // drive amplitude (forcing inside a step on the jump-adapted grid)
    double drive_c;       // constant forcing: tilt - Poisson bias + potential offset
    // FP32 estimates of the countdown X = E / (rate dt): X ~= -log2(1 - phi) * c,
    // trusted when its fraction is farther than tol0 + tol1 X from an integer.
    float c_lam, c_mua, c_mub;   // ln 2 / (rate dt)
    float tol0_lam, tol0_mua, tol0_mub, tol1;
    float zeta_ln2;              // -zeta ln 2: z = zeta E = log2(1 - phi) * zeta_ln2
    float inv_spp;               // 1 / spp (the drive phase inside a step, FP32 paths)
};

// ---------------------------------------------------------------------------
// Kernel arguments of the ensemble kernels (passed by value).  Arrays are
// structure-of-arrays over paths.
// ---------------------------------------------------------------------------
struct KArgs {
    void *x;              // folded position: float or double
    int32_t *w;           // folded periods
    void *v;              // velocity (inertial): float or double
    void *xi;             // position at the window start
    int32_t *wi;          // periods at the window start
    int32_t *sP;          // Algorithm 3 countdown
    uint32_t *kP;         // Poisson kicks so far
    int32_t *sD;          // Algorithm 4 countdown
    uint32_t *mD;         // dichotomous flips so far
    int32_t *d;           // dichotomous state (0: -Fa, 1: +Fb)
    double *vp;           // per-path velocity, eq. (31)
    double *thP;          // jump-adapted grid: fraction of its step at which the next kick falls
    Partial *part;        // per-chunk partials
    PointConst p;
    uint64_t n0, n1;      // step range of this launch (export: first path, count)
    uint32_t snapshot;    // store the window snapshot at the end of the launch
    uint32_t pad;
    double t_window;      // (n - n_window) dt for the velocity kernel
    // step-size control on chi (0 halvings: off)
    int32_t *lev;         // per path: current step dt / 2^lev (the same in a group of 64)
    uint32_t *kA;         // per path: steps taken (index of the next Algorithm 2 draw)
    uint32_t sc_J;        // most halvings
    uint32_t noise;       // noise mask of the model
    double sc_tol;        // tolerance on max(|chi_x|, |chi_v|)
    double sc_h[9];       // step of each level, dt / 2^l
    double sc_g3[9];      // its three-point size G sqrt(3 dt / 2^l)
};
constexpr uint32_t SC_MAX_HALVINGS = 8;

} // namespace bm
