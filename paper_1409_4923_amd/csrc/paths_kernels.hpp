// paths_kernels.hpp -- __global__ kernels of the single-ensemble path:
// initial conditions, the hot integration loop, per-path velocity with wave
// partials, and the state export.  Included once per precision/dynamics
// translation unit (paths_f32.hip, paths_f64.hip), which instantiate them.
#pragma once

#include "paths.hpp"

namespace bm {

template <typename R> __device__ __forceinline__ R *arr(void *p) { return reinterpret_cast<R *>(p); }

template <typename R, int POT, int NOISE>
__device__ __forceinline__ void load_path(const KArgs &a, uint32_t p, Path<R> &s)
{
    s.x = arr<R>(a.x)[p];
    s.w = a.w[p];
    s.v = arr<R>(a.v)[p];
    if constexpr ((NOISE & NZ_POISSON) != 0) { s.sP = a.sP[p]; s.kP = a.kP[p]; }
    else { s.sP = 0; s.kP = 0u; }
    if constexpr ((NOISE & NZ_DICH) != 0) { s.sD = a.sD[p]; s.mD = a.mD[p]; s.d = a.d[p]; }
    else { s.sD = 0; s.mD = 0u; s.d = 0; }
}

template <typename R, int POT, int NOISE>
__device__ __forceinline__ void store_path(const KArgs &a, uint32_t p, const Path<R> &s)
{
    arr<R>(a.x)[p] = s.x;
    a.w[p] = s.w;
    arr<R>(a.v)[p] = s.v;
    if constexpr ((NOISE & NZ_POISSON) != 0) { a.sP[p] = s.sP; a.kP[p] = s.kP; }
    if constexpr ((NOISE & NZ_DICH) != 0) { a.sD[p] = s.sD; a.mD[p] = s.mD; a.d[p] = s.d; }
    if (a.snapshot) { arr<R>(a.xi)[p] = s.x; a.wi[p] = s.w; }
}

// Drive + tilt at phase k (0 <= k < spp), or the constant tilt without a drive.
template <typename R> __device__ __forceinline__ R drive_at(const KArgs &a, uint32_t k)
{
    return a.spp ? reinterpret_cast<const R *>(a.tab)[k] : (R)a.F;
}

// One complete step n -> n+1 of one path: jump processes, then Algorithm 1, then
// folding.  `dxi` is the Algorithm 2 increment for this step.
template <typename R, int DYN, int POT, int NOISE>
__device__ __forceinline__ void full_step(const KArgs &a, uint32_t path, Path<R> &s, R dxi, R h,
                                          R gam, R A0, R A1, R bias, R Fa, R Fb)
{
    R z = R(0);
    if constexpr ((NOISE & NZ_POISSON) != 0) z = poisson_update<R>(a, path, s);
    if constexpr ((NOISE & NZ_DICH) != 0) dich_update<R>(a, path, s);
    R cst = R(0);
    if constexpr ((NOISE & NZ_DICH) != 0) cst = s.d ? Fb : -Fa;
    if constexpr ((NOISE & NZ_POISSON) != 0) cst = cst - bias;
    pc_step<DYN, POT, R>(s, h, gam, dxi, z, A0, A1, cst);
    fold<POT, R>(s);
}

template <typename R>
__device__ __forceinline__ R three_point(uint32_t u, R g3)
{
    return u < T_MINUS ? -g3 : (u < T_PLUS ? g3 : R(0));
}

// ---------------------------------------------------------------------------
// Integration kernel: advances paths over steps [n0, n1).  Steps are grouped in
// blocks of 16 sharing one Philox call for Algorithm 2 (4 words x 4 base-6
// digits).  Lane layout: path = (blockIdx.x * PPL + j) * blockDim.x + threadIdx.x.
// ---------------------------------------------------------------------------
template <typename R, int DYN, int POT, int NOISE, int PPL>
__global__ void __launch_bounds__(512) k_advance(const KArgs a)
{
    const uint32_t base = blockIdx.x * PPL * blockDim.x + threadIdx.x;
    if ((uint64_t)base >= a.n_paths) return;
    uint32_t path[PPL];
    bool valid[PPL];
    Path<R> s[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const uint64_t p = (uint64_t)base + (uint64_t)j * blockDim.x;
        valid[j] = p < a.n_paths;
        path[j] = valid[j] ? (uint32_t)p : base;
        load_path<R, POT, NOISE>(a, path[j], s[j]);
    }
    const R h = (R)a.dt, gam = (R)a.gamma, g3 = (R)a.g3;
    const R bias = (R)a.bias, Fa = (R)a.Fa, Fb = (R)a.Fb;

    uint64_t n = a.n0;
    uint32_t k = a.spp ? (uint32_t)(n % a.spp) : 0u;
    R A0 = drive_at<R>(a, k);

    // Generic single step (used at block-unaligned starts and ends).
    auto one_step = [&](uint64_t nn) {
        const uint32_t k1 = (a.spp && k + 1u == a.spp) ? 0u : k + 1u;
        const R A1 = drive_at<R>(a, a.spp ? k1 : 0u);
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            R dxi = R(0);
            if constexpr ((NOISE & NZ_GAUSS) != 0) {
                const U4 q = philox4x32_10((uint32_t)(nn >> 4), path[j], a.point, TAG_GAUSS,
                                           a.key0, a.key1);
                uint32_t u = pick(q, (uint32_t)(nn >> 2) & 3u);
                for (uint32_t t = 0; t < (uint32_t)(nn & 3u); ++t) u *= 6u;
                dxi = three_point<R>(u, g3);
            }
            full_step<R, DYN, POT, NOISE>(a, path[j], s[j], dxi, h, gam, A0, A1, bias, Fa, Fb);
        }
        k = k1;
        A0 = A1;
    };

    while (n < a.n1 && (n & 15u) != 0u) { one_step(n); ++n; }

    while (n + 16u <= a.n1) {
        U4 q[PPL];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            if constexpr ((NOISE & NZ_GAUSS) != 0)
                q[j] = philox4x32_10((uint32_t)(n >> 4), path[j], a.point, TAG_GAUSS, a.key0, a.key1);
            else
                q[j] = U4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int wd = 0; wd < 4; ++wd) {
            uint32_t u[PPL];
#pragma unroll
            for (int j = 0; j < PPL; ++j) u[j] = pick(q[j], (uint32_t)wd);
#pragma unroll
            for (int dg = 0; dg < 4; ++dg) {
                const uint32_t k1 = (a.spp && k + 1u == a.spp) ? 0u : k + 1u;
                const R A1 = drive_at<R>(a, a.spp ? k1 : 0u);
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    R dxi = R(0);
                    if constexpr ((NOISE & NZ_GAUSS) != 0) {
                        dxi = three_point<R>(u[j], g3);
                        u[j] *= 6u;   // next base-6 digit
                    }
                    full_step<R, DYN, POT, NOISE>(a, path[j], s[j], dxi, h, gam, A0, A1, bias, Fa, Fb);
                }
                k = k1;
                A0 = A1;
            }
        }
        n += 16u;
    }

    while (n < a.n1) { one_step(n); ++n; }

#pragma unroll
    for (int j = 0; j < PPL; ++j)
        if (valid[j]) store_path<R, POT, NOISE>(a, path[j], s[j]);
}

// ---------------------------------------------------------------------------
// Initial conditions (tag 2), computed in FP64 and stored in the path precision.
// ---------------------------------------------------------------------------
template <typename R, int DYN, int POT, int NOISE>
__global__ void __launch_bounds__(256) k_init(const KArgs a)
{
    const uint64_t p64 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p64 >= a.n_paths) return;
    const uint32_t p = (uint32_t)p64;
    const U4 q = philox4x32_10(0u, p, a.point, TAG_INIT, a.key0, a.key1);
    const double L = period<POT>();
    double x = a.x0_lo + a.x0_w * ((double)q.x * 0x1p-32);
    const double kf = floor(x / L);
    x = x - kf * L;
    int32_t w = (int32_t)kf;
    R xr = (R)x;
    if (xr >= (R)L) { xr -= (R)L; w += 1; }   // rounding to the path precision may reach L
    const double v = (DYN == DYN_INERTIAL) ? a.v0_lo + a.v0_w * ((double)q.y * 0x1p-32) : 0.0;
    arr<R>(a.x)[p] = xr;
    a.w[p] = w;
    arr<R>(a.v)[p] = (R)v;
    if constexpr ((NOISE & NZ_POISSON) != 0) {
        a.sP[p] = (int32_t)floor(expo64(q.z) / a.lam_dt);
        a.kP[p] = 0u;
    }
    if constexpr ((NOISE & NZ_DICH) != 0) {
        const int32_t dstar = ((double)q.w * 0x1p-32 < a.p_hi) ? 1 : 0;
        a.d[p] = 1 - dstar;    // step 0 flips into dstar and draws its dwell
        a.sD[p] = 0;
        a.mD[p] = 0u;
    }
    if (a.snapshot) { arr<R>(a.xi)[p] = xr; a.wi[p] = w; }
}

// ---------------------------------------------------------------------------
// eq. (31) per path in FP64, plus one double-double partial per wave (64 paths).
// Launched with 256-lane work-groups; chunk c covers paths [64c, 64c + 64).
// ---------------------------------------------------------------------------
template <typename R, int POT>
__global__ void __launch_bounds__(256) k_velocity(const KArgs a)
{
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double L = period<POT>();
    double vp = 0.0;
    bool have = p < a.n_paths;
    if (have) {
        const double dx = (double)(a.w[p] - a.wi[p]) * L +
                          ((double)arr<R>(a.x)[p] - (double)arr<R>(a.xi)[p]);
        vp = dx / a.t_window;
        a.vp[p] = vp;
    }
    const bool fin = have && isfinite(vp);
    DD s1 = dd_from(fin ? vp : 0.0);
    DD s2 = dd_from(fin ? vp * vp : 0.0);
    if (fin) {
        // exact square as a double-double: vp*vp + fma residual
        const double sq = vp * vp;
        s2 = DD{sq, fma(vp, vp, -sq)};
    }
    uint32_t cnt = fin ? 1u : 0u;
    uint32_t bad = (have && !fin) ? 1u : 0u;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        DD o1{__shfl_xor(s1.hi, off, 64), __shfl_xor(s1.lo, off, 64)};
        DD o2{__shfl_xor(s2.hi, off, 64), __shfl_xor(s2.lo, off, 64)};
        s1 = dd_add(s1, o1);
        s2 = dd_add(s2, o2);
        cnt += __shfl_xor(cnt, off, 64);
        bad += __shfl_xor(bad, off, 64);
    }
    const uint64_t chunk = p >> 6;
    if ((threadIdx.x & 63u) == 0u && (chunk << 6) < a.n_paths) {
        a.part[chunk] = Partial{s1.hi, s1.lo, s2.hi, s2.lo, cnt, bad};
    }
}

// ---------------------------------------------------------------------------
// Export of paths [n0, n0 + n1) (n0/n1 reused as first/count) to FP64 arrays.
// ---------------------------------------------------------------------------
template <typename R, int POT>
__global__ void __launch_bounds__(256) k_read(const KArgs a, double *xo, double *vo, int64_t *no,
                                              double *vpo, int with_vp)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n1) return;
    const uint64_t p = a.n0 + i;
    const double L = period<POT>();
    if (xo) xo[i] = (double)a.w[p] * L + (double)arr<R>(a.x)[p];
    if (vo) vo[i] = (double)arr<R>(a.v)[p];
    if (no) {
        no[5 * i + 0] = a.sP ? a.sP[p] : 0;
        no[5 * i + 1] = a.kP ? (int64_t)a.kP[p] : 0;
        no[5 * i + 2] = a.sD ? a.sD[p] : 0;
        no[5 * i + 3] = a.mD ? (int64_t)a.mD[p] : 0;
        no[5 * i + 4] = a.d ? a.d[p] : 0;
    }
    if (vpo && with_vp) {
        const double dx = (double)(a.w[p] - a.wi[p]) * L +
                          ((double)arr<R>(a.x)[p] - (double)arr<R>(a.xi)[p]);
        vpo[i] = dx / a.t_window;
    }
}

} // namespace bm
