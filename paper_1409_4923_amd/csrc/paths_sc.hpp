// paths_sc.hpp -- the integration kernel with step-size control on chi (the
// paragraph after Algorithm 1: the difference between predictor and corrector
// estimates the local error and can steer the step size).
//
// One wavefront is one control group of 64 consecutive paths, so the step size,
// the position inside the current step of dt and the index of the next random draw
// are wave-uniform (scalar registers): the control costs two compares and two ballots
// per step, never a divergent branch.  Steps are dt / 2^l, l <= J; a step may double
// only where the doubled step starts on its own grid, so no step crosses a multiple
// of dt and the drive at t = (n + u / 2^J) dt is entry (n mod spp) 2^J + u of a table
// built on the host.  The jump processes keep their dt grid (Algorithms 3 and 4,
// drawn inline when a countdown runs out: rare, and not worth the window queues of
// the fixed-step kernel).
#pragma once

#include "paths_kernels.hpp"

namespace bm {

template <typename R, int DYN, int POT>
__global__ void __launch_bounds__(512) k_advance_sc(const KArgs a)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const PointConst &c = a.p;
    const uint32_t first = p & ~63u;                    // first path of this lane's group
    if (first >= c.n_paths) return;                     // the whole wave
    const bool valid = p < c.n_paths;
    const uint32_t path = valid ? p : first;            // lanes past the end shadow a valid path
    const bool hasG = (a.noise & NZ_GAUSS) != 0, hasP = (a.noise & NZ_POISSON) != 0,
               hasD = (a.noise & NZ_DICH) != 0;

    Path<R> s;
    s.x = arr<R>(a.x)[path];
    s.w = a.w[path];
    s.v = arr<R>(a.v)[path];
    s.sP = hasP ? a.sP[path] : 0;
    s.kP = hasP ? a.kP[path] : 0u;
    s.sD = hasD ? a.sD[path] : 0;
    s.mD = hasD ? a.mD[path] : 0u;
    s.d = hasD ? a.d[path] : 0;
    s.thP = 0.0;
    // group-uniform control state, taken from the group's first path
    uint32_t lev = __builtin_amdgcn_readfirstlane((uint32_t)a.lev[first]);
    uint32_t k = __builtin_amdgcn_readfirstlane(a.kA[first]);
    const uint32_t J = a.sc_J, full = 1u << J;
    lev = lev < J ? lev : J;                            // the host keeps it in range; never index past it
    const R tol = (R)a.sc_tol, tol16 = (R)(a.sc_tol * 0.0625);
    const R ngam = (R)(-c.gamma), kp = pot_factor<POT, R>();
    const R Fa = (R)c.Fa, Fb = (R)c.Fb;
    const R *tab = reinterpret_cast<const R *>(c.tab);

    U4 q = U4{0u, 0u, 0u, 0u};
    uint32_t uw = 0u;
    bool fresh = true;                                  // q / uw not yet formed for draw k
    uint32_t kph = (uint32_t)(a.n0 % c.spp);
    for (uint64_t n = a.n0; n < a.n1; ++n) {
        // Algorithms 4 and 3 at step n of dt (countdown semantics of the fixed grid)
        R level = R(0), z = R(0);
        if (hasD) {
            if (s.sD <= 0) {
                s.d = 1 - s.d;
                s.sD = (int32_t)flip_draw<R>(c, path, s.mD, s.d);
                ++s.mD;
            } else {
                --s.sD;
            }
            level = s.d ? Fb : -Fa;
        }
        if (hasP) {
            if (s.sP <= 0) {
                const U4 b = philox4x32_10(s.kP >> 1, path, c.point, TAG_POISSON, c.key0, c.key1);
                const bool second = (s.kP & 1u) != 0u;
                uint32_t sn;
                kick_from<R>(c, second ? b.z : b.x, second ? b.w : b.y, sn, z);
                s.sP = (int32_t)sn;
                ++s.kP;
            } else {
                --s.sP;
            }
        }
        const uint32_t base = kph << J;
        uint32_t u = 0;
        while (u < full) {
            const uint32_t hu = 1u << (J - lev);
            const R h = (R)a.sc_h[lev];
            const R hh = h * R(0.5);
            R dxi = R(0);
            if (hasG) {
                if (fresh || (k & 15u) == 0u)
                    q = philox4x32_10(k >> 4, path, c.point, TAG_GAUSS, c.key0, c.key1);
                if (fresh || (k & 3u) == 0u) {
                    uw = pick(q, (k >> 2) & 3u);
                    for (uint32_t t = 0; t < (k & 3u); ++t) uw = times6(uw);
                }
                fresh = false;
                dxi = three_point<R>(uw, (R)a.sc_g3[lev]);
                uw = times6(uw);                        // the next base-6 digit
            }
            const R A0 = tab[base + u] + level, A1 = tab[base + u + hu] + level;
            const R chi = pc_step_chi<DYN, POT, R>(s, h, hh, ngam, kp, dxi, A0, A1);
            ++k;
            u += hu;
            const bool over = valid && !(chi <= tol);          // a NaN counts as too large
            const bool big = valid && !(chi < tol16);
            if (__builtin_amdgcn_ballot_w64(over) != 0) {
                if (lev < J) ++lev;
            } else if (__builtin_amdgcn_ballot_w64(big) == 0 && lev > 0 && (u & (2u * hu - 1u)) == 0u) {
                --lev;
            }
        }
        if (hasP) {                                     // the kick of step n, after its last sub-step
            if constexpr (DYN == DYN_INERTIAL) s.v = s.v + z;
            else s.x = s.x + z;
        }
        fold<POT, R>(s);
        kph = (kph + 1u == c.spp) ? 0u : kph + 1u;
    }
    if (!valid) return;
    arr<R>(a.x)[path] = s.x;
    a.w[path] = s.w;
    arr<R>(a.v)[path] = s.v;
    if (hasP) { a.sP[path] = s.sP; a.kP[path] = s.kP; }
    if (hasD) { a.sD[path] = s.sD; a.mD[path] = s.mD; a.d[path] = s.d; }
    a.lev[path] = (int32_t)lev;
    a.kA[path] = k;
    if (a.snapshot) { arr<R>(a.xi)[path] = s.x; a.wi[path] = s.w; }
}

} // namespace bm
