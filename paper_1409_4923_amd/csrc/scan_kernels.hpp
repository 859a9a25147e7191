// scan_kernels.hpp -- persistent, work-stealing parameter scan (the paper's
// "solve for multiple values of the system parameters in a single kernel call",
// Sec. 5, Execution configuration optimizations).
//
// Work items are (point, chunk of 64 * PPL paths), ordered longest-first on the
// host.  Every wave of a persistent grid repeatedly claims the next item with one
// atomic add, integrates its paths over the point's whole horizon with the same
// device code as the ensemble path (initial conditions, Algorithms 1-4, window
// snapshot), and writes one double-double partial per 64 paths.  A per-point
// kernel then combines the partials in the same fixed order as bm_reduce, so a
// scan point equals the ensemble result for that point bit for bit.
#pragma once

#include "paths_kernels.hpp"

namespace bm {

struct ScanItem {
    uint32_t point;    // index into the point table
    uint32_t chunk;    // chunk of 64 * PPL paths
};

struct PointRed {
    uint64_t off;      // first 64-path partial of the point
    uint64_t n_chunks; // number of 64-path partials
    double tw;         // t_f - t_i
};

struct ScanArgs {
    const PointConst *points;
    const ScanItem *items;
    const PointRed *red;
    Partial *part;
    uint32_t *counter;
    uint32_t n_items;
    uint32_t pad;
};

template <typename R, int DYN, int POT, int NOISE, int PPL>
__global__ void __launch_bounds__(512) k_scan(const ScanArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t qs = PPL * blockDim.x;
    const double L = period<POT>();
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(a.counter, 1u);
        it = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl(it, 0, 64));
        if (it >= a.n_items) break;                      // every wave exits here
        const ScanItem item = a.items[it];
        const PointConst P = a.points[item.point];
        const uint32_t base = item.chunk * 64u * PPL + lane;
        uint32_t path[PPL];
        bool valid[PPL];
        Path<R> s[PPL];
        R xi[PPL];
        int32_t wi[PPL];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            const uint32_t p = base + 64u * (uint32_t)j;
            valid[j] = p < P.n_paths;
            path[j] = valid[j] ? p : P.n_paths - 1u;
            s[j] = init_path<R, DYN, POT, NOISE>(P, path[j]);
            xi[j] = s[j].x;
            wi[j] = s[j].w;
        }
        advance_range<R, DYN, POT, NOISE, PPL>(P, path, s, 0, P.n_window, smem, qs, threadIdx.x);
#pragma unroll
        for (int j = 0; j < PPL; ++j) { xi[j] = s[j].x; wi[j] = s[j].w; }
        advance_range<R, DYN, POT, NOISE, PPL>(P, path, s, P.n_window, P.n_steps, smem, qs, threadIdx.x);
        const PointRed rd = a.red[item.point];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            const double dx = (double)(s[j].w - wi[j]) * L + ((double)s[j].x - (double)xi[j]);
            const Partial q = wave_partial(dx / rd.tw, valid[j]);
            const uint64_t c64 = (uint64_t)item.chunk * PPL + (uint64_t)j;
            if (lane == 0 && c64 < rd.n_chunks) a.part[rd.off + c64] = q;
        }
    }
}

} // namespace bm
