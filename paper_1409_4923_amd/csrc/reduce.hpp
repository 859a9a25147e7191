// reduce.hpp -- FP64 ensemble statistics (eq. 31 over the paths; Sec. 4 1/sqrt(N)
// error): double-double sums of v_p and v_p^2 per 64-path chunk, combined in an
// order that depends only on the number of chunks.  Compile with
// -ffp-contract=off (error-free transformations).
#pragma once

#include "bmotor.h"
#include "common.hpp"

namespace bm {

__device__ __forceinline__ void finish_stats(DD s1, DD s2, uint64_t n, uint64_t bad, double tw, bm_stats *out)
{
#pragma clang fp contract(off)
    bm_stats st;
    st.n = n;
    st.n_nonfinite = bad;
    st.t_window = tw;
    const double nn = (double)n;
    if (n == 0) {
        st.mean = st.var = st.se = __builtin_nan("");
    } else {
        // mean = s1 / n as a double-double
        const double mh = s1.hi / nn;
        const double r = ((s1.hi - mh * nn) - fma(mh, nn, -(mh * nn))) + s1.lo;
        const double ml = r / nn;
        st.mean = mh + ml;
        if (n < 2) {
            st.var = st.se = __builtin_nan("");
        } else {
            // s2 - s1 * mean, with the product kept to double-double accuracy
            const double p = s1.hi * mh;
            const double pe = fma(s1.hi, mh, -p) + (s1.hi * ml + s1.lo * mh);
            const DD num = dd_add(s2, DD{-p, -pe});
            const double var = (num.hi + num.lo) / (nn - 1.0);
            st.var = var;
            st.se = sqrt(var / nn);
        }
    }
    *out = st;
}

// One 256-lane work-group combines n_chunks partials: lane t folds chunks
// [n t / 256, n (t+1) / 256) in order, then a fixed LDS tree; lane 0 writes.
__device__ __forceinline__ void reduce_chunks(const Partial *part, uint64_t n_chunks, double tw, bm_stats *out)
{
    __shared__ double l1h[256], l1l[256], l2h[256], l2l[256];
    __shared__ uint64_t lc[256], lb[256];
    const uint32_t t = threadIdx.x;
    const uint64_t lo = n_chunks * t / 256, hi = n_chunks * (t + 1) / 256;
    DD s1{0.0, 0.0}, s2{0.0, 0.0};
    uint64_t c = 0, b = 0;
    for (uint64_t i = lo; i < hi; ++i) {
        const Partial q = part[i];
        s1 = dd_add(s1, DD{q.s1_hi, q.s1_lo});
        s2 = dd_add(s2, DD{q.s2_hi, q.s2_lo});
        c += q.n;
        b += q.n_bad;
    }
    l1h[t] = s1.hi; l1l[t] = s1.lo; l2h[t] = s2.hi; l2l[t] = s2.lo; lc[t] = c; lb[t] = b;
    __syncthreads();
    for (uint32_t st = 128; st >= 1; st >>= 1) {
        if (t < st) {
            const DD a1{l1h[t], l1l[t]}, b1{l1h[t + st], l1l[t + st]};
            const DD a2{l2h[t], l2l[t]}, b2{l2h[t + st], l2l[t + st]};
            const DD r1 = dd_add(a1, b1), r2 = dd_add(a2, b2);
            l1h[t] = r1.hi; l1l[t] = r1.lo; l2h[t] = r2.hi; l2l[t] = r2.lo;
            lc[t] += lc[t + st];
            lb[t] += lb[t + st];
        }
        __syncthreads();
    }
    if (t == 0) finish_stats(DD{l1h[0], l1l[0]}, DD{l2h[0], l2l[0]}, lc[0], lb[0], tw, out);
}


// Per-wave partial of 64 consecutive paths: exact-error butterfly (commutative,
// so every lane ends with the same bits).  Lanes without a path pass have = false.
__device__ __forceinline__ Partial wave_partial(double vp, bool have)
{
    const bool fin = have && isfinite(vp);
    DD s1 = dd_from(fin ? vp : 0.0);
    DD s2 = dd_from(0.0);
    if (fin) {
        const double sq = vp * vp;
        s2 = DD{sq, fma(vp, vp, -sq)};              // exact square as a double-double
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
    return Partial{s1.hi, s1.lo, s2.hi, s2.lo, cnt, bad};
}

} // namespace bm
