// paths_kernels.hpp -- __global__ kernels of the single-ensemble path:
// initial conditions, the hot integration loop, per-path velocity with wave
// partials, and the state export.  Included once per precision/dynamics
// translation unit (paths_f32.hip, paths_f64.hip), which instantiate them.
#pragma once

#include <type_traits>

#include "bmotor.h"
#include "launch.hpp"
#include "paths.hpp"
#include "reduce.hpp"

namespace bm {

template <typename R> __device__ __forceinline__ R *arr(void *p) { return reinterpret_cast<R *>(p); }

template <typename R>
__device__ __forceinline__ R three_point(uint32_t u, R g3)
{
    return u < T_MINUS ? -g3 : (u < T_PLUS ? g3 : R(0));
}

template <typename R, int POT, int NOISE>
__device__ __forceinline__ void load_path(const KArgs &a, uint32_t p, Path<R> &s)
{
    s.x = arr<R>(a.x)[p];
    s.w = a.w[p];
    s.v = arr<R>(a.v)[p];
    if constexpr ((NOISE & NZ_POISSON) != 0) { s.sP = a.sP[p]; s.kP = a.kP[p]; }
    else { s.sP = 0; s.kP = 0u; }
    if constexpr ((NOISE & NZ_JGRID) != 0) s.thP = a.thP[p];
    else s.thP = 0.0;
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
    if constexpr ((NOISE & NZ_JGRID) != 0) a.thP[p] = s.thP;
    if constexpr ((NOISE & NZ_DICH) != 0) { a.sD[p] = s.sD; a.mD[p] = s.mD; a.d[p] = s.d; }
    if (a.snapshot) { arr<R>(a.xi)[p] = s.x; a.wi[p] = s.w; }
}

// Constant-within-step forcing at phase k: drive + tilt - Poisson bias + potential
// offset, from the host-built table (period a.spp >= 1, extended by 16 entries so
// that the 17 values of a 16-step block are contiguous).
template <typename R> __device__ __forceinline__ R drive_at(const PointConst &a, uint32_t k)
{
    return reinterpret_cast<const R *>(a.tab)[k];
}

// Per-lane cursor into the LDS jump queues of the current window.

template <typename R> struct JumpCursor {
    uint32_t nP;    // offset of the next kick in the window
    R zP;           // its amplitude
    const KickEntry<R> *pP;   // the queue entry after it
    uint32_t nD;    // offset of the next flip
    uint32_t cD;    // element index of the next queue slot
    // jump-adapted grid
    JGKick<R> g;    // next kick (g.off == JG_NONE: none left in the window)
    uint32_t gs;    // queue slot of g
    uint32_t gn;    // kicks queued for this window
    uint32_t poff;  // offset of the first kick not yet drawn
    double pth;     // its fraction of the step (FP64: kick times decide the integer state)
};

// Forcing at the time t_n + theta dt inside a step of drive phase k (jump-adapted
// grid): a cos(2 pi (k + theta) / spp) + tilt - Poisson bias + potential offset.
// The phase k may be passed unreduced (k < spp + 16): cos is periodic in it.
template <typename R> __device__ __forceinline__ R drive_inside(const PointConst &a, uint32_t k, double th)
{
    if constexpr (sizeof(R) == 4) {
        const float turns = ((float)k + (float)th) * a.inv_spp;      // within 2 ulp of the quotient
        return (float)a.drive_a * __builtin_amdgcn_cosf(turns) + (float)a.drive_c;
    } else {
        constexpr double PI = 3.14159265358979323846;
        return a.drive_a * cos(2.0 * PI * ((double)k + th) / (double)a.spp) + a.drive_c;
    }
}

// Gaussian increment (times G sqrt(3 dt) or G sqrt(dt)) of the piece that follows
// kick k on the jump-adapted grid (tag 5, indexed by kick number).
template <typename R, int NOISE>
__device__ __forceinline__ R piece_noise(const PointConst &a, uint32_t path, uint32_t k, R g3)
{
    if constexpr ((NOISE & NZ_GAUSS) != 0) {
        const U4 q = philox4x32_10(k >> 4, path, a.point, TAG_KICK_NOISE, a.key0, a.key1);
        uint32_t u = pick(q, (k >> 2) & 3u);
        for (uint32_t t = 0; t < (k & 3u); ++t) u = times6(u);
        return three_point<R>(u, g3);
    } else if constexpr ((NOISE & NZ_NORMAL) != 0) {
        const U4 q = philox4x32_10(k >> 2, path, a.point, TAG_KICK_NOISE, a.key0, a.key1);
        const bool hi = ((k >> 1) & 1u) != 0;
        R zc, zs;
        normal_pair(hi ? q.z : q.x, hi ? q.w : q.y, zc, zs);
        return g3 * ((k & 1u) ? zs : zc);
    } else {
        return R(0);
    }
}

// sqrt of a piece's fraction of the step: the hardware square root (1 ulp) in FP32,
// the correctly rounded one in FP64.
__device__ __forceinline__ float piece_sqrt(float f) { return __builtin_amdgcn_sqrtf(f); }
__device__ __forceinline__ double piece_sqrt(double f) { return sqrt(f); }

// Most kicks one step of the jump-adapted grid may hold (a Poisson(16) count
// exceeds it with probability below 10^-1000).
constexpr uint32_t JG_MAX_KICKS = 4096;

// Time of the next kick in steps from the start of the current one's step: th + E /
// (lambda dt) in FP64 (out of line: it is needed once per kick, not per step).
__device__ __noinline__ double jg_next_time(double th, uint32_t w, double lam_dt)
{
    return th + expo64(w) / lam_dt;
}

// Draws the kick that falls at (off, th) of the window -- its amplitude, the
// increment of the piece after it -- and the time of the next kick, counted from
// it in FP64: off += floor(T), th = T - floor(T) with T = th + E / (lambda dt).
template <typename R, int NOISE>
__device__ __forceinline__ JGKick<R> jg_draw(const PointConst &a, uint32_t path, uint32_t &kP, uint32_t &off,
                                             double &th)
{
    const U4 b = philox4x32_10(kP >> 1, path, a.point, TAG_POISSON, a.key0, a.key1);
    const bool second = (kP & 1u) != 0u;
    JGKick<R> e;
    e.off = off;
    e.th = (R)th;
    e.z = amplitude<R>(a, second ? b.w : b.y);
    e.u = piece_noise<R, NOISE>(a, path, kP, (R)a.g3);
    const double T = jg_next_time(th, second ? b.z : b.x, a.lam_dt);
    const double Tf = floor(T);
    off += (uint32_t)Tf;                     // < 2^31 + window: validated on the host
    th = T - Tf;
    ++kP;
    return e;
}

// The same draw out of line, for the rare step that holds more kicks than a queue
// (arguments and results by value, so that the caller's state stays in registers).
template <typename R> struct JGDrawn {
    JGKick<R> e;
    double th;
    uint32_t kP, off;
};
template <typename R, int NOISE>
__device__ __noinline__ JGDrawn<R> jg_draw_inline(const PointConst a, uint32_t path, uint32_t kP, uint32_t off,
                                                  double th)
{
    JGDrawn<R> d;
    d.e = jg_draw<R, NOISE>(a, path, kP, off, th);
    d.th = th;
    d.kP = kP;
    d.off = off;
    return d;
}

// Fill the queue of one window (wave-uniform loop, as for the fixed grid) behind the
// J.gn kicks carried over from the previous window, up to jg_cap<R>() kicks, with the
// kicks that fall before the window's end.  Returns the number of leading steps of
// the window whose kicks are all queued: wlen, or, when the queue is full, the offset
// of the first kick it does not hold (J.poff).
template <typename R, int NOISE>
__device__ __forceinline__ uint32_t jg_window(const PointConst &a, uint32_t path, uint32_t wlen, uint32_t &kP,
                                              JumpCursor<R> &J, JGKick<R> *q, uint32_t qs)
{
    uint32_t slot = J.gn;
    bool active = J.poff < wlen && slot < jg_cap<R>();
    while (__any(active)) {
        if (active) {
            q[slot * qs] = jg_draw<R, NOISE>(a, path, kP, J.poff, J.pth);
            ++slot;
            active = J.poff < wlen && slot < jg_cap<R>();
        }
    }
    J.gn = slot;
    J.gs = 0;
    if (slot > 0) J.g = q[0];
    else J.g.off = JG_NONE;
    return J.poff < wlen ? J.poff : wlen;
}

// At the end of a window of wlen steps: the kicks still queued (drawn for steps past
// an early end) move to the front of the queue with their offsets rebased, and the
// offset of the first kick not yet drawn is rebased too.  The kick draws stay in
// their sequence, so nothing is drawn twice or given back.
template <typename R>
__device__ __forceinline__ void jg_carry(JumpCursor<R> &J, JGKick<R> *q, uint32_t qs, uint32_t wlen)
{
    const uint32_t left = J.gn - J.gs;                    // gs <= gn <= jg_cap (jg_advance)
    for (uint32_t i = 0; i < jg_cap<R>() && __any(i < left); ++i) {
        if (i < left) {
            JGKick<R> e = q[(J.gs + i) * qs];               // source index >= destination
            e.off -= wlen;
            q[i * qs] = e;
        }
    }
    J.gn = left;
    J.gs = 0;
    J.poff -= wlen;
}

// Moves the cursor past the kick just applied.  Within a window every kick before
// its end is queued; only the single-step fallback (INL) draws past its queue.  The
// cursor index stops at the queue's end (gs <= gn), also while kicks are drawn inline.
template <typename R, int NOISE, bool INL>
__device__ __forceinline__ void jg_advance(const PointConst &a, uint32_t path, uint32_t wlen, uint32_t &kP,
                                           JumpCursor<R> &J, const JGKick<R> *q, uint32_t qs)
{
    if (J.gs < J.gn) ++J.gs;                  // the kick applied was the queue's entry gs
    if (J.gs < J.gn) J.g = q[J.gs * qs];
    else if (INL && J.poff < wlen) {
        const JGDrawn<R> d = jg_draw_inline<R, NOISE>(a, path, kP, J.poff, J.pth);
        J.g = d.e;
        J.pth = d.th;
        J.poff = d.off;
        kP = d.kP;
    }
    else J.g.off = JG_NONE;
}

// One step of the jump-adapted grid.  When no lane of the wave has a kick in this
// step it is a plain Algorithm 1 step.  Otherwise every lane integrates the first
// piece of its step -- the whole step, or up to its first kick at t_n + theta dt --
// with the same instructions; lanes with a kick then integrate the remaining pieces
// (one per further kick in the step, then the rest of the step).  The first piece
// takes the step's own Gaussian increment scaled by sqrt(theta); a piece after
// kick k takes the increment drawn for k.
// The pieces of a kicked lane's step after its first kick (at fraction `from`, drive
// A_from there, u the increment of the next piece): one per further kick in the step,
// then the rest of the step.  The cursor already points past the first kick.
template <typename R, int DYN, int POT, int NOISE, bool INL>
__device__ __forceinline__ void jg_rest(const PointConst &a, uint32_t path, Path<R> &s, JumpCursor<R> &J,
                                        const JGKick<R> *q, uint32_t qs, uint32_t wlen, uint32_t off,
                                        uint32_t kph, R h, R hh, R ngam, R kp, R A1, R lev, R from, R A_from, R u)
{
    // further kicks in this step (lambda dt <= 16 is enforced on the host; the bound
    // only guarantees that every lane leaves the loop)
    for (uint32_t it = 0; J.g.off == off && it < JG_MAX_KICKS; ++it) {
        const R th = J.g.th;
        const R A_th = drive_inside<R>(a, kph, (double)th) + lev;
        pc_step<DYN, POT, true, R>(s, (th - from) * h, (th - from) * hh, ngam, kp, u * piece_sqrt(th - from), J.g.z,
                                   A_from, A_th);
        from = th;
        A_from = A_th;
        u = J.g.u;
        jg_advance<R, NOISE, INL>(a, path, wlen, s.kP, J, q, qs);
    }
    pc_step<DYN, POT, false, R>(s, (R(1) - from) * h, (R(1) - from) * hh, ngam, kp, u * piece_sqrt(R(1) - from), R(0),
                                A_from, A1);
}

template <typename R, int DYN, int POT, int NOISE, bool INL>
__device__ __forceinline__ void jg_step(const PointConst &a, uint32_t path, Path<R> &s, JumpCursor<R> &J,
                                        const JGKick<R> *q, uint32_t qs, uint32_t wlen, uint32_t off,
                                        uint32_t kph, R dxi, R h, R hh, R ngam, R kp, R A0, R A1, R lev)
{
    const bool kick = J.g.off == off;
    const bool any = __builtin_amdgcn_ballot_w64(kick) != 0;      // some lane of the wave kicks now
    R th1 = R(1), A_e = A1, dxi1 = dxi, z1 = R(0);
    if constexpr (sizeof(R) == 4 && !INL) {
        // FP32: one instance of the first piece for every step.  When a lane of the
        // wave kicks, the kick's length, drive, increment and amplitude are formed in
        // every lane and selected (no divergent branch; the cosine and the square root
        // go to the transcendental unit); otherwise the piece is the whole step
        // (th1 = 1 makes th1 dt exact).
        if (any) {
            const R thk = J.g.th;
            R A_k = drive_inside<R>(a, kph, (double)thk);
            if constexpr ((NOISE & NZ_DICH) != 0) A_k = A_k + lev;
            const R dxk = dxi * piece_sqrt(thk);
            th1 = kick ? thk : R(1);
            A_e = kick ? A_k : A1;
            dxi1 = kick ? dxk : dxi;
            z1 = kick ? J.g.z : R(0);
        }
        pc_step<DYN, POT, true, R>(s, th1 * h, th1 * hh, ngam, kp, dxi1, z1, A0, A_e);
        if (!any) return;
        // the kicked lanes' cursors move on: every lane reads the entry after its
        // cursor, the kicked lanes take it
        const R u_after = J.g.u;                 // increment of the piece after the kick
        const uint32_t nidx = J.gs < J.gn ? J.gs + 1u : J.gs;
        const bool more = nidx < J.gn;
        const JGKick<R> e = q[(more ? nidx : 0u) * qs];
        J.gs = kick ? nidx : J.gs;
        J.g.off = kick ? (more ? e.off : JG_NONE) : J.g.off;
        J.g.th = kick ? e.th : J.g.th;
        J.g.z = kick ? e.z : J.g.z;
        J.g.u = kick ? e.u : J.g.u;
        if (kick) jg_rest<R, DYN, POT, NOISE, INL>(a, path, s, J, q, qs, wlen, off, kph, h, hh, ngam, kp, A1, lev,
                                                   th1, A_e, u_after);
    } else {
        if (!any) {
            pc_step<DYN, POT, false, R>(s, h, hh, ngam, kp, dxi, R(0), A0, A1);
            return;
        }
        if (kick) {
            th1 = J.g.th;
            A_e = drive_inside<R>(a, kph, (double)th1) + lev;
            dxi1 = dxi * piece_sqrt(th1);
            z1 = J.g.z;
        }
        pc_step<DYN, POT, true, R>(s, th1 * h, th1 * hh, ngam, kp, dxi1, z1, A0, A_e);
        if (kick) {
            const R u_after = J.g.u;
            jg_advance<R, NOISE, INL>(a, path, wlen, s.kP, J, q, qs);
            jg_rest<R, DYN, POT, NOISE, INL>(a, path, s, J, q, qs, wlen, off, kph, h, hh, ngam, kp, A1, lev, th1,
                                             A_e, u_after);
        }
    }
}

// One step of one path at window offset `off` (drive phase kph): flips due at this
// step, Algorithm 1, and the Poisson kick due at this step, which Algorithm 3 adds
// to the corrector's result.  `dxi` is the Algorithm 2 increment.  (Folding is
// done by the caller.)
template <typename R, int DYN, int POT, int NOISE, bool INL = false>
__device__ __forceinline__ void full_step(const PointConst &a, uint32_t path, Path<R> &s, JumpCursor<R> &J,
                                          const JGKick<R> *gq, const uint32_t *fq,
                                          uint32_t qs, uint32_t wlen, uint32_t off, uint32_t kph, R dxi, R h,
                                          R hh, R ngam, R kp,
                                          R A0, R A1, R Fa, R Fb)
{
    if constexpr ((NOISE & NZ_DICH) != 0) {
        if (J.nD == off) {                       // Algorithm 4: s <= 0 at this step
            s.d = 1 - s.d;
            // the window ends before a full queue's marker: every flip is queued
            const uint32_t e = fq[J.cD];
            J.cD += qs;
            J.nD = e & ~INLINE_BIT;
        }
    }
    R lev = R(0);
    if constexpr ((NOISE & NZ_DICH) != 0) {
        lev = s.d ? Fb : -Fa;
        A0 = A0 + lev;
        A1 = A1 + lev;
    }
    if constexpr ((NOISE & NZ_JGRID) != 0) {
        jg_step<R, DYN, POT, NOISE, INL>(a, path, s, J, gq, qs, wlen, off, kph, dxi, h, hh, ngam, kp, A0, A1, lev);
    } else {
        pc_step<DYN, POT, false, R>(s, h, hh, ngam, kp, dxi, R(0), A0, A1);
    }
    if constexpr (queued_kicks<NOISE>()) {
        if (J.nP == off) {                       // Algorithm 3: s <= 0 at this step
            if constexpr (DYN == DYN_INERTIAL) s.v = s.v + J.zP;
            else s.x = s.x + J.zP;
            const KickEntry<R> e = *J.pP;
            J.pP += qs;
            J.nP = e.off;
            J.zP = e.z;
        }
    }
}


// LDS bytes of the jump queues per lane and path.
template <typename R, int NOISE> constexpr uint32_t queue_bytes()
{
    return (queued_kicks<NOISE>() ? (JCAP + 1) * (uint32_t)sizeof(KickEntry<R>) : 0u) +
           (((NOISE & NZ_JGRID) != 0) ? jg_cap<R>() * (uint32_t)sizeof(JGKick<R>) : 0u) +
           (((NOISE & NZ_DICH) != 0) ? (JCAP + 1) * 4u : 0u);
}

// ---------------------------------------------------------------------------
// The integration loop: advances PPL paths per lane over steps [n0, n1) in
// windows of 2^a.jw_log2 steps (aligned to multiples of it).  Per window the jumps are
// queued, then the steps run in blocks of 16 sharing one Philox call for
// Algorithm 2 (4 words x 4 base-6 digits; the normal increments of the
// non-simplified scheme take one call per 4 steps) and 17 scalar loads of the
// forcing table; x is folded after every step whose index is a multiple of 16.
// smem holds the jump queues, slot-major with stride qs; column col(j) is this
// lane's j-th path.
// ---------------------------------------------------------------------------
template <typename R, int DYN, int POT, int NOISE, int PPL>
__device__ __forceinline__ void advance_range(const PointConst &a, const uint32_t (&path)[PPL],
                                              Path<R> (&s)[PPL], uint64_t n0, uint64_t n1,
                                              unsigned char *smem, uint32_t qs, uint32_t col0)
{
    KickEntry<R> *kq = reinterpret_cast<KickEntry<R> *>(smem);
    JGKick<R> *gq = reinterpret_cast<JGKick<R> *>(smem);       // jump-adapted grid (no fixed-grid queue)
    uint32_t *fq = reinterpret_cast<uint32_t *>(
        smem + (queued_kicks<NOISE>() ? (JCAP + 1) * qs * sizeof(KickEntry<R>) : 0) +
        (((NOISE & NZ_JGRID) != 0) ? jg_cap<R>() * qs * sizeof(JGKick<R>) : 0));
    JumpCursor<R> J[PPL];
    const R h = (R)a.dt, hh = (R)(0.5 * a.dt), ngam = (R)(-a.gamma), g3 = (R)a.g3;
    const R kp = pot_factor<POT, R>();
    const R Fa = (R)a.Fa, Fb = (R)a.Fb;
    const uint32_t wave_cols = qs / PPL;
    auto col = [&](int j) { return (uint32_t)j * wave_cols + col0; };

    uint64_t n = n0;
    uint32_t k = (uint32_t)(n % a.spp);           // drive phase of step n
    if constexpr ((NOISE & NZ_JGRID) != 0) {
#pragma unroll
        for (int j = 0; j < PPL; ++j) {           // next kick not yet drawn; empty queue
            J[j].poff = (uint32_t)s[j].sP;
            J[j].pth = s[j].thP;
            J[j].gn = 0;
        }
    }

    while (n < n1) {
        const uint64_t wnext = ((n >> a.jw_log2) + 1u) << a.jw_log2;
        uint64_t wend = wnext < n1 ? wnext : n1;
        const uint32_t wdrawn = (uint32_t)(wend - n);   // steps the queues were drawn for
        uint32_t wlen = wdrawn;
        uint32_t cover = wdrawn;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            if constexpr ((NOISE & NZ_JGRID) != 0) {
                const uint32_t c = jg_window<R, NOISE>(a, path[j], wlen, s[j].kP, J[j], gq + col(j), qs);
                cover = c < cover ? c : cover;
            }
            if constexpr (queued_kicks<NOISE>()) {
                const uint32_t c = kick_window<R>(a, path[j], wlen, (uint32_t)s[j].sP, s[j].kP, kq + col(j), qs);
                cover = c < cover ? c : cover;
                const KickEntry<R> e = kq[col(j)];
                J[j].nP = e.off;
                J[j].zP = e.z;
                J[j].pP = kq + col(j) + qs;
            }
            if constexpr ((NOISE & NZ_DICH) != 0) {
                const uint32_t c = flip_window<R>(a, path[j], wlen, (uint32_t)s[j].sD, s[j].mD, s[j].d,
                                                  fq + col(j), qs);
                cover = c < cover ? c : cover;
                const uint32_t e = fq[col(j)];
                J[j].nD = e & ~INLINE_BIT;
                J[j].cD = qs;
            }
        }
        // A lane whose step holds more kicks than its queue (jump-adapted grid only):
        // that one step runs alone, drawing the kicks past the queue at the step.
        bool single = false;
        if constexpr (queued_kicks<NOISE>() || (NOISE & (NZ_DICH | NZ_JGRID)) != 0) {
            // A full kick or flip queue ends the window for the wave at the first
            // jump it does not hold (the minimum over the lanes; on the fixed grid at
            // least JCAP steps in), rounded down to a 16-step block boundary when one
            // lies after n.
            if (__any(cover < wlen)) {
                uint32_t wl = wlen;
                for (;;) {
                    const uint64_t b = __ballot(cover < wl);
                    if (b == 0) break;
                    // one lane's value, the same in every lane: keep it scalar, so
                    // that step counters and forcing-table reads stay wave-uniform
                    wl = __builtin_amdgcn_readfirstlane((uint32_t)__shfl(cover, __ffsll((long long)b) - 1));
                }
                if constexpr ((NOISE & NZ_JGRID) != 0) {
                    if (wl == 0) {
                        single = true;
                        wl = 1;
                    }
                }
                uint64_t we = n + wl;
                if (!single && (we & ~(uint64_t)15) > n) we &= ~(uint64_t)15;
                wend = we;
                wlen = (uint32_t)(we - n);
            }
        }
        uint32_t off = 0;

        // Generic single step (block-unaligned window heads and tails); INL: the
        // single step whose kicks overflow a queue.
        auto one_step = [&](auto inl) {
            constexpr bool INL = decltype(inl)::value;
            const R A0 = drive_at<R>(a, k);
            const R A1 = drive_at<R>(a, k + 1u);
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                R dxi = R(0);
                if constexpr ((NOISE & NZ_GAUSS) != 0) {
                    const U4 q = philox4x32_10((uint32_t)(n >> 4), path[j], a.point, TAG_GAUSS,
                                               a.key0, a.key1);
                    uint32_t u = pick(q, (uint32_t)(n >> 2) & 3u);
                    for (uint32_t t = 0; t < (uint32_t)(n & 3u); ++t) u = times6(u);
                    dxi = three_point<R>(u, g3);
                }
                if constexpr ((NOISE & NZ_NORMAL) != 0) {
                    // step n: words (2j, 2j+1) of block n/4, j = (n mod 4)/2; cos even, sin odd
                    const U4 q = philox4x32_10((uint32_t)(n >> 2), path[j], a.point, TAG_GAUSS,
                                               a.key0, a.key1);
                    const bool hi = ((n >> 1) & 1u) != 0;
                    R zc, zs;
                    normal_pair(hi ? q.z : q.x, hi ? q.w : q.y, zc, zs);
                    dxi = g3 * ((n & 1u) ? zs : zc);
                }
                full_step<R, DYN, POT, NOISE, INL>(a, path[j], s[j], J[j], gq + col(j), fq + col(j), qs,
                                                   wlen, off, k,
                                                   dxi, h, hh, ngam, kp, A0, A1, Fa, Fb);
            }
            k = (k + 1u == a.spp) ? 0u : k + 1u;
            ++n;
            ++off;
            if ((n & 15u) == 0u) {                   // fold at absolute multiples of 16 steps
#pragma unroll
                for (int j = 0; j < PPL; ++j) fold<POT, R>(s[j]);
            }
        };

        bool blocks = true;
        if constexpr ((NOISE & NZ_JGRID) != 0) {
            if (single) {
                one_step(std::true_type{});
                blocks = false;
            }
        }
        while (blocks && n < wend && (n & 15u) != 0u) one_step(std::false_type{});

        while (blocks && n + 16u <= wend) {
            U4 q[PPL];
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                if constexpr ((NOISE & NZ_GAUSS) != 0)
                    q[j] = philox4x32_10((uint32_t)(n >> 4), path[j], a.point, TAG_GAUSS, a.key0, a.key1);
                else
                    q[j] = U4{0u, 0u, 0u, 0u};
            }
            R A[17];                                  // forcing at steps n .. n+16
            const R *arow = reinterpret_cast<const R *>(a.tab) + k;   // k + 16 < spp + 16
#pragma unroll
            for (int t = 0; t < 17; ++t) A[t] = arow[t];
#pragma unroll
            for (int wd = 0; wd < 4; ++wd) {
                uint32_t u[PPL];
#pragma unroll
                for (int j = 0; j < PPL; ++j) u[j] = pick(q[j], (uint32_t)wd);
                R zn[PPL][4];                         // normal increments of steps 4 wd .. 4 wd + 3
                if constexpr ((NOISE & NZ_NORMAL) != 0) {
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        const U4 qn = philox4x32_10((uint32_t)(n >> 2) + (uint32_t)wd, path[j], a.point,
                                                    TAG_GAUSS, a.key0, a.key1);
                        normal_pair(qn.x, qn.y, zn[j][0], zn[j][1]);
                        normal_pair(qn.z, qn.w, zn[j][2], zn[j][3]);
                    }
                }
#pragma unroll
                for (int dg = 0; dg < 4; ++dg) {
                    const R A0 = A[4 * wd + dg], A1 = A[4 * wd + dg + 1];
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        R dxi = R(0);
                        if constexpr ((NOISE & NZ_GAUSS) != 0) {
                            dxi = three_point<R>(u[j], g3);
                            u[j] = times6(u[j]);   // next base-6 digit
                        }
                        if constexpr ((NOISE & NZ_NORMAL) != 0) dxi = g3 * zn[j][dg];
                        full_step<R, DYN, POT, NOISE>(a, path[j], s[j], J[j], gq + col(j),
                                                      fq + col(j), qs, wlen, off, k + (uint32_t)(4 * wd + dg), dxi, h, hh, ngam,
                                                      kp, A0, A1, Fa, Fb);
                    }
                    ++off;
                }
            }
            n += 16u;
            k = (k + 16u) % a.spp;
#pragma unroll
            for (int j = 0; j < PPL; ++j) fold<POT, R>(s[j]);   // x mod L at the block end
        }

        while (n < wend) one_step(std::false_type{});

        // Countdowns at the window end: the next jump lies at or beyond it.  A window
        // that ended early gives back the draws of the jumps queued past its end
        // (fixed grid); on the jump-adapted grid such kicks stay queued for the next.
        const bool early = wlen < wdrawn;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            if constexpr (queued_kicks<NOISE>()) {
                s[j].sP = (int32_t)(J[j].nP - wlen);
                if (early)
                    s[j].kP -= queued_beyond(kq + col(j), qs, wlen, wdrawn,
                                             [](const KickEntry<R> &e) { return e.off; });
            }
            if constexpr ((NOISE & NZ_JGRID) != 0) jg_carry<R>(J[j], gq + col(j), qs, wlen);
            if constexpr ((NOISE & NZ_DICH) != 0) {
                s[j].sD = (int32_t)(J[j].nD - wlen);
                if (early)
                    s[j].mD -= queued_beyond(fq + col(j), qs, wlen, wdrawn, [](uint32_t e) { return e; });
            }
        }
    }
    if constexpr ((NOISE & NZ_JGRID) != 0) {
        // every kick drawn lay before the last window's end and has been applied
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            s[j].sP = (int32_t)J[j].poff;
            s[j].thP = J[j].pth;
        }
    }
}

// Ensemble integration kernel: lane layout path = (blockIdx.x * PPL + j) * blockDim.x + tid.
template <typename R, int DYN, int POT, int NOISE, int PPL>
__global__ void __launch_bounds__(512) k_advance(const KArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t base = blockIdx.x * PPL * blockDim.x + threadIdx.x;
    if (base >= a.p.n_paths) return;
    uint32_t path[PPL];
    bool valid[PPL];
    Path<R> s[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const uint64_t p = (uint64_t)base + (uint64_t)j * blockDim.x;
        valid[j] = p < a.p.n_paths;
        path[j] = valid[j] ? (uint32_t)p : base;
        load_path<R, POT, NOISE>(a, path[j], s[j]);
    }
    advance_range<R, DYN, POT, NOISE, PPL>(a.p, path, s, a.n0, a.n1, smem, PPL * blockDim.x, threadIdx.x);
#pragma unroll
    for (int j = 0; j < PPL; ++j)
        if (valid[j]) store_path<R, POT, NOISE>(a, path[j], s[j]);
}

// ---------------------------------------------------------------------------
// Initial conditions (tag 2), computed in FP64 and stored in the path precision:
// x ~ U[x0_lo, x0_hi) folded, v ~ U[v0_lo, v0_hi), Poisson countdown
// floor(E / (lambda dt)), dichotomous state opposite to a stationary draw with
// countdown 0 (the first step flips into the stationary state).
// ---------------------------------------------------------------------------
template <typename R, int DYN, int POT, int NOISE>
__device__ __forceinline__ Path<R> init_path(const PointConst &a, uint32_t p)
{
    const U4 q = philox4x32_10(0u, p, a.point, TAG_INIT, a.key0, a.key1);
    const double L = period<POT>();
    double x = a.x0_lo + a.x0_w * ((double)q.x * 0x1p-32);
    const double kf = floor(x / L);
    x = x - kf * L;
    Path<R> s;
    s.w = (int32_t)kf;
    s.x = (R)x;
    if (s.x >= (R)L) { s.x -= (R)L; s.w += 1; }   // rounding to the path precision may reach L
    s.v = (DYN == DYN_INERTIAL) ? (R)(a.v0_lo + a.v0_w * ((double)q.y * 0x1p-32)) : R(0);
    s.sP = 0; s.kP = 0u; s.sD = 0; s.mD = 0u; s.d = 0; s.thP = 0.0;
    if constexpr ((NOISE & NZ_JGRID) != 0) {
        const double T = expo64(q.z) / a.lam_dt;          // first kick time in steps
        const double Tf = floor(T);
        s.sP = (int32_t)Tf;
        s.thP = T - Tf;
    } else if constexpr ((NOISE & NZ_POISSON) != 0) {
        s.sP = (int32_t)floor(expo64(q.z) / a.lam_dt);
    }
    if constexpr ((NOISE & NZ_DICH) != 0) {
        const int32_t dstar = ((double)q.w * 0x1p-32 < a.p_hi) ? 1 : 0;
        s.d = 1 - dstar;
    }
    return s;
}

template <typename R, int DYN, int POT, int NOISE>
__global__ void __launch_bounds__(256) k_init(const KArgs a)
{
    const uint64_t p64 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p64 >= a.p.n_paths) return;
    const uint32_t p = (uint32_t)p64;
    const Path<R> s = init_path<R, DYN, POT, NOISE>(a.p, p);
    arr<R>(a.x)[p] = s.x;
    a.w[p] = s.w;
    arr<R>(a.v)[p] = s.v;
    if constexpr ((NOISE & NZ_POISSON) != 0) { a.sP[p] = s.sP; a.kP[p] = s.kP; }
    if constexpr ((NOISE & NZ_JGRID) != 0) a.thP[p] = s.thP;
    if constexpr ((NOISE & NZ_DICH) != 0) { a.d[p] = s.d; a.sD[p] = s.sD; a.mD[p] = s.mD; }
    if (a.snapshot) { arr<R>(a.xi)[p] = s.x; a.wi[p] = s.w; }
    if (a.lev) { a.lev[p] = (int32_t)a.sc_J; a.kA[p] = 0u; }   // step control starts at the smallest step
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
    bool have = p < a.p.n_paths;
    if (have) {
        const double dx = (double)(a.w[p] - a.wi[p]) * L +
                          ((double)arr<R>(a.x)[p] - (double)arr<R>(a.xi)[p]);
        vp = dx / a.t_window;
        a.vp[p] = vp;
    }
    const Partial part = wave_partial(vp, have);
    const uint64_t chunk = p >> 6;
    if ((threadIdx.x & 63u) == 0u && (chunk << 6) < a.p.n_paths) {
        a.part[chunk] = part;
    }
}

// ---------------------------------------------------------------------------
// Export of paths [n0, n0 + n1) (n0/n1 reused as first/count) to FP64 arrays and
// to lossless per-path records (every field widened exactly).  flags (launch.hpp):
// READ_VP the per-path velocity exists, READ_SNAP the window snapshot exists
// (before the window start the record's window fields are 0, not the workspace's
// unwritten contents).
// ---------------------------------------------------------------------------

template <typename R, int POT>
__global__ void __launch_bounds__(256) k_read(const KArgs a, double *xo, double *vo, int64_t *no,
                                              double *vpo, int flags, bm_path *so)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n1) return;
    const uint64_t p = a.n0 + i;
    const double L = period<POT>();
    if (xo) xo[i] = (double)a.w[p] * L + (double)arr<R>(a.x)[p];
    if (vo) vo[i] = (double)arr<R>(a.v)[p];
    const int64_t nz[5] = {a.sP ? a.sP[p] : 0, a.kP ? (int64_t)a.kP[p] : 0, a.sD ? a.sD[p] : 0,
                           a.mD ? (int64_t)a.mD[p] : 0, a.d ? a.d[p] : 0};
    if (no) {
        for (int j = 0; j < 5; ++j) no[5 * i + j] = nz[j];
    }
    if (vpo && (flags & READ_VP)) {
        const double dx = (double)(a.w[p] - a.wi[p]) * L +
                          ((double)arr<R>(a.x)[p] - (double)arr<R>(a.xi)[p]);
        vpo[i] = dx / a.t_window;
    }
    if (so) {
        bm_path r;
        r.periods = a.w[p];
        r.x = (double)arr<R>(a.x)[p];
        r.v = (double)arr<R>(a.v)[p];
        const bool snap = (flags & READ_SNAP) != 0;
        r.periods_window = snap ? a.wi[p] : 0;
        r.x_window = snap ? (double)arr<R>(a.xi)[p] : 0.0;
        r.kick_frac = a.thP ? a.thP[p] : 0.0;
        for (int j = 0; j < 5; ++j) r.noise[j] = nz[j];
        r.step_level = a.lev ? a.lev[p] : 0;
        r.steps_taken = a.kA ? (int64_t)a.kA[p] : 0;
        so[i] = r;
    }
}

// ---------------------------------------------------------------------------
// Import of records into paths [n0, n0 + n1): the inverse of k_read's records.
// Out-of-range values are clamped so that the path kernels' assumptions (countdowns
// and counts in range, state 0/1, a kick fraction in [0, 1)) hold whatever the input.
// snap: 0 leave the window snapshot, 1 set it to the written position, 2 take it
// from the record.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t clamp_i32(int64_t v, int64_t lo, int64_t hi)
{
    return (int32_t)(v < lo ? lo : (v > hi ? hi : v));
}

template <typename R, int POT>
__global__ void __launch_bounds__(256) k_write(const KArgs a, const bm_path *si, uint32_t snap)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n1) return;
    const uint64_t p = a.n0 + i;
    const bm_path r = si[i];
    const int32_t w = clamp_i32(r.periods, INT32_MIN, INT32_MAX);
    arr<R>(a.x)[p] = (R)r.x;
    a.w[p] = w;
    arr<R>(a.v)[p] = (R)r.v;
    if (snap == 1u) {
        arr<R>(a.xi)[p] = (R)r.x;
        a.wi[p] = w;
    } else if (snap == 2u) {
        arr<R>(a.xi)[p] = (R)r.x_window;
        a.wi[p] = clamp_i32(r.periods_window, INT32_MIN, INT32_MAX);
    }
    if (a.sP) a.sP[p] = clamp_i32(r.noise[0], 0, INT32_MAX);
    if (a.kP) a.kP[p] = (uint32_t)(r.noise[1] < 0 ? 0 : (r.noise[1] > (int64_t)UINT32_MAX ? UINT32_MAX : r.noise[1]));
    if (a.thP) a.thP[p] = (r.kick_frac >= 0.0 && r.kick_frac < 1.0) ? r.kick_frac : 0.0;
    if (a.sD) a.sD[p] = clamp_i32(r.noise[2], 0, INT32_MAX);
    if (a.mD) a.mD[p] = (uint32_t)(r.noise[3] < 0 ? 0 : (r.noise[3] > (int64_t)UINT32_MAX ? UINT32_MAX : r.noise[3]));
    if (a.d) a.d[p] = r.noise[4] != 0 ? 1 : 0;
    if (a.lev) {
        a.lev[p] = clamp_i32(r.step_level, 0, (int64_t)a.sc_J);
        a.kA[p] = (uint32_t)(r.steps_taken < 0 ? 0 : (r.steps_taken > (int64_t)UINT32_MAX ? UINT32_MAX : r.steps_taken));
    }
}

// ---------------------------------------------------------------------------
// eq. (19): histogram of the folded positions y = x mod L in n_bins equal bins of
// [0, L), bin = floor(y n_bins / L), computed in FP64; counts are added to `hist`
// (integer atomics: the result does not depend on their order).
// ---------------------------------------------------------------------------
template <typename R, int POT>
__global__ void __launch_bounds__(256) k_density(const KArgs a, uint32_t n_bins, unsigned long long *hist)
{
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.p.n_paths) return;
    const double L = period<POT>();
    const double x = (double)arr<R>(a.x)[p];
    const double y = x - L * floor(x / L);
    const double t = y * (double)n_bins / L;
    uint32_t b = t >= (double)n_bins ? n_bins - 1u : (uint32_t)t;   // y rounded up to L
    if (!(t >= 0.0)) return;                                          // non-finite position
    atomicAdd(&hist[b], 1ull);
}

} // namespace bm
