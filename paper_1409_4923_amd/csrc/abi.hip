// abi.hip -- libbmotor C ABI: argument validation, workspace layout, launch
// sequencing, and the fixed-order FP64 ensemble reduction (eq. 31).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bmotor.h"
#include "common.hpp"
#include "launch.hpp"
#include "paths.hpp"
#include "reduce.hpp"
#include "host.hpp"

using namespace bm;
using namespace bm::host;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
namespace bm {
namespace host {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return BM_OK;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(BM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const char *last_error_text() { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Validation and derived constants
// ---------------------------------------------------------------------------
static bool fin(double v) { return std::isfinite(v); }

// Largest countdown an exponential variate can produce: E = -ln(1 - phi) <= 32 ln 2.
static constexpr double E_MAX = 22.18070977791825;

int validate(const bm_model *m, const bm_run *r)
{
    if (!m || !r) return fail(BM_ERR_INVALID_ARG, "model and run must not be NULL");
    if (m->size != sizeof(bm_model)) return fail(BM_ERR_INVALID_ARG, "bm_model.size mismatch");
    if (r->size != sizeof(bm_run)) return fail(BM_ERR_INVALID_ARG, "bm_run.size mismatch");
    if (m->dyn > BM_INERTIAL) return fail(BM_ERR_INVALID_ARG, "unknown dynamics %u", m->dyn);
    if (m->pot > BM_POT_FREE) return fail(BM_ERR_INVALID_ARG, "unknown potential %u", m->pot);
    if (m->noise & ~31u) return fail(BM_ERR_INVALID_ARG, "unknown noise bits 0x%x", m->noise);
    if ((m->noise & BM_NOISE_JUMP_GRID) && !(m->noise & BM_NOISE_POISSON))
        return fail(BM_ERR_INVALID_ARG, "BM_NOISE_JUMP_GRID needs BM_NOISE_POISSON");
    if ((m->noise & BM_NOISE_GAUSS) && (m->noise & BM_NOISE_NORMAL))
        return fail(BM_ERR_INVALID_ARG, "BM_NOISE_GAUSS and BM_NOISE_NORMAL are alternatives");
    if (r->prec > BM_F32) return fail(BM_ERR_INVALID_ARG, "unknown precision %u", r->prec);
    if (m->dyn == BM_INERTIAL && !(fin(m->gamma) && m->gamma > 0))
        return fail(BM_ERR_INVALID_ARG, "gamma must be finite and > 0");
    if (!fin(m->drive_amp) || !fin(m->force)) return fail(BM_ERR_INVALID_ARG, "drive/force not finite");
    double dt;
    if (r->steps_per_period > 0) {
        if (!(fin(m->drive_omega) && m->drive_omega > 0))
            return fail(BM_ERR_INVALID_ARG, "drive_omega must be > 0 when steps_per_period > 0");
        if (r->dt != 0.0) return fail(BM_ERR_INVALID_ARG, "dt must be 0 when steps_per_period > 0");
        dt = (2.0 * M_PI / m->drive_omega) / (double)r->steps_per_period;
    } else {
        if (m->drive_amp != 0.0)
            return fail(BM_ERR_INVALID_ARG, "a periodic drive needs steps_per_period > 0");
        if (!(fin(r->dt) && r->dt > 0)) return fail(BM_ERR_INVALID_ARG, "dt must be finite and > 0");
        dt = r->dt;
    }
    if (m->noise & (BM_NOISE_GAUSS | BM_NOISE_NORMAL))
        if (!(fin(m->D) && m->D >= 0)) return fail(BM_ERR_INVALID_ARG, "D must be finite and >= 0");
    if (m->noise & BM_NOISE_POISSON) {
        if (!(fin(m->shot_rate) && m->shot_rate > 0))
            return fail(BM_ERR_INVALID_ARG, "shot_rate must be finite and > 0");
        if (!(fin(m->shot_mean) && m->shot_mean >= 0))
            return fail(BM_ERR_INVALID_ARG, "shot_mean must be finite and >= 0");
        if (E_MAX / (m->shot_rate * dt) >= 2147483000.0)
            return fail(BM_ERR_UNSUPPORTED, "shot_rate*dt too small: waiting times overflow int32");
        if ((m->noise & BM_NOISE_JUMP_GRID) && m->shot_rate * dt > 16.0)
            return fail(BM_ERR_UNSUPPORTED, "jump-adapted grid needs shot_rate*dt <= 16");
    }
    if (m->noise & BM_NOISE_DICH) {
        if (!(fin(m->dich_Fa) && fin(m->dich_Fb) && m->dich_Fa >= 0 && m->dich_Fb >= 0))
            return fail(BM_ERR_INVALID_ARG, "dichotomous levels must be finite and >= 0");
        if (!(fin(m->dich_mua) && fin(m->dich_mub) && m->dich_mua > 0 && m->dich_mub > 0))
            return fail(BM_ERR_INVALID_ARG, "dichotomous rates must be finite and > 0");
        if (E_MAX / (std::fmin(m->dich_mua, m->dich_mub) * dt) >= 2147483000.0)
            return fail(BM_ERR_UNSUPPORTED, "dichotomous rate*dt too small: dwell overflows int32");
    }
    if (r->n_paths < 1 || r->n_paths > 0xFFFFFFFFull)
        return fail(BM_ERR_INVALID_ARG, "n_paths must be in [1, 2^32 - 1]");
    if (!(fin(r->x0_lo) && fin(r->x0_hi) && r->x0_lo <= r->x0_hi))
        return fail(BM_ERR_INVALID_ARG, "need finite x0_lo <= x0_hi");
    if (!(fin(r->v0_lo) && fin(r->v0_hi) && r->v0_lo <= r->v0_hi))
        return fail(BM_ERR_INVALID_ARG, "need finite v0_lo <= v0_hi");
    if (r->window_start > 0xFFFFFFFFull) return fail(BM_ERR_INVALID_ARG, "window_start >= 2^32");
    if (!(fin(r->step_tol) && r->step_tol >= 0)) return fail(BM_ERR_INVALID_ARG, "step_tol must be finite and >= 0");
    if (r->pad != 0) return fail(BM_ERR_INVALID_ARG, "bm_run.pad must be 0");
    if (r->step_tol > 0) {
        if (r->max_halvings < 1 || r->max_halvings > SC_MAX_HALVINGS)
            return fail(BM_ERR_INVALID_ARG, "max_halvings must be in [1, %u] with step_tol > 0", SC_MAX_HALVINGS);
        if (m->noise & (BM_NOISE_NORMAL | BM_NOISE_JUMP_GRID))
            return fail(BM_ERR_UNSUPPORTED, "step control runs the three-point scheme with jumps on the dt grid");
    } else if (r->max_halvings != 0) {
        return fail(BM_ERR_INVALID_ARG, "max_halvings must be 0 without step control (step_tol = 0)");
    }
    return BM_OK;
}

// Step-size control on chi is requested.
static bool step_control(const bm_run *r) { return r->step_tol > 0; }

double step_of(const bm_model *m, const bm_run *r)
{
    return r->steps_per_period > 0 ? (2.0 * M_PI / m->drive_omega) / (double)r->steps_per_period
                                   : r->dt;
}

// Entries of the forcing table: one drive period plus one block of 16 steps; under
// step control one period on the grid of the smallest step (2^max_halvings entries
// per step of dt) plus 16.
size_t table_entries(const bm_run *r)
{
    const size_t per = r->steps_per_period ? r->steps_per_period : 1u;
    return (step_control(r) ? per << r->max_halvings : per) + 16;
}

// ---------------------------------------------------------------------------
// Workspace layout (structure of arrays, each 256-byte aligned)
// ---------------------------------------------------------------------------
struct Layout {
    size_t x, w, v, xi, wi, sP, kP, thP, sD, mD, d, lev, kA, vp, part, tab, total;
};

static size_t up(size_t v) { return (v + 255) & ~(size_t)255; }

static Layout layout(const bm_model *m, const bm_run *r)
{
    const size_t N = r->n_paths;
    const size_t rs = r->prec == BM_F32 ? 4 : 8;
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += up(bytes); return at; };
    L.x = take(N * rs);
    L.w = take(N * 4);
    L.v = take(N * rs);
    L.xi = take(N * rs);
    L.wi = take(N * 4);
    L.sP = take(N * 4);
    L.kP = take(N * 4);
    L.thP = (m->noise & BM_NOISE_JUMP_GRID) ? take(N * 8) : 0;
    L.sD = take(N * 4);
    L.mD = take(N * 4);
    L.d = take(N * 4);
    L.lev = step_control(r) ? take(N * 4) : 0;
    L.kA = step_control(r) ? take(N * 4) : 0;
    L.vp = take(N * 8);
    L.part = take(((N + 63) / 64) * sizeof(Partial));
    L.tab = take(table_entries(r) * rs);
    L.total = o;
    return L;
}

extern "C" int bm_ensemble_workspace_size(const bm_model *model, const bm_run *run, size_t *bytes)
{
    int rc = validate(model, run);
    if (rc) return rc;
    if (!bytes) return fail(BM_ERR_INVALID_ARG, "bytes must not be NULL");
    *bytes = layout(model, run).total;
    return ok();
}

// ---------------------------------------------------------------------------
// Device check: the kernels are built for gfx950 only.
// ---------------------------------------------------------------------------
int check_device(int *dev_out)
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(BM_ERR_DEVICE, "no HIP device available");
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BM_ERR_DEVICE, "device %d is %s; libbmotor is built for gfx950 only", dev,
                    prop.gcnArchName);
    *dev_out = dev;
    return BM_OK;
}

} // namespace host
} // namespace bm

extern "C" uint32_t bm_abi_version(void) { return BM_ABI_VERSION; }
extern "C" const char *bm_last_error(void) { return last_error_text(); }

// ---------------------------------------------------------------------------
// Ensemble handle
// ---------------------------------------------------------------------------
struct bm_ensemble {
    bm_model model;
    bm_run run;
    Layout lay;
    char *ws;
    hipStream_t stream;
    KArgs k;                 // template of the kernel arguments
    uint64_t n_done;
    uint32_t ppl, block;
    std::vector<double> tab64;
    std::vector<float> tab32;
};

namespace bm {
namespace host {

// Constant part of the forcing without a drive: tilt - Poisson bias + potential offset.
double forcing_constant(const bm_model *m)
{
    const double bias = (m->noise & BM_NOISE_POISSON) ? m->shot_rate * m->shot_mean : 0.0;
    const double pot_off = m->pot == BM_POT_RATCHET ? -M_PI : 0.0;
    return (m->force - bias) + pot_off;
}

// Table of the constant-within-step forcing per drive phase, in FP64:
// a cos(2 pi k / spp) + F - lambda zeta + potential offset, k = 0 .. spp-1,
// followed by 16 entries repeating the start (one block of steps).
void forcing_table(const bm_model *m, const bm_run *r, std::vector<double> &tab)
{
    const uint32_t spp = r->steps_per_period;
    const size_t n = table_entries(r);
    const double c = forcing_constant(m);
    tab.assign(n, c);
    if (!spp) return;
    // the phase grid: spp entries per period, or spp 2^max_halvings under step control
    const uint64_t period = step_control(r) ? (uint64_t)spp << r->max_halvings : spp;
    for (size_t j = 0; j < n; ++j) {
        const uint64_t i = j % period;
        tab[j] = m->drive_amp * std::cos(2.0 * M_PI * (double)i / (double)period) + c;
    }
}


// Per-point constants shared by the ensemble and scan kernels.
PointConst point_const(const bm_model *m, const bm_run *r, const void *d_tab)
{
    PointConst k;
    std::memset(&k, 0, sizeof k);
    k.tab = d_tab;
    k.n_paths = (uint32_t)r->n_paths;
    k.n_steps = r->n_steps;
    k.n_window = r->window_start;
    k.spp = r->steps_per_period ? r->steps_per_period : 1u;
    k.point = r->point_id;
    k.key0 = (uint32_t)r->seed;
    k.key1 = (uint32_t)(r->seed >> 32);
    const double h = step_of(m, r);
    k.dt = h;
    k.gamma = m->dyn == BM_INERTIAL ? m->gamma : 0.0;
    if (m->noise & BM_NOISE_GAUSS) {
        const double G = m->dyn == BM_INERTIAL ? std::sqrt(2.0 * m->gamma * m->D) : std::sqrt(2.0 * m->D);
        k.g3 = G * std::sqrt(3.0 * h);
    }
    if (m->noise & BM_NOISE_NORMAL) {           // scale of a standard normal: G sqrt(dt)
        const double G = m->dyn == BM_INERTIAL ? std::sqrt(2.0 * m->gamma * m->D) : std::sqrt(2.0 * m->D);
        k.g3 = G * std::sqrt(h);
    }
    // FP32 countdown estimates: error < 3e-7 / (rate dt) + 4.2e-7 X (rounding of
    // 1 - phi, v_log_f32 near 1, the scale); the tolerance is about 7x / 10x that.
    const double LN2 = 0.69314718055994530942;
    k.tol1 = 4e-6f;
    // Jump window: the longest 16 2^j <= 1024 steps in which a lane expects at most
    // about four jumps (the fastest rate of the model decides).
    double rate_dt = 0.0;
    if (m->noise & BM_NOISE_POISSON) rate_dt = std::fmax(rate_dt, m->shot_rate * h);
    if (m->noise & BM_NOISE_DICH) rate_dt = std::fmax(rate_dt, std::fmax(m->dich_mua, m->dich_mub) * h);
    k.jw_log2 = JW_LOG2_MAX;
    while (k.jw_log2 > 4 && rate_dt * (double)(1u << k.jw_log2) > 4.5) --k.jw_log2;
    if (m->noise & BM_NOISE_POISSON) {
        k.lam_dt = m->shot_rate * h;
        k.zeta = m->shot_mean;
        k.c_lam = (float)(LN2 / k.lam_dt);
        k.tol0_lam = (float)(2e-6 / k.lam_dt + 1e-6);
        k.zeta_ln2 = (float)(-m->shot_mean * LN2);
    }
    if (m->noise & BM_NOISE_DICH) {
        k.Fa = m->dich_Fa;
        k.Fb = m->dich_Fb;
        k.mua_dt = m->dich_mua * h;
        k.mub_dt = m->dich_mub * h;
        k.p_hi = m->dich_mua / (m->dich_mua + m->dich_mub);
        k.c_mua = (float)(LN2 / k.mua_dt);
        k.c_mub = (float)(LN2 / k.mub_dt);
        k.tol0_mua = (float)(2e-6 / k.mua_dt + 1e-6);
        k.tol0_mub = (float)(2e-6 / k.mub_dt + 1e-6);
    }
    k.inv_spp = (float)(1.0 / (double)k.spp);
    k.drive_a = r->steps_per_period ? m->drive_amp : 0.0;
    k.drive_c = forcing_constant(m);
    k.x0_lo = r->x0_lo; k.x0_w = r->x0_hi - r->x0_lo;
    k.v0_lo = r->v0_lo; k.v0_w = r->v0_hi - r->v0_lo;
    return k;
}

} // namespace host
} // namespace bm

static void fill_kargs(bm_ensemble *e)
{
    KArgs &k = e->k;
    std::memset(&k, 0, sizeof k);
    char *b = e->ws;
    const Layout &L = e->lay;
    k.x = b + L.x; k.w = (int32_t *)(b + L.w); k.v = b + L.v; k.xi = b + L.xi;
    k.wi = (int32_t *)(b + L.wi);
    k.sP = (int32_t *)(b + L.sP); k.kP = (uint32_t *)(b + L.kP);
    k.thP = (e->model.noise & BM_NOISE_JUMP_GRID) ? (double *)(b + L.thP) : nullptr;
    k.sD = (int32_t *)(b + L.sD); k.mD = (uint32_t *)(b + L.mD); k.d = (int32_t *)(b + L.d);
    k.vp = (double *)(b + L.vp);
    k.part = (Partial *)(b + L.part);
    k.p = point_const(&e->model, &e->run, b + L.tab);
    k.noise = e->model.noise;
    if (step_control(&e->run)) {
        k.lev = (int32_t *)(b + L.lev);
        k.kA = (uint32_t *)(b + L.kA);
        k.sc_J = e->run.max_halvings;
        k.sc_tol = e->run.step_tol;
        const bm_model *m = &e->model;
        const double G = !(m->noise & BM_NOISE_GAUSS) ? 0.0
                        : m->dyn == BM_INERTIAL ? std::sqrt(2.0 * m->gamma * m->D) : std::sqrt(2.0 * m->D);
        for (uint32_t l = 0; l <= k.sc_J; ++l) {
            k.sc_h[l] = std::ldexp(k.p.dt, -(int)l);
            k.sc_g3[l] = G * std::sqrt(3.0 * k.sc_h[l]);
        }
    }
}

static void fill_table(bm_ensemble *e)
{
    forcing_table(&e->model, &e->run, e->tab64);
    e->tab32.assign(e->tab64.begin(), e->tab64.end());
}

// Creates the handle and uploads the drive table; `init` enqueues the initial
// conditions, otherwise the workspace already holds the state after steps_done.
static int open_ensemble(const bm_model *model, const bm_run *run, void *d_ws, size_t ws_bytes, void *stream,
                         bool init, uint64_t steps_done, bm_ensemble **out)
{
    int rc = validate(model, run);
    if (rc) return rc;
    if (!out) return fail(BM_ERR_INVALID_ARG, "out must not be NULL");
    if (steps_done > 0xFFFFFFFFull) return fail(BM_ERR_UNSUPPORTED, "total step count must stay below 2^32");
    const Layout L = layout(model, run);
    if (!d_ws || ((uintptr_t)d_ws & 255u)) return fail(BM_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < L.total) return fail(BM_ERR_WORKSPACE, "workspace %zu B < %zu B needed", ws_bytes, L.total);
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;

    bm_ensemble *e = new (std::nothrow) bm_ensemble();
    if (!e) return fail(BM_ERR_INVALID_ARG, "out of host memory");
    e->model = *model;
    e->run = *run;
    e->lay = L;
    e->ws = (char *)d_ws;
    e->stream = (hipStream_t)stream;
    e->n_done = steps_done;
    const bm_tune dt = default_tune(model->dyn, model->pot, model->noise, run->prec);
    e->ppl = dt.paths_per_lane;
    e->block = dt.block;
    fill_kargs(e);
    fill_table(e);

    const bool f32 = run->prec == BM_F32;
    const void *src = f32 ? (const void *)e->tab32.data() : (const void *)e->tab64.data();
    const size_t tb = (f32 ? 4 : 8) * e->tab64.size();
    // The table is read from host memory owned by the handle: wait for the copy so
    // that the handle can be destroyed at any time after this returns.
    hipError_t he = hipMemcpyAsync((char *)d_ws + L.tab, src, tb, hipMemcpyHostToDevice, e->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
    if (he != hipSuccess) { delete e; return hip_fail(he, "drive table upload"); }

    if (init) {
        KArgs k = e->k;
        k.snapshot = run->window_start == 0 ? 1u : 0u;
        const int pot = (int)model->pot, noise = (int)model->noise;
        if (f32)
            he = model->dyn == BM_INERTIAL ? launch_init_f32_in(pot, noise, k, e->stream)
                                           : launch_init_f32_od(pot, noise, k, e->stream);
        else
            he = model->dyn == BM_INERTIAL ? launch_init_f64_in(pot, noise, k, e->stream)
                                           : launch_init_f64_od(pot, noise, k, e->stream);
        if (he != hipSuccess) { delete e; return hip_fail(he, "init kernel launch"); }
    }
    *out = e;
    return ok();
}

extern "C" int bm_ensemble_create(const bm_model *model, const bm_run *run, void *d_ws,
                                  size_t ws_bytes, void *stream, bm_ensemble **out)
{
    return open_ensemble(model, run, d_ws, ws_bytes, stream, true, 0, out);
}

extern "C" int bm_ensemble_attach(const bm_model *model, const bm_run *run, void *d_ws, size_t ws_bytes,
                                  uint64_t steps_done, void *stream, bm_ensemble **out)
{
    return open_ensemble(model, run, d_ws, ws_bytes, stream, false, steps_done, out);
}

extern "C" int bm_ensemble_destroy(bm_ensemble *e)
{
    if (!e) return fail(BM_ERR_INVALID_ARG, "NULL handle");
    delete e;
    return ok();
}

extern "C" int bm_ensemble_set_tune(bm_ensemble *e, const bm_tune *t)
{
    if (!e) return fail(BM_ERR_INVALID_ARG, "NULL handle");
    const bm_tune use = t ? *t : default_tune(e->model.dyn, e->model.pot, e->model.noise, e->run.prec);
    // the step-control kernel draws its jumps inline: no LDS queues to fit
    const uint32_t queued = step_control(&e->run) ? (e->model.noise & BM_NOISE_GAUSS) : e->model.noise;
    int rc = check_tune(&use, queued, e->run.prec);
    if (rc) return rc;
    if (t && step_control(&e->run) && use.paths_per_lane != 1)
        return fail(BM_ERR_UNSUPPORTED, "step control runs one path per lane");
    e->ppl = use.paths_per_lane;
    e->block = use.block;
    return ok();
}

extern "C" int bm_ensemble_steps(const bm_ensemble *e, uint64_t *n_done)
{
    if (!e || !n_done) return fail(BM_ERR_INVALID_ARG, "NULL argument");
    *n_done = e->n_done;
    return ok();
}

static hipError_t launch_advance(const bm_ensemble *e, const KArgs &k)
{
    const int pot = (int)e->model.pot, noise = (int)e->model.noise;
    const int ppl = (int)e->ppl, blk = (int)e->block;
    if (step_control(&e->run)) {                   // one path per lane, a wave per control group
        if (e->run.prec == BM_F32)
            return e->model.dyn == BM_INERTIAL ? launch_advance_sc_f32_in(pot, blk, k, e->stream)
                                               : launch_advance_sc_f32_od(pot, blk, k, e->stream);
        return e->model.dyn == BM_INERTIAL ? launch_advance_sc_f64_in(pot, blk, k, e->stream)
                                           : launch_advance_sc_f64_od(pot, blk, k, e->stream);
    }
    if (e->run.prec == BM_F32)
        return e->model.dyn == BM_INERTIAL ? launch_advance_f32_in(pot, noise, ppl, blk, k, e->stream)
                                           : launch_advance_f32_od(pot, noise, ppl, blk, k, e->stream);
    return e->model.dyn == BM_INERTIAL ? launch_advance_f64_in(pot, noise, 1, blk, k, e->stream)
                                       : launch_advance_f64_od(pot, noise, 1, blk, k, e->stream);
}

extern "C" int bm_integrate(bm_ensemble *e, uint64_t n_steps)
{
    if (!e) return fail(BM_ERR_INVALID_ARG, "NULL handle");
    if (n_steps > 0xFFFFFFFFull - e->n_done)
        return fail(BM_ERR_UNSUPPORTED, "total step count must stay below 2^32");
    uint64_t n = e->n_done;
    const uint64_t end = e->n_done + n_steps;
    while (n < end) {
        uint64_t stop = end;
        const uint64_t nw = e->run.window_start;
        if (n < nw && nw < stop) stop = nw;       // split so the snapshot falls on a launch end
        KArgs k = e->k;
        k.n0 = n;
        k.n1 = stop;
        k.snapshot = (stop == nw && nw > 0) ? 1u : 0u;
        hipError_t he = launch_advance(e, k);
        if (he != hipSuccess) return hip_fail(he, "integration kernel launch");
        n = stop;
        e->n_done = n;
    }
    return ok();
}

__global__ void __launch_bounds__(256) k_reduce_final(const Partial *part, uint64_t n_chunks, double tw,
                                                      bm_stats *out)
{
    reduce_chunks(part, n_chunks, tw, out);
}

static void set_window(bm_ensemble *e, KArgs &k)
{
    k.t_window = (double)(e->n_done - e->run.window_start) * k.p.dt;
}

extern "C" int bm_reduce(bm_ensemble *e, bm_stats *d_out)
{
    if (!e) return fail(BM_ERR_INVALID_ARG, "NULL handle");
    if (!d_out) return fail(BM_ERR_INVALID_ARG, "d_out must not be NULL");
    if (e->n_done <= e->run.window_start)
        return fail(BM_ERR_STATE, "window incomplete: %llu steps done, window starts at %llu",
                    (unsigned long long)e->n_done, (unsigned long long)e->run.window_start);
    KArgs k = e->k;
    set_window(e, k);
    const int pot = (int)e->model.pot;
    hipError_t he = e->run.prec == BM_F32 ? launch_velocity_f32(pot, k, e->stream)
                                          : launch_velocity_f64(pot, k, e->stream);
    if (he != hipSuccess) return hip_fail(he, "velocity kernel launch");
    const uint64_t chunks = (e->run.n_paths + 63) / 64;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, e->stream, k.part, chunks, k.t_window, d_out);
    he = hipGetLastError();
    if (he != hipSuccess) return hip_fail(he, "reduction kernel launch");
    return ok();
}

// Range of paths [first, first + count) inside the ensemble and the kernel arguments
// restricted to the arrays its model has.
static int path_range(const bm_ensemble *e, uint64_t first, uint64_t count, KArgs &k)
{
    if (first > e->run.n_paths || count > e->run.n_paths - first)
        return fail(BM_ERR_INVALID_ARG, "path range [%llu, +%llu) outside the ensemble",
                    (unsigned long long)first, (unsigned long long)count);
    k = e->k;
    k.n0 = first;
    k.n1 = count;
    const uint32_t noise = e->model.noise;
    if (!(noise & BM_NOISE_POISSON)) { k.sP = nullptr; k.kP = nullptr; }
    if (!(noise & BM_NOISE_DICH)) { k.sD = nullptr; k.mD = nullptr; k.d = nullptr; }
    return BM_OK;
}

extern "C" int bm_read_paths(bm_ensemble *e, uint64_t first, uint64_t count, double *d_x, double *d_v,
                             int64_t *d_noise, double *d_vp, bm_path *d_state)
{
    if (!e) return fail(BM_ERR_INVALID_ARG, "NULL handle");
    KArgs k;
    int rc = path_range(e, first, count, k);
    if (rc) return rc;
    if ((uintptr_t)d_state & 7u) return fail(BM_ERR_INVALID_ARG, "d_state must be 8-byte aligned");
    if (count == 0) return ok();
    const bool with_vp = e->n_done > e->run.window_start;
    const int flags = (with_vp ? READ_VP : 0) | (e->n_done >= e->run.window_start ? READ_SNAP : 0);
    if (with_vp) set_window(e, k);
    const int pot = (int)e->model.pot;
    hipError_t he = e->run.prec == BM_F32
                         ? launch_read_f32(pot, k, d_x, d_v, d_noise, d_vp, flags, d_state, e->stream)
                         : launch_read_f64(pot, k, d_x, d_v, d_noise, d_vp, flags, d_state, e->stream);
    if (he != hipSuccess) return hip_fail(he, "export kernel launch");
    return ok();
}

extern "C" int bm_write_paths(bm_ensemble *e, uint64_t first, uint64_t count, const bm_path *d_state)
{
    if (!e) return fail(BM_ERR_INVALID_ARG, "NULL handle");
    KArgs k;
    int rc = path_range(e, first, count, k);
    if (rc) return rc;
    if (!d_state || ((uintptr_t)d_state & 7u))
        return fail(BM_ERR_INVALID_ARG, "d_state must be a non-NULL, 8-byte aligned device pointer");
    if (count == 0) return ok();
    const uint64_t nw = e->run.window_start;
    const uint32_t snap = e->n_done > nw ? 2u : (e->n_done == nw ? 1u : 0u);
    const int pot = (int)e->model.pot;
    hipError_t he = e->run.prec == BM_F32 ? launch_write_f32(pot, k, d_state, snap, e->stream)
                                          : launch_write_f64(pot, k, d_state, snap, e->stream);
    if (he != hipSuccess) return hip_fail(he, "import kernel launch");
    return ok();
}

extern "C" int bm_density(bm_ensemble *e, uint32_t n_bins, uint64_t *d_counts)
{
    if (!e) return fail(BM_ERR_INVALID_ARG, "NULL handle");
    if (!d_counts) return fail(BM_ERR_INVALID_ARG, "d_counts must not be NULL");
    if (n_bins < 1 || n_bins > (1u << 20)) return fail(BM_ERR_INVALID_ARG, "n_bins must be in [1, 2^20]");
    const int pot = (int)e->model.pot;
    hipError_t he = e->run.prec == BM_F32
                        ? launch_density_f32(pot, e->k, n_bins, (unsigned long long *)d_counts, e->stream)
                        : launch_density_f64(pot, e->k, n_bins, (unsigned long long *)d_counts, e->stream);
    if (he != hipSuccess) return hip_fail(he, "density kernel launch");
    return ok();
}
