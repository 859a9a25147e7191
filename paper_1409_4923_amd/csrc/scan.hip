// scan.hip -- batched parameter scan (persistent work-stealing launch captured
// in a hipGraph), its autotuner, and the per-model default launch shapes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <unistd.h>
#include <vector>

#include "bmotor.h"
#include "host.hpp"
#include "launch.hpp"
#include "paths.hpp"
#include "reduce.hpp"
#include "scan_kernels.hpp"

using namespace bm;
using namespace bm::host;

// ---------------------------------------------------------------------------
// Launch shapes
// ---------------------------------------------------------------------------
namespace {
// An installed launch shape and the device it was installed on.
struct TuneEntry {
    bm_tune t;
    std::string arch;   // architecture name without feature suffixes ("" if unknown)
    int cus;            // compute units
};
using TuneKey = std::tuple<uint32_t, uint32_t, uint32_t, uint32_t>;
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

// Architecture name (up to the first ':') and CU count of the current device.
bool current_device(std::string &arch, int &cus)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    arch.assign(prop.gcnArchName);
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch.resize(c);
    cus = prop.multiProcessorCount;
    return true;
}

void install(const TuneKey &key, const bm_tune &t)
{
    TuneEntry e{t, std::string(), 0};
    if (!current_device(e.arch, e.cus)) { e.arch.clear(); e.cus = 0; }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = e;
}

bm_tune builtin_tune()
{
    bm_tune t;
    t.size = sizeof(bm_tune);
    t.paths_per_lane = 1;
    t.block = 256;
    t.groups_per_cu = 0;
    return t;
}
} // namespace

namespace bm {
namespace host {

bm_tune default_tune(uint32_t dyn, uint32_t pot, uint32_t noise, uint32_t prec)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(std::make_tuple(dyn, pot, noise, prec));
        if (it != g_tune.end()) return it->second.t;
    }
    bm_tune t = builtin_tune();
    // FP32 inertial paths without jump processes: two paths per lane give the step
    // loop independent work to interleave (measured 1.47 against 1.41e12 path-steps/s
    // on 2^20 paths); with jump queues the second path costs occupancy instead.
    if (prec == BM_F32 && dyn == BM_INERTIAL && (noise & (BM_NOISE_POISSON | BM_NOISE_DICH)) == 0) {
        t.paths_per_lane = 2;
        t.block = 128;
    }
    return t;
}

// LDS of the jump queues of one work-group (see queue_bytes in paths_kernels.hpp).
size_t queue_lds_bytes(uint32_t noise, uint32_t prec, uint32_t ppl, uint32_t block)
{
    const size_t kick = prec == BM_F32 ? sizeof(KickEntry<float>) : sizeof(KickEntry<double>);
    size_t per = 0;
    const size_t jg = prec == BM_F32 ? sizeof(JGKick<float>) : sizeof(JGKick<double>);
    if (noise & BM_NOISE_JUMP_GRID) per += (prec == BM_F32 ? jg_cap<float>() : jg_cap<double>()) * jg;
    else if (noise & BM_NOISE_POISSON) per += (JCAP + 1) * kick;
    if (noise & BM_NOISE_DICH) per += (JCAP + 1) * 4;
    return per * ppl * block;
}

int check_tune(const bm_tune *t, uint32_t noise, uint32_t prec)
{
    if (t->size != sizeof(bm_tune)) return fail(BM_ERR_INVALID_ARG, "bm_tune.size mismatch");
    if (t->paths_per_lane != 1 && t->paths_per_lane != 2)
        return fail(BM_ERR_INVALID_ARG, "paths_per_lane must be 1 or 2");
    if (t->paths_per_lane == 2 && prec != BM_F32)
        return fail(BM_ERR_UNSUPPORTED, "paths_per_lane = 2 is built for FP32 paths only");
    if (t->block != 64 && t->block != 128 && t->block != 256 && t->block != 512)
        return fail(BM_ERR_INVALID_ARG, "block must be 64, 128, 256 or 512");
    if (t->groups_per_cu > 64) return fail(BM_ERR_INVALID_ARG, "groups_per_cu must be <= 64");
    if (queue_lds_bytes(noise, prec, t->paths_per_lane, t->block) > 65536)
        return fail(BM_ERR_UNSUPPORTED, "jump queues of %u x %u lanes exceed 64 KiB of LDS",
                    t->paths_per_lane, t->block);
    return BM_OK;
}

} // namespace host
} // namespace bm

extern "C" int bm_tune_set_default(uint32_t dyn, uint32_t pot, uint32_t noise, uint32_t prec, const bm_tune *t)
{
    if (!t) return fail(BM_ERR_INVALID_ARG, "tune must not be NULL");
    if (dyn > BM_INERTIAL || pot > BM_POT_FREE || (noise & ~31u) || prec > BM_F32)
        return fail(BM_ERR_INVALID_ARG, "unknown model key");
    int rc = check_tune(t, noise, prec);
    if (rc) return rc;
    install(std::make_tuple(dyn, pot, noise, prec), *t);
    return ok();
}

extern "C" int bm_tune_lookup(uint32_t dyn, uint32_t pot, uint32_t noise, uint32_t prec, bm_tune *out)
{
    if (!out) return fail(BM_ERR_INVALID_ARG, "out must not be NULL");
    if (dyn > BM_INERTIAL || pot > BM_POT_FREE || (noise & ~31u) || prec > BM_F32)
        return fail(BM_ERR_INVALID_ARG, "unknown model key");
    *out = default_tune(dyn, pot, noise, prec);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.find(std::make_tuple(dyn, pot, noise, prec)) == g_tune.end())
        return fail(BM_ERR_STATE, "no shape installed for this model; the built-in default applies");
    return ok();
}

// ---------------------------------------------------------------------------
// Tuning cache file: a flat JSON document written by bm_tune_save.  The reader
// accepts any JSON text whose "entries" member is an array of objects with
// string / integer members, and ignores members it does not know.
// ---------------------------------------------------------------------------
namespace {

struct Json {
    const char *p, *end;
    void ws() { while (p < end && (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r')) ++p; }
    bool lit(char c) { ws(); if (p < end && *p == c) { ++p; return true; } return false; }
    bool str(std::string &out)
    {
        ws();
        if (p >= end || *p != '"') return false;
        ++p;
        out.clear();
        while (p < end && *p != '"') {
            if (*p == '\\') return false;           // the cache never holds escapes
            out.push_back(*p++);
        }
        if (p >= end) return false;
        ++p;
        return true;
    }
    bool num(long long &v)
    {
        ws();
        const char *q = p;
        bool neg = false;
        if (q < end && *q == '-') { neg = true; ++q; }
        if (q >= end || *q < '0' || *q > '9') return false;
        long long r = 0;
        while (q < end && *q >= '0' && *q <= '9') {
            if (r > 100000000000000LL) return false;
            r = r * 10 + (*q++ - '0');
        }
        if (q < end && (*q == '.' || *q == 'e' || *q == 'E')) return false;   // integers only
        p = q;
        v = neg ? -r : r;
        return true;
    }
    // Skips one value of any kind (nested objects / arrays, strings, numbers, literals).
    bool skip(int depth = 0)
    {
        if (depth > 32) return false;
        ws();
        if (p >= end) return false;
        std::string s;
        long long n;
        if (*p == '"') return str(s);
        if (*p == '{' || *p == '[') {
            const char close = *p == '{' ? '}' : ']';
            const bool obj = *p == '{';
            ++p;
            if (lit(close)) return true;
            do {
                if (obj && !(str(s) && lit(':'))) return false;
                if (!skip(depth + 1)) return false;
            } while (lit(','));
            return lit(close);
        }
        if (num(n)) return true;
        for (const char *w : {"true", "false", "null"}) {
            const size_t l = std::strlen(w);
            if ((size_t)(end - p) >= l && std::strncmp(p, w, l) == 0) { p += l; return true; }
        }
        // a non-integer number
        const char *q = p;
        while (q < end && (std::strchr("+-.eE", *q) || (*q >= '0' && *q <= '9'))) ++q;
        if (q == p) return false;
        p = q;
        return true;
    }
};

struct FileEntry {
    std::string arch;
    long long cus = -1, dyn = -1, pot = -1, noise = -1, prec = -1, ppl = -1, block = -1, gpc = -1;
};

bool parse_entry(Json &j, FileEntry &e)
{
    if (!j.lit('{')) return false;
    if (j.lit('}')) return true;
    do {
        std::string k;
        if (!(j.str(k) && j.lit(':'))) return false;
        long long *slot = k == "cus" ? &e.cus : k == "dyn" ? &e.dyn : k == "pot" ? &e.pot
                        : k == "noise" ? &e.noise : k == "prec" ? &e.prec : k == "paths_per_lane" ? &e.ppl
                        : k == "block" ? &e.block : k == "groups_per_cu" ? &e.gpc : nullptr;
        if (k == "arch") {
            if (!j.str(e.arch)) return false;
        } else if (slot) {
            if (!j.num(*slot)) return false;
        } else if (!j.skip()) {
            return false;
        }
    } while (j.lit(','));
    return j.lit('}');
}

bool parse_file(const std::string &text, std::vector<FileEntry> &out)
{
    Json j{text.data(), text.data() + text.size()};
    if (!j.lit('{')) return false;
    bool seen = false;
    if (!j.lit('}')) {
        do {
            std::string k;
            if (!(j.str(k) && j.lit(':'))) return false;
            if (k == "entries") {
                seen = true;
                if (!j.lit('[')) return false;
                if (!j.lit(']')) {
                    do {
                        FileEntry e;
                        if (!parse_entry(j, e)) return false;
                        out.push_back(e);
                    } while (j.lit(','));
                    if (!j.lit(']')) return false;
                }
            } else if (!j.skip()) {
                return false;
            }
        } while (j.lit(','));
        if (!j.lit('}')) return false;
    }
    j.ws();
    return seen && j.p == j.end;
}

} // namespace

extern "C" int bm_tune_save(const char *path)
{
    if (!path || !*path) return fail(BM_ERR_INVALID_ARG, "path must not be empty");
    std::string text = "{\"format\": \"libbmotor-tune\", \"version\": 1, \"entries\": [";
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        bool first = true;
        for (const auto &kv : g_tune) {
            const TuneEntry &e = kv.second;
            if (e.arch.empty()) continue;                     // installed without a device
            char buf[320];
            std::snprintf(buf, sizeof buf,
                          "%s\n  {\"arch\": \"%s\", \"cus\": %d, \"dyn\": %u, \"pot\": %u, \"noise\": %u, "
                          "\"prec\": %u, \"paths_per_lane\": %u, \"block\": %u, \"groups_per_cu\": %u}",
                          first ? "" : ",", e.arch.c_str(), e.cus, std::get<0>(kv.first), std::get<1>(kv.first),
                          std::get<2>(kv.first), std::get<3>(kv.first), e.t.paths_per_lane, e.t.block,
                          e.t.groups_per_cu);
            text += buf;
            first = false;
        }
    }
    text += "\n]}\n";
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(BM_ERR_INVALID_ARG, "cannot write %s", tmp.c_str());
    const bool wrote = std::fwrite(text.data(), 1, text.size(), f) == text.size();
    const bool closed = std::fclose(f) == 0;
    if (!wrote || !closed || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(BM_ERR_INVALID_ARG, "cannot write %s", path);
    }
    return ok();
}

extern "C" int bm_tune_load(const char *path, uint32_t *n_loaded)
{
    if (!path || !*path) return fail(BM_ERR_INVALID_ARG, "path must not be empty");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(BM_ERR_INVALID_ARG, "cannot open %s", path);
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (1u << 24)) text.append(buf, n);
    std::fclose(f);
    std::vector<FileEntry> es;
    if (!parse_file(text, es)) return fail(BM_ERR_INVALID_ARG, "%s is not a libbmotor tuning cache", path);
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    std::string arch;
    int cus = 0;
    if (!current_device(arch, cus)) return fail(BM_ERR_DEVICE, "cannot query the current device");
    std::vector<std::pair<TuneKey, bm_tune>> use;
    for (const FileEntry &e : es) {
        if (e.arch != arch || e.cus != cus) continue;
        const long long v[8] = {e.dyn, e.pot, e.noise, e.prec, e.ppl, e.block, e.gpc, e.cus};
        for (long long x : v)
            if (x < 0 || x > 0xFFFFFFFFLL) return fail(BM_ERR_INVALID_ARG, "%s: entry with a missing or bad field", path);
        if (e.dyn > BM_INERTIAL || e.pot > BM_POT_FREE || (e.noise & ~31LL) || e.prec > BM_F32)
            return fail(BM_ERR_INVALID_ARG, "%s: unknown model key", path);
        bm_tune t;
        t.size = sizeof(bm_tune);
        t.paths_per_lane = (uint32_t)e.ppl;
        t.block = (uint32_t)e.block;
        t.groups_per_cu = (uint32_t)e.gpc;
        rc = check_tune(&t, (uint32_t)e.noise, (uint32_t)e.prec);
        if (rc) return fail(rc, "%s: %s", path, last_error_text());
        use.emplace_back(std::make_tuple((uint32_t)e.dyn, (uint32_t)e.pot, (uint32_t)e.noise, (uint32_t)e.prec), t);
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto &u : use) g_tune[u.first] = TuneEntry{u.second, arch, cus};
    }
    if (n_loaded) *n_loaded = (uint32_t)use.size();
    return ok();
}

extern "C" int bm_tune_get_default(uint32_t dyn, uint32_t pot, uint32_t noise, uint32_t prec, bm_tune *out)
{
    if (!out) return fail(BM_ERR_INVALID_ARG, "out must not be NULL");
    if (dyn > BM_INERTIAL || pot > BM_POT_FREE || (noise & ~31u) || prec > BM_F32)
        return fail(BM_ERR_INVALID_ARG, "unknown model key");
    *out = default_tune(dyn, pot, noise, prec);
    return ok();
}

// ---------------------------------------------------------------------------
// Kernels of the graph besides the scan itself
// ---------------------------------------------------------------------------
__global__ void k_zero_counter(uint32_t *c) { *c = 0u; }

__global__ void __launch_bounds__(256) k_reduce_points(const Partial *part, const PointRed *red, bm_stats *out)
{
    const PointRed r = red[blockIdx.x];
    reduce_chunks(part + r.off, r.n_chunks, r.tw, out + blockIdx.x);
}

// ---------------------------------------------------------------------------
// Validation and workspace layout
// ---------------------------------------------------------------------------
namespace {

struct ScanLayout {
    size_t points, tables, items, red, counter, part, total;
    uint64_t n_items_max;    // items with one path per lane
    uint64_t n_chunks;       // 64-path partials over all points
};

size_t up(size_t v) { return (v + 255) & ~(size_t)255; }

int validate_scan(const bm_model *models, const bm_run *runs, size_t n)
{
    if (!models || !runs) return fail(BM_ERR_INVALID_ARG, "models and runs must not be NULL");
    if (n == 0 || n > 0xFFFFFFFFull) return fail(BM_ERR_INVALID_ARG, "n_points must be in [1, 2^32 - 1]");
    for (size_t i = 0; i < n; ++i) {
        int rc = validate(&models[i], &runs[i]);
        if (rc) return fail(rc, "point %zu: %s", i, last_error_text());
        if (models[i].noise & (BM_NOISE_NORMAL | BM_NOISE_JUMP_GRID))
            return fail(BM_ERR_UNSUPPORTED,
                        "point %zu: the scan runs the three-point scheme on the fixed grid only", i);
        if (runs[i].step_tol > 0)
            return fail(BM_ERR_UNSUPPORTED, "point %zu: the scan runs fixed steps (step_tol must be 0)", i);
        if (runs[i].n_steps <= runs[i].window_start)
            return fail(BM_ERR_INVALID_ARG, "point %zu: n_steps must exceed window_start", i);
        if (runs[i].n_steps > 0xFFFFFFFFull) return fail(BM_ERR_UNSUPPORTED, "point %zu: n_steps >= 2^32", i);
        if (models[i].dyn != models[0].dyn || models[i].pot != models[0].pot ||
            models[i].noise != models[0].noise || runs[i].prec != runs[0].prec)
            return fail(BM_ERR_UNSUPPORTED, "point %zu: all points must share dyn, pot, noise and prec", i);
    }
    return BM_OK;
}

ScanLayout scan_layout(const bm_run *runs, size_t n)
{
    ScanLayout L{};
    const size_t rs = runs[0].prec == BM_F32 ? 4 : 8;
    size_t tab = 0;
    for (size_t i = 0; i < n; ++i) {
        tab += table_entries(&runs[i]) * rs;
        const uint64_t c = (runs[i].n_paths + 63) / 64;
        L.n_chunks += c;
        L.n_items_max += c;
    }
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += up(bytes); return at; };
    L.points = take(n * sizeof(PointConst));
    L.tables = take(tab);
    L.items = take(L.n_items_max * sizeof(ScanItem));
    L.red = take(n * sizeof(PointRed));
    L.counter = take(sizeof(uint32_t));
    L.part = take(L.n_chunks * sizeof(Partial));
    L.total = o;
    return L;
}

hipError_t launch_scan(uint32_t prec, uint32_t dyn, int pot, int noise, const bm_tune &t, int n_cu,
                       const ScanArgs &a, hipStream_t s)
{
    const int ppl = (int)t.paths_per_lane, blk = (int)t.block, gpc = (int)t.groups_per_cu;
    if (prec == BM_F32)
        return dyn == BM_INERTIAL ? launch_scan_f32_in(pot, noise, ppl, blk, gpc, n_cu, a, s)
                                  : launch_scan_f32_od(pot, noise, ppl, blk, gpc, n_cu, a, s);
    return dyn == BM_INERTIAL ? launch_scan_f64_in(pot, noise, 1, blk, gpc, n_cu, a, s)
                              : launch_scan_f64_od(pot, noise, 1, blk, gpc, n_cu, a, s);
}

} // namespace

extern "C" int bm_scan_workspace_size(const bm_model *models, const bm_run *runs, size_t n_points, size_t *bytes)
{
    int rc = validate_scan(models, runs, n_points);
    if (rc) return rc;
    if (!bytes) return fail(BM_ERR_INVALID_ARG, "bytes must not be NULL");
    *bytes = scan_layout(runs, n_points).total;
    return ok();
}

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct bm_scan_plan {
    hipStream_t stream = nullptr;       // caller's stream (graph launches)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void release(bm_scan_plan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
}

extern "C" int bm_scan_plan_create(const bm_model *models, const bm_run *runs, size_t n, const bm_tune *tune,
                                   void *d_ws, size_t ws_bytes, bm_stats *d_results, void *stream,
                                   bm_scan_plan **out)
{
    int rc = validate_scan(models, runs, n);
    if (rc) return rc;
    if (!out || !d_results) return fail(BM_ERR_INVALID_ARG, "out and d_results must not be NULL");
    const uint32_t prec = runs[0].prec, dyn = models[0].dyn, pot = models[0].pot, noise = models[0].noise;
    const bm_tune t = tune ? *tune : default_tune(dyn, pot, noise, prec);
    rc = check_tune(&t, noise, prec);
    if (rc) return rc;
    const ScanLayout L = scan_layout(runs, n);
    if (!d_ws || ((uintptr_t)d_ws & 255u)) return fail(BM_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < L.total) return fail(BM_ERR_WORKSPACE, "workspace %zu B < %zu B needed", ws_bytes, L.total);
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    int n_cu = 0;
    hipError_t he = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (he != hipSuccess) return hip_fail(he, "hipDeviceGetAttribute");

    // Host image of the uploaded part of the workspace: points, tables, items, red.
    char *ws = (char *)d_ws;
    const size_t upload = L.counter;
    std::vector<unsigned char> img(upload, 0);
    const size_t rs = prec == BM_F32 ? 4 : 8;
    std::vector<double> tab;
    size_t tab_off = L.tables;
    uint64_t chunk_off = 0;
    const uint32_t per_item = 64u * t.paths_per_lane;
    std::vector<ScanItem> items;
    items.reserve(L.n_items_max);
    for (size_t i = 0; i < n; ++i) {
        forcing_table(&models[i], &runs[i], tab);
        for (size_t j = 0; j < tab.size(); ++j) {
            if (rs == 4) { const float f = (float)tab[j]; std::memcpy(&img[tab_off + 4 * j], &f, 4); }
            else std::memcpy(&img[tab_off + 8 * j], &tab[j], 8);
        }
        const PointConst pc = point_const(&models[i], &runs[i], ws + tab_off);
        std::memcpy(&img[L.points + i * sizeof(PointConst)], &pc, sizeof pc);
        tab_off += tab.size() * rs;
        PointRed rd;
        rd.off = chunk_off;
        rd.n_chunks = (runs[i].n_paths + 63) / 64;
        rd.tw = (double)(runs[i].n_steps - runs[i].window_start) * pc.dt;
        std::memcpy(&img[L.red + i * sizeof(PointRed)], &rd, sizeof rd);
        chunk_off += rd.n_chunks;
        const uint32_t n_items = (uint32_t)((runs[i].n_paths + per_item - 1) / per_item);
        for (uint32_t c = 0; c < n_items; ++c) items.push_back(ScanItem{(uint32_t)i, c});
    }
    // longest horizon first (longest-processing-time order), then point, then chunk
    std::stable_sort(items.begin(), items.end(), [&](const ScanItem &x, const ScanItem &y) {
        const uint64_t a = runs[x.point].n_steps, b = runs[y.point].n_steps;
        if (a != b) return a > b;
        if (x.point != y.point) return x.point < y.point;
        return x.chunk < y.chunk;
    });
    std::memcpy(&img[L.items], items.data(), items.size() * sizeof(ScanItem));

    hipStream_t s = (hipStream_t)stream;
    he = hipMemcpyAsync(d_ws, img.data(), upload, hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);      // img is released on return
    if (he != hipSuccess) return hip_fail(he, "scan upload");

    ScanArgs a;
    std::memset(&a, 0, sizeof a);
    a.points = (const PointConst *)(ws + L.points);
    a.items = (const ScanItem *)(ws + L.items);
    a.red = (const PointRed *)(ws + L.red);
    a.part = (Partial *)(ws + L.part);
    a.counter = (uint32_t *)(ws + L.counter);
    a.n_items = (uint32_t)items.size();

    bm_scan_plan *p = new (std::nothrow) bm_scan_plan();
    if (!p) return fail(BM_ERR_INVALID_ARG, "out of host memory");
    p->stream = s;
    hipStream_t cs = nullptr;
    he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (he != hipSuccess) { release(p); return hip_fail(he, "hipStreamCreate"); }
    he = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (he == hipSuccess) {
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, cs, a.counter);
        hipError_t le = hipGetLastError();
        if (le == hipSuccess) le = launch_scan(prec, dyn, (int)pot, (int)noise, t, n_cu, a, cs);
        if (le == hipSuccess) {
            hipLaunchKernelGGL(k_reduce_points, dim3((uint32_t)n), dim3(256), 0, cs, a.part, a.red, d_results);
            le = hipGetLastError();
        }
        hipError_t ee = hipStreamEndCapture(cs, &p->graph);
        he = le != hipSuccess ? le : ee;
    }
    if (he == hipSuccess) he = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (he != hipSuccess) { release(p); return hip_fail(he, "scan graph capture"); }
    *out = p;
    return ok();
}

extern "C" int bm_scan_plan_launch(bm_scan_plan *p)
{
    if (!p) return fail(BM_ERR_INVALID_ARG, "NULL plan");
    hipError_t he = hipGraphLaunch(p->exec, p->stream);
    if (he != hipSuccess) return hip_fail(he, "hipGraphLaunch");
    return ok();
}

extern "C" int bm_scan_plan_destroy(bm_scan_plan *p)
{
    if (!p) return fail(BM_ERR_INVALID_ARG, "NULL plan");
    release(p);
    return ok();
}

extern "C" int bm_scan(const bm_model *models, const bm_run *runs, size_t n, const bm_tune *tune, void *d_ws,
                       size_t ws_bytes, bm_stats *d_results, void *stream)
{
    bm_scan_plan *p = nullptr;
    int rc = bm_scan_plan_create(models, runs, n, tune, d_ws, ws_bytes, d_results, stream, &p);
    if (rc) return rc;
    rc = bm_scan_plan_launch(p);
    // wait for the launch before the executable graph is released
    const hipError_t he = hipStreamSynchronize((hipStream_t)stream);
    const int rd = bm_scan_plan_destroy(p);
    if (rc) return rc;
    if (he != hipSuccess) return hip_fail(he, "scan");
    return rd;
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
extern "C" int bm_scan_autotune(const bm_model *models, const bm_run *runs, size_t n, uint64_t max_steps,
                                void *d_ws, size_t ws_bytes, bm_stats *d_results, void *stream, bm_tune *best,
                                float *best_ms)
{
    int rc = validate_scan(models, runs, n);
    if (rc) return rc;
    if (!best) return fail(BM_ERR_INVALID_ARG, "best must not be NULL");
    if (max_steps < 32) return fail(BM_ERR_INVALID_ARG, "max_steps must be >= 32");
    // Horizons scaled by one factor so that the longest is max_steps (at least 32
    // steps each): the timed scans keep the spread of work over the points, which
    // decides how the persistent grid's tail balances.
    std::vector<bm_run> short_runs(runs, runs + n);
    uint64_t longest = 0;
    for (const auto &r : short_runs) longest = r.n_steps > longest ? r.n_steps : longest;
    if (longest > max_steps) {
        const double f = (double)max_steps / (double)longest;
        for (auto &r : short_runs) {
            uint64_t ns = (uint64_t)std::llround((double)r.n_steps * f);
            if (ns < 32) ns = 32;
            if (ns > r.n_steps) ns = r.n_steps;
            r.n_steps = ns;
            r.window_start = ns / 2;
        }
    }
    const uint32_t prec = runs[0].prec, noise = models[0].noise;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(BM_ERR_DEVICE, "hipEventCreate failed");
    float best_t = 0.0f;
    bool have = false;
    bm_tune bt = builtin_tune();
    const uint32_t ppls[2] = {1, 2};
    const uint32_t blocks[4] = {64, 128, 256, 512};
    int result = BM_OK;
    for (uint32_t pi = 0; pi < (prec == BM_F32 ? 2u : 1u) && result == BM_OK; ++pi) {
        for (uint32_t bi = 0; bi < 4 && result == BM_OK; ++bi) {
            bm_tune t = builtin_tune();
            t.paths_per_lane = ppls[pi];
            t.block = blocks[bi];
            if (queue_lds_bytes(noise, prec, t.paths_per_lane, t.block) > 65536) continue;
            bm_scan_plan *p = nullptr;
            rc = bm_scan_plan_create(models, short_runs.data(), n, &t, d_ws, ws_bytes, d_results, stream, &p);
            if (rc) { result = rc; break; }
            // warm-up, then the better of two timed launches
            float ms = 0.0f;
            hipError_t he = hipGraphLaunch(p->exec, s);
            for (int rep = 0; rep < 2 && he == hipSuccess; ++rep) {
                float t_ms = 0.0f;
                he = hipEventRecord(e0, s);
                if (he == hipSuccess) he = hipGraphLaunch(p->exec, s);
                if (he == hipSuccess) he = hipEventRecord(e1, s);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                if (he == hipSuccess) he = hipEventElapsedTime(&t_ms, e0, e1);
                if (he == hipSuccess && (rep == 0 || t_ms < ms)) ms = t_ms;
            }
            release(p);
            if (he != hipSuccess) { result = hip_fail(he, "autotune timing"); break; }
            if (!have || ms < best_t) { best_t = ms; bt = t; have = true; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result) return result;
    *best = bt;
    if (best_ms) *best_ms = best_t;
    install(std::make_tuple(models[0].dyn, models[0].pot, noise, prec), bt);
    return ok();
}
