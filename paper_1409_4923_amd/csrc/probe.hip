// probe.hip -- VALU issue-rate probe for the roofline of the path kernels.
//
// The path kernels are bound by vector-ALU issue.  Their roofline peak is derived
// from the chip's unit counts and clock (one wave64 instruction per CU per clock,
// 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 lane-ops/s); this probe measures what the
// device issues for three instruction mixes: eight independent non-packed FP32 FMA
// chains per lane; the same with a compare and a select after every FMA (the
// instruction classes of Algorithm 2's three-point increment); and the same with an
// exp2 after every FMA (the transcendental unit, as in the cosines of the drift and
// the GELU of the surrogate).  It is not part of
// the method: it is built into its own library, libbmprobe.so, which only the
// benchmark's calibration loads.
//
//   int bmp_valu_probe(uint32_t mix, uint32_t iters, float *d_out, size_t n_out,
//                      void *stream, double *lane_ops_per_s);
//   const char *bmp_last_error(void);
//
// Runs n_out / 256 work-groups of 256 lanes, each lane carrying eight independent
// non-packed FP32 FMA chains for `iters` iterations (mix 0), each FMA followed
// by a compare and a select (mix 1) or by a v_exp_f32 (mix 2); d_out [n_out]
// (device, caller-owned) receives one float per lane.  One warm-up launch, then the
// best of three timed launches on `stream`; *lane_ops_per_s = lanes x iters x 8 x
// (1, 3 or 2) / time.
// Synchronises `stream`.  Returns 0, -1 for bad arguments (n_out a multiple of 256
// in [256, 2^28], iters in [1, 2^24], mix 0, 1 or 2, non-NULL pointers) or -4 when a
// HIP call fails; bmp_last_error() gives the calling thread's message.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace {

thread_local std::string g_msg;

int probe_fail(int code, const char *msg, hipError_t e = hipSuccess)
{
    g_msg = msg;
    if (e != hipSuccess) { g_msg += ": "; g_msg += hipGetErrorString(e); }
    return code;
}

constexpr int PROBE_CHAINS = 8;

template <int MIX>
__global__ void __launch_bounds__(256) k_valu_probe(float *out, float a, float b, uint32_t iters)
{
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    float x[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) x[k] = (float)threadIdx.x * 1e-3f + (float)k;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < PROBE_CHAINS; ++k) {
            if constexpr (MIX == 2) {
                // 2^(b - a x): stays in (0, 2^b] for x > 0
                x[k] = __builtin_amdgcn_exp2f(__builtin_fmaf(x[k], -a, b));
            } else {
                x[k] = __builtin_fmaf(x[k], a, b);
            }
            if constexpr (MIX == 1) x[k] = (x[k] > 0.5f) ? x[k] : b;    // compare + select
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) s += x[k];
    out[gid] = s;                                                        // keeps the chains live
}

} // namespace

extern "C" const char *bmp_last_error(void) { return g_msg.c_str(); }

extern "C" int bmp_valu_probe(uint32_t mix, uint32_t iters, float *d_out, size_t n_out, void *stream,
                              double *lane_ops_per_s)
{
    if (mix > 2) return probe_fail(-1, "mix must be 0 (FMA), 1 (FMA + compare + select) or 2 (FMA + exp2)");
    if (iters == 0 || iters > (1u << 24)) return probe_fail(-1, "iters must be in [1, 2^24]");
    if (!d_out || !lane_ops_per_s) return probe_fail(-1, "d_out and lane_ops_per_s must not be NULL");
    if (n_out < 256 || n_out % 256 != 0 || n_out / 256 > (1u << 20))
        return probe_fail(-1, "n_out must be a multiple of 256 in [256, 2^28]");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return probe_fail(-4, "hipEventCreate failed");
    }
    const unsigned blocks = (unsigned)(n_out / 256);
    float best = 0.0f;
    hipError_t he = hipSuccess;
    for (int rep = 0; rep < 4 && he == hipSuccess; ++rep) {            // first launch: warm-up
        he = hipEventRecord(e0, s);
        if (he == hipSuccess) {
            if (mix == 2) k_valu_probe<2><<<blocks, 256, 0, s>>>(d_out, 0.999f, 0.001f, iters);
            else if (mix == 1) k_valu_probe<1><<<blocks, 256, 0, s>>>(d_out, 0.999f, 0.001f, iters);
            else k_valu_probe<0><<<blocks, 256, 0, s>>>(d_out, 0.999f, 0.001f, iters);
            he = hipGetLastError();
        }
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he == hipSuccess && rep > 0 && (rep == 1 || ms < best)) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (he != hipSuccess) return probe_fail(-4, "VALU probe", he);
    const double ops_per_iter = PROBE_CHAINS * (mix == 1 ? 3.0 : mix == 2 ? 2.0 : 1.0);
    *lane_ops_per_s = (double)n_out * iters * ops_per_iter / (best * 1e-3);
    g_msg.clear();
    return 0;
}
