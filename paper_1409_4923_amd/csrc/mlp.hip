// mlp.hip -- ensemble MLP surrogate: inference, training (back-propagation of the
// mean squared error, Adam), ensemble statistics and the routing of uncertain
// queries to the Monte Carlo fallback.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "bmotor.h"
#include "common.hpp"
#include "host.hpp"
#include "mlp_kernels.hpp"

using namespace bm;
using namespace bm::host;
using namespace bm::mlp;

static_assert(NPARAM == BM_MLP_PARAMS, "parameter block differs from bmotor.h");
static_assert(NBF == BM_MLP_BF16, "BF16 block differs from bmotor.h");
static_assert(IN == BM_MLP_INPUTS && H == BM_MLP_HIDDEN, "shape differs from bmotor.h");

namespace {


// ---------------------------------------------------------------------------
// Small layers
// ---------------------------------------------------------------------------
// Layer 1 (5 -> 256) + GELU of the training forward; block = one row, lane = output;
// grid (rows, members).  Row r of member m reads x[idx ? idx[m * idx_stride + r] : r].
__global__ void __launch_bounds__(256) k_l1_fwd(const float *x, const uint32_t *idx, uint64_t idx_stride,
                                                const bf16_t *wbf, const float *params, int rows, float *u_out,
                                                float *z_out, bf16_t *a_out)
{
    const int r = blockIdx.x, m = blockIdx.y, o = threadIdx.x;
    const uint64_t src = idx ? (uint64_t)idx[(uint64_t)m * idx_stride + r] : (uint64_t)r;
    float u[IN];
    normalise(x + src * IN, u);
    const bf16_t *w = wbf + (uint64_t)m * NBF + BOFF_W1 + o * IN;
    float z = params[(uint64_t)m * NPARAM + OFF_B1 + o];
#pragma unroll
    for (int j = 0; j < IN; ++j) z = fmaf(bf2f(w[j]), u[j], z);
    const uint64_t row = (uint64_t)m * rows + r;
    if (u_out && o < IN) u_out[row * IN + o] = u[o];
    if (z_out) z_out[row * H + o] = z;
    a_out[row * H + o] = f2bf(gelu(z));
}

// Output layer, loss and the output layer's gradients of the training step, fused.
// Per row (one wave, four features per lane): y = a3 . W4 + b4, e = y - t,
// dy = 2 e / B and dz3 = dy W4 gelu'(z3); per work-group of HEAD_ROWS rows the sums of
// dy a3 (dW4), dy (db4) and e^2 (loss), combined over its waves in a fixed order.
// grid (B / HEAD_ROWS, members), 256 lanes; B is a multiple of HEAD_ROWS.
constexpr int HEAD_ROWS = 16;
constexpr int HEAD_W = H + 2;          // partial record: dW4[256], db4, sum e^2

__global__ void __launch_bounds__(256) k_head(const bf16_t *a3, const float *z3, const bf16_t *wbf,
                                              const float *params, const float *t, const uint32_t *idx,
                                              uint64_t idx_stride, int B, bf16_t *dz3, float *hpart)
{
    __shared__ float red[4][HEAD_W];
    const int m = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bf16_t *W4 = wbf + (uint64_t)m * NBF + BOFF_W4;
    float w[4], sw[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = bf2f(W4[lane * 4 + j]);
    const float b4 = params[(uint64_t)m * NPARAM + OFF_B4];
    float sb = 0.0f, se = 0.0f;
#pragma unroll
    for (int rr = 0; rr < HEAD_ROWS / 4; ++rr) {
        const int r = blockIdx.x * HEAD_ROWS + wave * (HEAD_ROWS / 4) + rr;
        const uint64_t row = (uint64_t)m * B + r;
        float av[4];
        float y = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            av[j] = bf2f(a3[row * H + lane * 4 + j]);
            y = fmaf(av[j], w[j], y);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) y += __shfl_xor(y, off, 64);   // the same sum in every lane
        const uint64_t src = idx ? (uint64_t)idx[(uint64_t)m * idx_stride + r] : (uint64_t)r;
        const float e = (y + b4) - t[src];
        const float dy = 2.0f * e / (float)B;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            dz3[row * H + lane * 4 + j] = f2bf(dy * w[j] * gelu_grad(z3[row * H + lane * 4 + j]));
            sw[j] = fmaf(dy, av[j], sw[j]);
        }
        sb += dy;
        se = fmaf(e, e, se);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wave][lane * 4 + j] = sw[j];
    if (lane == 0) {
        red[wave][H] = sb;
        red[wave][H + 1] = se;
    }
    __syncthreads();
    float *out = hpart + ((uint64_t)m * gridDim.x + blockIdx.x) * HEAD_W;
    for (int o = threadIdx.x; o < HEAD_W; o += 256) out[o] = ((red[0][o] + red[1][o]) + red[2][o]) + red[3][o];
}

// dW4, db4 and the loss of each member: the work-group partials added in order;
// grid (members), 256 lanes.
__global__ void __launch_bounds__(256) k_head_final(const float *hpart, int nblk, int B, float *grad, float *loss)
{
    const int m = blockIdx.x;
    const float *p = hpart + (uint64_t)m * nblk * HEAD_W;
    float *g = grad + (uint64_t)m * NPARAM;
    for (int o = threadIdx.x; o < HEAD_W; o += 256) {
        float s = 0.0f;
#pragma unroll 8
        for (int b = 0; b < nblk; ++b) s += p[(uint64_t)b * HEAD_W + o];
        if (o < H) g[OFF_W4 + o] = s;
        else if (o == H) g[OFF_B4] = s;
        else if (loss) loss[m] = s / (float)B;
    }
}

// Gradients that are column sums over the batch rather than GEMMs: the 5-wide input
// layer (dW1[o][j] = sum_b dz1[b][o] u[b][j], db1 = sum_b dz1[b][:]).  (The biases of
// the 256 x 256 layers come with their weight-gradient GEMM, the output layer with
// k_head.)  Pass 1: grid
// (n_chunks, members), lane = column o, each block sums one chunk of consecutive
// rows; pass 2 adds the chunks in order, so the result does not depend on the launch.
constexpr int RED_MAX_CHUNKS = 64;
constexpr int NV1 = IN + 1;            // dW1[o][0..4], db1[o]

__host__ __device__ inline int red_rows(int B) { return B / 64 < 16 ? 16 : B / 64; }

__global__ void __launch_bounds__(256) k_colsum(const bf16_t *dz, const float *u, int B, int rows, float *part)
{
    const int c = blockIdx.x, m = blockIdx.y, o = threadIdx.x, nchunk = gridDim.x;
    float s[NV1];
#pragma unroll
    for (int q = 0; q < NV1; ++q) s[q] = 0.0f;
    const uint64_t row0 = (uint64_t)m * B + (uint64_t)c * rows;
#pragma unroll 8
    for (int r = 0; r < rows; ++r) {
        const uint64_t row = row0 + r;
        const float d = bf2f(dz[row * H + o]);
#pragma unroll
        for (int j = 0; j < IN; ++j) s[j] = fmaf(d, u[row * IN + j], s[j]);
        s[IN] += d;
    }
#pragma unroll
    for (int q = 0; q < NV1; ++q) part[(((uint64_t)m * nchunk + c) * NV1 + q) * H + o] = s[q];
}

// grid (NV1, members): block q adds the chunks of sum q (dW1[:][q], or db1 for q = IN).
__global__ void __launch_bounds__(256) k_colsum_final(const float *part, int nchunk, float *grad)
{
    const int q = blockIdx.x, m = blockIdx.y, o = threadIdx.x;
    float s = 0.0f;
    // the chunks in order; unrolled so that the loads of several chunks are in flight
#pragma unroll 8
    for (int c = 0; c < nchunk; ++c) s += part[(((uint64_t)m * nchunk + c) * NV1 + q) * H + o];
    float *g = grad + (uint64_t)m * NPARAM;
    if (q < IN) g[OFF_W1 + o * IN + q] = s;
    else g[OFF_B1 + o] = s;
}

hipError_t colsum(uint32_t nm, int B, const bf16_t *dz, const float *u, float *part, float *grad, hipStream_t s)
{
    const int rows = red_rows(B), nchunk = B / rows;
    hipLaunchKernelGGL(k_colsum, dim3(nchunk, nm), dim3(256), 0, s, dz, u, B, rows, part);
    hipLaunchKernelGGL(k_colsum_final, dim3(NV1, nm), dim3(256), 0, s, (const float *)part, nchunk, grad);
    return hipGetLastError();
}

// Weight and bias gradients of a 256 x 256 layer from the ks split-K partials of
// the weight-gradient GEMM, each element's partials added in order; grid
// (H * H / 256 + 1, members): the last block of a member adds the bias partials.
__global__ void __launch_bounds__(256) k_wgrad_sum(const float *wpart, const float *bpart, int ks, int nm,
                                                   float *grad, int woff, int boff)
{
    const int m = blockIdx.y, t = threadIdx.x;
    constexpr int NB = H * H / 256;
    float *g = grad + (uint64_t)m * NPARAM;
    float s = 0.0f;
    if ((int)blockIdx.x < NB) {
        const uint64_t e = (uint64_t)blockIdx.x * 256 + t;
        for (int kc = 0; kc < ks; ++kc) s += wpart[((uint64_t)kc * nm + m) * (H * H) + e];
        g[woff + e] = s;
    } else {
        for (int kc = 0; kc < ks; ++kc) s += bpart[((uint64_t)kc * nm + m) * H + t];
        g[boff + t] = s;
    }
}

// BF16 index of parameter p of a member, or -1 for biases.
__device__ __forceinline__ int bf_index(int p)
{
    if (p < OFF_B1) return BOFF_W1 + (p - OFF_W1);
    if (p >= OFF_W2 && p < OFF_B2) return BOFF_W2 + (p - OFF_W2);
    if (p >= OFF_W3 && p < OFF_B3) return BOFF_W3 + (p - OFF_W3);
    if (p >= OFF_W4 && p < OFF_B4) return BOFF_W4 + (p - OFF_W4);
    return -1;
}

__global__ void __launch_bounds__(256) k_cast(const float *params, bf16_t *wbf, uint64_t total)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const uint64_t m = i / NPARAM;
    const int p = (int)(i - m * NPARAM);
    const int b = bf_index(p);
    if (b >= 0) wbf[m * NBF + b] = f2bf(params[i]);
}

// Adam (Kingma & Ba) with bias-corrected moments, then the BF16 weight copy.
__global__ void __launch_bounds__(256) k_adam(float *params, const float *grad, float *mo, float *ve, bf16_t *wbf,
                                              uint64_t total, float lr, float b1, float b2, float eps, float c1,
                                              float c2)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const float g = grad[i];
    const float m = b1 * mo[i] + (1.0f - b1) * g;
    const float v = b2 * ve[i] + (1.0f - b2) * g * g;
    mo[i] = m;
    ve[i] = v;
    const float p = params[i] - lr * (m * c1) / (sqrtf(v * c2) + eps);
    params[i] = p;
    const uint64_t mem = i / NPARAM;
    const int b = bf_index((int)(i - mem * NPARAM));
    if (b >= 0) wbf[mem * NBF + b] = f2bf(p);
}

// Initial parameters U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from Philox (tag 4).
__global__ void __launch_bounds__(256) k_init_params(float *params, uint64_t total, uint32_t k0, uint32_t k1)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const uint64_t m = i / NPARAM;
    const int p = (int)(i - m * NPARAM);
    const U4 q = philox4x32_10((uint32_t)p, (uint32_t)m, 0u, 4u, k0, k1);
    const float u = (float)(q.x >> 8) * 0x1p-24f * 2.0f - 1.0f;
    const float fan = (p < OFF_W2) ? (float)IN : (float)H;
    params[i] = u / sqrtf(fan);
}

// Ensemble mean / population std over members and the routing flag; grid over rows.
__global__ void __launch_bounds__(256) k_stats(const float *y, int members, uint64_t B, float thr, float *mean,
                                               float *stdv, uint32_t *blk_count)
{
    const uint64_t b = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    bool flag = false;
    if (b < B) {
        float s = 0.0f;
        for (int m = 0; m < members; ++m) s += y[(uint64_t)m * B + b];
        const float mu = s / (float)members;
        float v = 0.0f;
        for (int m = 0; m < members; ++m) {
            const float d = y[(uint64_t)m * B + b] - mu;
            v = fmaf(d, d, v);
        }
        const float sd = sqrtf(v / (float)members);
        mean[b] = mu;
        stdv[b] = sd;
        flag = !(sd <= thr);                    // NaN std also falls back
    }
    __shared__ uint32_t cnt[4];
    const unsigned long long bal = __ballot(flag);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) blk_count[blockIdx.x] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// Exclusive scan of the block counts (one block, sequential chunks) and the total.
__global__ void __launch_bounds__(256) k_scan_counts(uint32_t *blk, uint64_t nblk, uint32_t *total)
{
    __shared__ uint32_t part[256];
    const uint64_t per = (nblk + 255) / 256;
    const uint64_t lo = per * threadIdx.x, hi = lo + per < nblk ? lo + per : nblk;
    uint32_t s = 0;
    for (uint64_t i = lo; i < hi; ++i) s += blk[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < 256; ++i) { const uint32_t c = part[i]; part[i] = acc; acc += c; }
        *total = acc;
    }
    __syncthreads();
    uint32_t acc = part[threadIdx.x];
    for (uint64_t i = lo; i < hi; ++i) { const uint32_t c = blk[i]; blk[i] = acc; acc += c; }
}

// Scatter the flagged row indices in increasing order.
__global__ void __launch_bounds__(256) k_compact(const float *stdv, uint64_t B, float thr, const uint32_t *blk_off,
                                                 uint32_t *out)
{
    const uint64_t b = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const bool flag = b < B && !(stdv[b] <= thr);
    __shared__ uint32_t cnt[4];
    const unsigned long long bal = __ballot(flag);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) cnt[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t base = blk_off[blockIdx.x];
    for (int i = 0; i < w; ++i) base += cnt[i];
    const uint32_t rank = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
    if (flag) out[base + rank] = (uint32_t)b;
}

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------
size_t up(size_t v) { return (v + 255) & ~(size_t)255; }

struct MlpLayout {
    size_t u, z1, z2, z3, a1, a2, a3, y, dz1, dz2, dz3, hpart, red, wpart, bpart, blk, total;
};

// Split of the batch (the K of the weight-gradient GEMMs) over work-groups: the
// largest power of two <= min(WG_MAX_SPLIT, B / 256) with B / ksplit a multiple of 32.
constexpr int WG_MAX_SPLIT = 8;
int wgrad_split(int B)
{
    int ks = 1;
    while (2 * ks <= WG_MAX_SPLIT && 2 * ks * 256 <= B && B % (2 * ks * TK) == 0) ks *= 2;
    return ks;
}

MlpLayout mlp_layout(uint32_t nm, uint64_t batch, bool training)
{
    MlpLayout L{};
    const uint64_t R = batch;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += up(bytes); return at; };
    if (training) {                    // inference keeps its activations in registers
        L.a1 = take(nm * R * H * 2);
        L.a2 = take(nm * R * H * 2);
        L.a3 = take(nm * R * H * 2);
        L.u = take(nm * R * IN * 4);
        L.z1 = take(nm * R * H * 4);
        L.z2 = take(nm * R * H * 4);
        L.z3 = take(nm * R * H * 4);
        L.dz1 = take(nm * R * H * 2);
        L.dz2 = take(nm * R * H * 2);
        L.dz3 = take(nm * R * H * 2);
        L.hpart = take(nm * (R / HEAD_ROWS) * HEAD_W * 4);
        L.red = take((size_t)nm * RED_MAX_CHUNKS * NV1 * H * 4);
        L.wpart = take((size_t)WG_MAX_SPLIT * nm * H * H * 4);
        L.bpart = take((size_t)WG_MAX_SPLIT * nm * H * 4);
    } else {
        L.y = take(nm * batch * 4);
        L.blk = take(((batch + 255) / 256) * 4 + 4);
    }
    L.total = o;
    return L;
}

int check_members(uint32_t nm)
{
    if (nm < 1 || nm > BM_MLP_MAX_MEMBERS)
        return fail(BM_ERR_INVALID_ARG, "n_members must be in [1, %d]", BM_MLP_MAX_MEMBERS);
    return BM_OK;
}

int check_ws(const MlpLayout &L, void *d_ws, size_t ws_bytes)
{
    if (!d_ws || ((uintptr_t)d_ws & 255u)) return fail(BM_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < L.total) return fail(BM_ERR_WORKSPACE, "workspace %zu B < %zu B needed", ws_bytes, L.total);
    return BM_OK;
}

// k tiles of 128 when every work-group's k range allows (K = 256 layers, 256-row
// splits of the batch), else of 32.
template <int EPI, bool TA, bool TB>
hipError_t gemm(const GemmArgs &g, int members, hipStream_t s)
{
    const int ks = g.ksplit > 1 ? g.ksplit : 1;
    const int krange = ks > 1 ? g.kchunk : g.K;
    const dim3 grid((uint32_t)(g.N / TN), (uint32_t)((g.M + TM - 1) / TM), (uint32_t)(members * ks));
    if (krange % 128 == 0)
        hipLaunchKernelGGL((k_gemm<EPI, TA, TB, 128>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm<EPI, TA, TB, TK>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

GemmArgs gemm_args()
{
    GemmArgs g;
    std::memset(&g, 0, sizeof g);
    return g;
}

// ---------------------------------------------------------------------------
// Fused inference: one work-group runs 128 rows of one member through all four
// layers; activations never leave the registers.  The 256 x 256 layers are
// computed transposed, Z^T = W A^T, with W as the MFMA A operand and the
// activations as the B operand: a 16 x 16 output tile leaves lane (g = lane/16,
// c = lane%16) holding features 4g..4g+3 of row c, which is exactly the B-operand
// slot of the next layer if its contraction index is permuted -- k-step s, slot j
// of lane group g stands for feature 32 s + 4 g + j (j < 4) or 32 s + 16 + 4 g +
// (j - 4) (j >= 4), and the W fragments are read from LDS in that order.
// The contraction runs outermost: each wave keeps the accumulators of all 16 output
// tiles of its 32 rows (128 registers) and walks the 8 k-steps of a layer, so W is
// staged one 32-wide k slice (all 256 output rows) at a time and the GELU epilogue
// runs once per layer.  256 registers per lane give two waves per SIMD (two
// work-groups per CU), so one group's epilogue overlaps the other's MFMAs.
// ---------------------------------------------------------------------------
constexpr int FROWS = 128;             // rows per work-group
constexpr int INFER_RT = 2;            // row tiles of 16 per wave
constexpr int INFER_BT = 256;          // 4 waves per work-group
constexpr int SK = 32;                 // row of a staged k slice (bf16), 16-byte pairs swizzled
constexpr int NSLICE = 16;             // k slices of the two 256 x 256 layers

__device__ __forceinline__ __bf16 to_bf(float f) { return (__bf16)f; }   // v_cvt_pk_bf16_f32 (RNE)

__device__ __forceinline__ int perm_feature(int s, int g, int j)
{
    return 32 * s + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

__global__ void __launch_bounds__(INFER_BT, 2) k_mlp_infer(const float *x, uint64_t rows, const bf16_t *wbf,
                                                           const float *params, float *y, uint64_t y_stride)
{
    constexpr int RT = INFER_RT, BT = INFER_BT;
    static_assert(BT == H, "thread t fills the small tables' entries of feature t");
    static_assert(BT / 64 * 16 * RT == FROWS, "the waves cover the group's rows");
    __shared__ __align__(16) bf16_t sW[3][H * SK];
    __shared__ __align__(16) float sL1[H * 8];          // per feature: W1[f][0..4], b1[f], pad
    __shared__ __align__(16) float sB[2][H];
    __shared__ float sW4[H];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4, c = lane & 15;
    const int m = blockIdx.y;
    const float *P = params + (uint64_t)m * NPARAM;
    const bf16_t *WB = wbf + (uint64_t)m * NBF;
#pragma unroll
    for (int j = 0; j < IN; ++j) sL1[t * 8 + j] = bf2f(WB[BOFF_W1 + t * IN + j]);
    sL1[t * 8 + 5] = P[OFF_B1 + t];
    sB[0][t] = P[OFF_B2 + t];
    sB[1][t] = P[OFF_B3 + t];
    sW4[t] = bf2f(WB[BOFF_W4 + t]);

    // slice T: layer 2 + T / 8, k columns 32 (T % 8) .. + 31 of all 256 rows, in
    // 16-byte units: unit u = t + i BT is row u / 4, columns 8 (u % 4) .. + 7
    constexpr int UNITS = H * 32 / 8 / BT;
    auto load_slice = [&](int T, uint4 (&v)[UNITS]) {
        const bf16_t *W = WB + (T < 8 ? BOFF_W2 : BOFF_W3) + 32 * (T & 7);
#pragma unroll
        for (int i = 0; i < UNITS; ++i) {
            const int u = t + i * BT;
            v[i] = *reinterpret_cast<const uint4 *>(W + (uint64_t)(u >> 2) * H + (u & 3) * 8);
        }
    };
    // In LDS a slice row holds four 16-byte pairs: pair p is 8-byte unit p (k columns
    // 4p .. 4p + 3) followed by unit p + 4, which is exactly one lane group's A
    // fragment (one 16-byte read, no register shuffling), and it sits at position
    // p ^ ((r >> 1) & 3) of row r, so the 8 lanes a read serves at a time hit
    // different banks.  Inside the k loop a slice is staged in two halves of
    // UNITS / 2 units per thread.
    auto load_half = [&](int T, int hf, uint4 (&v)[UNITS / 2]) {
        const bf16_t *W = WB + (T < 8 ? BOFF_W2 : BOFF_W3) + 32 * (T & 7);
#pragma unroll
        for (int i = 0; i < UNITS / 2; ++i) {
            const int u = t + (i + hf * UNITS / 2) * BT;
            v[i] = *reinterpret_cast<const uint4 *>(W + (uint64_t)(u >> 2) * H + (u & 3) * 8);
        }
    };
    auto store_half = [&](int buf, int hf, const uint4 (&v)[UNITS / 2]) {
#pragma unroll
        for (int i = 0; i < UNITS / 2; ++i) {
            const int u = t + (i + hf * UNITS / 2) * BT;
            const int r = u >> 2, q = u & 3, f = (r >> 1) & 3;
            const int p0 = (2 * q) & 3, p1 = (2 * q + 1) & 3, hf = q >> 1;   // units 2q, 2q + 1
            *reinterpret_cast<uint2 *>(&sW[buf][r * SK + (p0 ^ f) * 8 + 4 * hf]) = uint2{v[i].x, v[i].y};
            *reinterpret_cast<uint2 *>(&sW[buf][r * SK + (p1 ^ f) * 8 + 4 * hf]) = uint2{v[i].z, v[i].w};
        }
    };
    auto store_slice = [&](int buf, const uint4 (&v)[UNITS]) {
#pragma unroll
        for (int i = 0; i < UNITS; ++i) {
            const int u = t + i * BT;
            const int r = u >> 2, q = u & 3, f = (r >> 1) & 3;
            const int p0 = (2 * q) & 3, p1 = (2 * q + 1) & 3, hf = q >> 1;   // units 2q, 2q + 1
            *reinterpret_cast<uint2 *>(&sW[buf][r * SK + (p0 ^ f) * 8 + 4 * hf]) = uint2{v[i].x, v[i].y};
            *reinterpret_cast<uint2 *>(&sW[buf][r * SK + (p1 ^ f) * 8 + 4 * hf]) = uint2{v[i].z, v[i].w};
        }
    };
    uint4 pv[UNITS];
    load_slice(0, pv);
    store_slice(0, pv);
    load_slice(1, pv);
    store_slice(1, pv);
    __syncthreads();

    // ---- layer 1 (5 -> 256, FP32 FMA on the BF16 weights) into B operands; each
    //      weight row read from LDS once for both row tiles ----
    const uint64_t base = (uint64_t)blockIdx.x * FROWS + (uint64_t)wave * 16 * RT;
    bf16x8 act[RT][8];
    float u[RT][IN];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const uint64_t r = base + 16 * rt + c;
        normalise(x + (r < rows ? r : 0) * IN, u[rt]);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float *w = &sL1[perm_feature(s, g, j) * 8];
            const float4 w03 = *reinterpret_cast<const float4 *>(w);
            const float2 w45 = *reinterpret_cast<const float2 *>(w + 4);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                float z = w45.y;
                z = fmaf(w03.x, u[rt][0], z);
                z = fmaf(w03.y, u[rt][1], z);
                z = fmaf(w03.z, u[rt][2], z);
                z = fmaf(w03.w, u[rt][3], z);
                z = fmaf(w45.x, u[rt][4], z);
                act[rt][s][j] = to_bf(gelu(z));
            }
        }
    }

    // ---- layers 2 and 3 on MFMA, k slice by k slice ----
    // Slice T lives in LDS buffer T % 3; slice T + 2 is fetched from global memory
    // during iteration T, half after half, and stored into the buffer slice T - 1
    // used, which every wave finished reading before the barrier that ended iteration
    // T - 1.  That barrier also published slice T + 1 before iteration T + 1 reads it.
    floatx4 acc[16][RT];
#pragma unroll
    for (int T = 0; T < NSLICE; ++T) {
        const int s = T & 7;
        uint4 ph[UNITS / 2];
        if (T + 2 < NSLICE) load_half(T + 2, 0, ph);
        // The MFMA block runs at raised wave priority, so the scheduler keeps the
        // matrix cores fed from this wave while the other group's wave on the SIMD
        // works through its VALU epilogue.
        __builtin_amdgcn_s_setprio(1);
        // lane (g, c) reads pair g (units g and 4 + g) of rows 16 ft + c
        const bf16_t *sfr = &sW[T % 3][c * SK + 8 * (g ^ ((c >> 1) & 3))];
#pragma unroll
        for (int ft = 0; ft < 16; ++ft) {
            if (ft == 8 && T + 2 < NSLICE) {
                store_half((T + 2) % 3, 0, ph);
                load_half(T + 2, 1, ph);
            }
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sfr + 16 * ft * SK);
            // the accumulators start at the bias of their output features
            const floatx4 bias = *reinterpret_cast<const floatx4 *>(&sB[T >> 3][16 * ft + 4 * g]);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                acc[ft][rt] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, act[rt][s], s == 0 ? bias : acc[ft][rt], 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
        if (s == 7) {
            // epilogue: acc[ft][rt][i] = Z^T[16 ft + 4 g + i][row c of tile rt] -> the
            // next layer's slot (k-step ft / 2, j = 4 (ft % 2) + i)
#pragma unroll
            for (int ft = 0; ft < 16; ++ft)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) act[rt][ft >> 1][4 * (ft & 1) + i] = to_bf(gelu(acc[ft][rt][i]));
        }
        if (T + 2 < NSLICE) store_half((T + 2) % 3, 1, ph);
        __syncthreads();
    }

    // ---- layer 4 (256 -> 1): partial dot per lane group, then across the 4 groups ----
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        float sum = 0.0f;
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) sum = fmaf((float)act[rt][s][j], sW4[perm_feature(s, g, j)], sum);
        sum += __shfl_xor(sum, 16, 64);
        sum += __shfl_xor(sum, 32, 64);
        const uint64_t r = base + 16 * rt + c;
        if (g == 0 && r < rows) y[(uint64_t)m * y_stride + r] = sum + P[OFF_B4];
    }
}

// Training forward of `rows` rows through layers 1-3 of all members, keeping what
// backward needs (normalised inputs, pre-activations z, BF16 activations); the output
// layer runs fused with the loss (k_head).
hipError_t train_forward(uint32_t nm, const float *params, const bf16_t *wbf, const float *x, const uint32_t *idx,
                         uint64_t idx_stride, int rows, char *ws, const MlpLayout &L, hipStream_t s)
{
    bf16_t *a1 = (bf16_t *)(ws + L.a1), *a2 = (bf16_t *)(ws + L.a2), *a3 = (bf16_t *)(ws + L.a3);
    float *u = (float *)(ws + L.u), *z1 = (float *)(ws + L.z1);
    float *z2 = (float *)(ws + L.z2), *z3 = (float *)(ws + L.z3);
    hipLaunchKernelGGL(k_l1_fwd, dim3((uint32_t)rows, nm), dim3(256), 0, s, x, idx, idx_stride, wbf, params, rows,
                       u, z1, a1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bf16_t *ain[2] = {a1, a2};
    bf16_t *aout[2] = {a2, a3};
    float *zo[2] = {z2, z3};
    const int woff[2] = {BOFF_W2, BOFF_W3}, boff[2] = {OFF_B2, OFF_B3};
    for (int l = 0; l < 2; ++l) {
        GemmArgs g = gemm_args();
        g.A = ain[l]; g.a_mstride = (uint64_t)rows * H; g.lda = H;
        g.B = wbf + woff[l]; g.b_mstride = NBF; g.ldb = H;
        g.M = rows; g.N = H; g.K = H;
        g.bias = params + boff[l]; g.bias_mstride = NPARAM;
        g.zout = zo[l]; g.zout_mstride = (uint64_t)rows * H;
        g.out_bf = aout[l]; g.out_mstride = (uint64_t)rows * H; g.ldc = H;
        e = gemm<EPI_FWD, false, false>(g, (int)nm, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int bm_mlp_workspace_size(uint32_t n_members, uint64_t batch, uint32_t training, size_t *bytes)
{
    int rc = check_members(n_members);
    if (rc) return rc;
    if (!bytes) return fail(BM_ERR_INVALID_ARG, "bytes must not be NULL");
    if (batch < 1 || batch > 0xFFFFFFFFull) return fail(BM_ERR_INVALID_ARG, "batch must be in [1, 2^32 - 1]");
    if (training && (batch % 64 != 0 || batch > 65536))
        return fail(BM_ERR_INVALID_ARG, "training batch must be a multiple of 64 and <= 65536");
    *bytes = mlp_layout(n_members, batch, training != 0).total;
    return ok();
}

extern "C" int bm_mlp_init(uint32_t n_members, uint64_t seed, float *d_params, void *stream)
{
    int rc = check_members(n_members);
    if (rc) return rc;
    if (!d_params) return fail(BM_ERR_INVALID_ARG, "d_params must not be NULL");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const uint64_t total = (uint64_t)n_members * NPARAM;
    hipLaunchKernelGGL(k_init_params, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       d_params, total, (uint32_t)seed, (uint32_t)(seed >> 32));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "bm_mlp_init");
}

extern "C" int bm_mlp_cast(uint32_t n_members, const float *d_params, uint16_t *d_wbf, void *stream)
{
    int rc = check_members(n_members);
    if (rc) return rc;
    if (!d_params || !d_wbf) return fail(BM_ERR_INVALID_ARG, "NULL pointer");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const uint64_t total = (uint64_t)n_members * NPARAM;
    hipLaunchKernelGGL(k_cast, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d_params,
                       (bf16_t *)d_wbf, total);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "bm_mlp_cast");
}

extern "C" int bm_mlp_forward(uint32_t n_members, const float *d_params, const uint16_t *d_wbf, const float *d_x,
                              uint64_t batch, float *d_y, void *d_ws, size_t ws_bytes, void *stream)
{
    int rc = check_members(n_members);
    if (rc) return rc;
    if (!d_params || !d_wbf || !d_x || !d_y) return fail(BM_ERR_INVALID_ARG, "NULL pointer");
    if (batch < 1 || batch > 0xFFFFFFFFull) return fail(BM_ERR_INVALID_ARG, "batch must be in [1, 2^32 - 1]");
    const MlpLayout L = mlp_layout(n_members, batch, false);
    rc = check_ws(L, d_ws, ws_bytes);
    if (rc) return rc;
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_infer, dim3((uint32_t)((batch + FROWS - 1) / FROWS), n_members), dim3(INFER_BT), 0,
                       s, d_x, batch, (const bf16_t *)d_wbf, d_params, d_y, batch);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "bm_mlp_forward");
}

extern "C" int bm_mlp_backward(uint32_t n_members, const float *d_params, const uint16_t *d_wbf, const float *d_x,
                               const float *d_t, const uint32_t *d_idx, uint64_t batch, float *d_grad,
                               float *d_loss, void *d_ws, size_t ws_bytes, void *stream)
{
    int rc = check_members(n_members);
    if (rc) return rc;
    if (!d_params || !d_wbf || !d_x || !d_t || !d_grad) return fail(BM_ERR_INVALID_ARG, "NULL pointer");
    if (batch < 64 || batch % 64 != 0 || batch > 65536)
        return fail(BM_ERR_INVALID_ARG, "training batch must be a multiple of 64 and <= 65536");
    const MlpLayout L = mlp_layout(n_members, batch, true);
    rc = check_ws(L, d_ws, ws_bytes);
    if (rc) return rc;
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_ws;
    const int B = (int)batch;
    const uint32_t nm = n_members;
    const bf16_t *wbf = (const bf16_t *)d_wbf;
    float *u = (float *)(ws + L.u);
    float *z1 = (float *)(ws + L.z1), *z2 = (float *)(ws + L.z2), *z3 = (float *)(ws + L.z3);
    bf16_t *a1 = (bf16_t *)(ws + L.a1), *a2 = (bf16_t *)(ws + L.a2), *a3 = (bf16_t *)(ws + L.a3);
    bf16_t *dz1 = (bf16_t *)(ws + L.dz1), *dz2 = (bf16_t *)(ws + L.dz2), *dz3 = (bf16_t *)(ws + L.dz3);
    float *hpart = (float *)(ws + L.hpart), *red = (float *)(ws + L.red);

    hipError_t e = train_forward(nm, d_params, wbf, d_x, d_idx, batch, B, ws, L, s);
    // output layer, loss, dW4 / db4 and dz3
    const int nhead = B / HEAD_ROWS;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_head, dim3(nhead, nm), dim3(256), 0, s, (const bf16_t *)a3, (const float *)z3, wbf,
                           d_params, d_t, d_idx, batch, B, dz3, hpart);
        hipLaunchKernelGGL(k_head_final, dim3(nm), dim3(256), 0, s, (const float *)hpart, nhead, B, d_grad,
                           d_loss);
        e = hipGetLastError();
    }
    // layers 3 and 2: weight gradients dW = dz^T a_prev, bias gradients, and dz_prev
    const bf16_t *dzs[2] = {dz3, dz2};
    bf16_t *dzp[2] = {dz2, dz1};
    const bf16_t *aprev[2] = {a2, a1};
    const float *zprev[2] = {z2, z1};
    const int woff[2] = {OFF_W3, OFF_W2}, boff[2] = {OFF_B3, OFF_B2}, bwoff[2] = {BOFF_W3, BOFF_W2};
    const int ks = wgrad_split(B);
    float *wpart = (float *)(ws + L.wpart), *bpart = (float *)(ws + L.bpart);
    for (int l = 0; l < 2 && e == hipSuccess; ++l) {
        // dW = dz^T a_prev split over the batch, with the bias gradient (the row sums
        // of dz^T) from the same staged tiles; then the partials added in order
        GemmArgs g = gemm_args();
        g.A = dzs[l]; g.a_mstride = (uint64_t)B * H; g.lda = H;          // (m = out, k = row): dz[k][m]
        g.B = aprev[l]; g.b_mstride = (uint64_t)B * H; g.ldb = H;        // (k = row, n = in): a[k][n]
        g.M = H; g.N = H; g.K = B;
        g.out_f = wpart; g.out_mstride = (uint64_t)H * H; g.ldc = H;
        g.ksplit = ks; g.kchunk = B / ks; g.out_kstride = (uint64_t)nm * H * H;
        g.bias_part = bpart; g.bias_kstride = (uint64_t)nm * H;
        e = gemm<EPI_STORE, true, true>(g, (int)nm, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_wgrad_sum, dim3(H * H / 256 + 1, nm), dim3(256), 0, s, (const float *)wpart,
                           (const float *)bpart, ks, (int)nm, d_grad, woff[l], boff[l]);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        GemmArgs d = gemm_args();
        d.A = dzs[l]; d.a_mstride = (uint64_t)B * H; d.lda = H;          // (m = row, k = out)
        d.B = wbf + bwoff[l]; d.b_mstride = NBF; d.ldb = H;              // (k = out, n = in): W[k][n]
        d.M = B; d.N = H; d.K = H;
        d.zin = zprev[l]; d.zin_mstride = (uint64_t)B * H; d.ldz = H;
        d.out_bf = dzp[l]; d.out_mstride = (uint64_t)B * H; d.ldc = H;
        e = gemm<EPI_DGRAD, false, true>(d, (int)nm, s);
    }
    if (e == hipSuccess) {
        e = colsum(nm, B, dz1, u, red, d_grad, s);
    }
    return e == hipSuccess ? ok() : hip_fail(e, "bm_mlp_backward");
}

extern "C" int bm_mlp_adam_step(uint32_t n_members, float *d_params, const float *d_grad, float *d_m, float *d_v,
                           uint16_t *d_wbf, uint32_t step, float lr, float beta1, float beta2, float eps,
                           void *stream)
{
    int rc = check_members(n_members);
    if (rc) return rc;
    if (!d_params || !d_grad || !d_m || !d_v || !d_wbf) return fail(BM_ERR_INVALID_ARG, "NULL pointer");
    if (step < 1) return fail(BM_ERR_INVALID_ARG, "step counts from 1");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(BM_ERR_INVALID_ARG, "need lr > 0, 0 <= beta < 1, eps > 0");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const uint64_t total = (uint64_t)n_members * NPARAM;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    hipLaunchKernelGGL(k_adam, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d_params,
                       d_grad, d_m, d_v, (bf16_t *)d_wbf, total, lr, beta1, beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "bm_mlp_adam_step");
}

// The kernels of a query: fused inference of every member into y, then mean, std,
// routing flags and per-256-row counts (blk), their exclusive scan and the ordered
// compaction of the routed rows.  Every element of y and blk a call reads is first
// written by that call, so neither buffer needs clearing.
static hipError_t enqueue_query(uint32_t n_members, const float *d_params, const uint16_t *d_wbf, const float *d_x,
                                uint64_t batch, float threshold, float *d_mean, float *d_std,
                                uint32_t *d_fallback_idx, uint32_t *d_fallback_count, float *y, uint32_t *blk,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_infer, dim3((uint32_t)((batch + FROWS - 1) / FROWS), n_members), dim3(INFER_BT), 0,
                       s, d_x, batch, (const bf16_t *)d_wbf, d_params, y, batch);
    hipError_t e = hipGetLastError();
    const uint64_t nblk = (batch + 255) / 256;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_stats, dim3((uint32_t)nblk), dim3(256), 0, s, y, (int)n_members, batch, threshold,
                           d_mean, d_std, blk);
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(256), 0, s, blk, nblk, d_fallback_count);
        hipLaunchKernelGGL(k_compact, dim3((uint32_t)nblk), dim3(256), 0, s, d_std, batch, threshold, blk,
                           d_fallback_idx);
        e = hipGetLastError();
    }
    return e;
}

static int check_query(uint32_t n_members, const float *d_params, const uint16_t *d_wbf, const float *d_x,
                       uint64_t batch, float threshold, float *d_mean, float *d_std, uint32_t *d_fallback_idx,
                       uint32_t *d_fallback_count)
{
    int rc = check_members(n_members);
    if (rc) return rc;
    if (!d_params || !d_wbf || !d_x || !d_mean || !d_std || !d_fallback_idx || !d_fallback_count)
        return fail(BM_ERR_INVALID_ARG, "NULL pointer");
    if (batch < 1 || batch > 0xFFFFFFFFull) return fail(BM_ERR_INVALID_ARG, "batch must be in [1, 2^32 - 1]");
    if (!(threshold >= 0)) return fail(BM_ERR_INVALID_ARG, "threshold must be >= 0");
    return BM_OK;
}

extern "C" int bm_surrogate_query(uint32_t n_members, const float *d_params, const uint16_t *d_wbf,
                                  const float *d_x, uint64_t batch, float threshold, float *d_mean, float *d_std,
                                  uint32_t *d_fallback_idx, uint32_t *d_fallback_count, void *d_ws,
                                  size_t ws_bytes, void *stream)
{
    int rc = check_query(n_members, d_params, d_wbf, d_x, batch, threshold, d_mean, d_std, d_fallback_idx,
                         d_fallback_count);
    if (rc) return rc;
    const MlpLayout L = mlp_layout(n_members, batch, false);
    rc = check_ws(L, d_ws, ws_bytes);
    if (rc) return rc;
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    char *ws = (char *)d_ws;
    const hipError_t e = enqueue_query(n_members, d_params, d_wbf, d_x, batch, threshold, d_mean, d_std,
                                       d_fallback_idx, d_fallback_count, (float *)(ws + L.y),
                                       (uint32_t *)(ws + L.blk), (hipStream_t)stream);
    return e == hipSuccess ? ok() : hip_fail(e, "bm_surrogate_query");
}


// ---------------------------------------------------------------------------
// Ensemble query without a caller workspace and without any allocation: the
// members' predictions and the per-256-row counts live in `scratch`, a file-scope
// device array (one copy per GPU, held until the process ends).  In host code the
// array's name stands for a host-side shadow, so its device address is looked up
// once per device with hipGetSymbolAddress and only that address is ever passed to
// a kernel.  Every element a query reads is first written by the same query, so
// the array needs no clearing between calls.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[BM_QUERY_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[SCRATCH_MAX_DEVICES];     // device address of `scratch` on each device

// Device address of `scratch` on device `dev` (the current device), looked up on the
// first call for that device.
int scratch_address(int dev, char **out)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return fail(BM_ERR_DEVICE, "device index %d beyond the %d the scratch table holds", dev,
                    SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(BM_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        scratch_dev[dev] = p;
    }
    *out = (char *)scratch_dev[dev];
    return BM_OK;
}
} // namespace

extern "C" int bm_surrogate_query_noalloc(uint32_t n_members, const float *d_params, const uint16_t *d_wbf,
                                          const float *d_x, uint64_t batch, float threshold, float *d_mean,
                                          float *d_std, uint32_t *d_fallback_idx, uint32_t *d_fallback_count,
                                          void *stream)
{
    int rc = check_query(n_members, d_params, d_wbf, d_x, batch, threshold, d_mean, d_std, d_fallback_idx,
                         d_fallback_count);
    if (rc) return rc;
    const MlpLayout L = mlp_layout(n_members, batch, false);
    if (L.total > BM_QUERY_SCRATCH_BYTES)
        return fail(BM_ERR_WORKSPACE,
                    "query of %u members x %llu rows needs %zu B of scratch; the built-in scratch holds %zu B "
                    "(use bm_surrogate_query with a workspace)",
                    n_members, (unsigned long long)batch, L.total, (size_t)BM_QUERY_SCRATCH_BYTES);
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    char *ws = nullptr;
    rc = scratch_address(dev, &ws);
    if (rc) return rc;
    const hipError_t e = enqueue_query(n_members, d_params, d_wbf, d_x, batch, threshold, d_mean, d_std,
                                       d_fallback_idx, d_fallback_count, (float *)(ws + L.y),
                                       (uint32_t *)(ws + L.blk), (hipStream_t)stream);
    return e == hipSuccess ? ok() : hip_fail(e, "bm_surrogate_query_noalloc");
}
