// mlp_kernels.hpp -- ensemble MLP surrogate for <v>(a, omega, F, D, gamma):
// members of 5 -> 256 -> 256 -> 256 -> 1 with tanh-GELU, BF16 weights and FP32
// accumulation.  The two 256 x 256 layers (99% of the work) run on
// v_mfma_f32_16x16x32_bf16 through one LDS-tiled GEMM with fused epilogues;
// the 5-input and 1-output layers are FP32 FMA kernels on the same BF16 weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bm {
namespace mlp {

constexpr int IN = 5;
constexpr int H = 256;
// FP32 parameter block of one member (row-major [out][in] weights):
constexpr int OFF_W1 = 0;                 // [256][5]
constexpr int OFF_B1 = OFF_W1 + H * IN;   // [256]
constexpr int OFF_W2 = OFF_B1 + H;        // [256][256]
constexpr int OFF_B2 = OFF_W2 + H * H;    // [256]
constexpr int OFF_W3 = OFF_B2 + H;        // [256][256]
constexpr int OFF_B3 = OFF_W3 + H * H;    // [256]
constexpr int OFF_W4 = OFF_B3 + H;        // [256]
constexpr int OFF_B4 = OFF_W4 + H;        // [1]
constexpr int NPARAM = OFF_B4 + 1;        // 133377
// BF16 weight block of one member: W1 | W2 | W3 | W4 (biases stay FP32)
constexpr int BOFF_W1 = 0;
constexpr int BOFF_W2 = BOFF_W1 + H * IN;
constexpr int BOFF_W3 = BOFF_W2 + H * H;
constexpr int BOFF_W4 = BOFF_W3 + H * H;
constexpr int NBF = BOFF_W4 + H;          // 132608

typedef uint16_t bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ bf16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (bf16_t)((u >> 16) | 0x0040u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float((uint32_t)b << 16); }

// tanh-GELU: 0.5 z (1 + tanh u), u = c (z + 0.044715 z^3), c = sqrt(2 / pi).
// Since 0.5 (1 + tanh u) = 1 / (1 + e^{-2u}), gelu = z sigma with
// sigma = 1 / (1 + 2^{-2 c log2(e) z (1 + 0.044715 z^2)}) on the hardware exp2 and
// reciprocal (1 ulp each); sigma saturates to 0 / 1 for large |u|.  t = tanh u.
__device__ __forceinline__ float gelu_t(float z, float &t)
{
    const float k = -2.0f * 0.7978845608028654f * 1.4426950408889634f;   // -2 c log2(e)
    const float w = z * fmaf(k * 0.044715f, z * z, k);
    const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(w));
    t = fmaf(2.0f, sg, -1.0f);
    return z * sg;
}
__device__ __forceinline__ float gelu(float z)
{
    float t;
    return gelu_t(z, t);
}
// d gelu / dz = 0.5 (1 + t) + 0.5 z (1 - t^2) c (1 + 3 * 0.044715 z^2)
__device__ __forceinline__ float gelu_grad(float z)
{
    float t;
    (void)gelu_t(z, t);
    const float c = 0.7978845608028654f;
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * c * fmaf(0.134145f, z * z, 1.0f);
}

// Input normalisation to [-1, 1] over the surrogate's domain:
// a in [0, 8], omega in [1, 10], F in [-0.5, 0.5], log10 D in [-4, -1], gamma in [0.5, 2].
__device__ __forceinline__ void normalise(const float *x, float u[IN])
{
    u[0] = x[0] * 0.25f - 1.0f;
    u[1] = (x[1] - 5.5f) * (1.0f / 4.5f);
    u[2] = x[2] * 2.0f;
    u[3] = (log10f(x[3]) + 2.5f) * (1.0f / 1.5f);
    u[4] = (x[4] - 1.25f) * (1.0f / 0.75f);
}

// ---------------------------------------------------------------------------
// GEMM  C[M x N] = A[M x K] * B[K x N], BF16 in, FP32 accumulate, per member
// (blockIdx.z selects the member through the *_mstride element strides).
//   A: TA = false -> element (m, k) at A[m * lda + k];  TA = true -> A[k * lda + m]
//   B: TB = false -> element (k, n) at B[n * ldb + k];  TB = true -> B[k * ldb + n]
// Tiles 64 x 64 x TKT, 256 lanes = 4 waves, each wave 32 x 32 = 2 x 2 MFMA tiles.
// Requirements (checked on the host): N % 64 == 0, K % TKT == 0, 16-byte aligned
// rows (lda, ldb multiples of 8).  M is arbitrary (rows >= M read as 0, not stored).
// ---------------------------------------------------------------------------
enum Epi : int {
    EPI_FWD = 0,       // z = acc + bias[n]; a = gelu(z) -> BF16 out (+ FP32 z if zout)
    EPI_DGRAD = 1,     // dz = acc * gelu'(z[m][n]) -> BF16 out
    EPI_STORE = 2,     // FP32 out = acc
};

struct GemmArgs {
    const bf16_t *A; const bf16_t *B;
    uint64_t a_mstride, b_mstride;        // element strides between members
    int M, N, K, lda, ldb;
    const float *bias; uint64_t bias_mstride;
    const float *zin; uint64_t zin_mstride; int ldz;    // EPI_DGRAD: z (FP32, [M][ldz])
    float *zout; uint64_t zout_mstride;                 // EPI_FWD: optional z out ([M][ldc])
    bf16_t *out_bf; float *out_f; uint64_t out_mstride; int ldc;
    // split K (EPI_STORE): blockIdx.z = member * ksplit + kc covers k in
    // [kc kchunk, (kc + 1) kchunk) and stores its partial at out_f + kc out_kstride;
    // with bias_part, the work-groups of the first column tile also store the row
    // sums of their A range, sum_k A(m, k), at bias_part[kc bias_kstride + member H + m]
    // (TA only).  ksplit 0 or 1: the whole K in one work-group.
    int ksplit, kchunk;
    uint64_t out_kstride;
    float *bias_part; uint64_t bias_kstride;
};

constexpr int TM = 64, TN = 64, TK = 32;

// TKT: k extent of the tiles staged per barrier (a multiple of 32 dividing K, or the
// split's kchunk): 32 keeps 10 KiB of LDS per work-group; 128 halves the barriers
// and global-load round trips four times over for the K = 256 layers.
template <int EPI, bool TA, bool TB, int TKT = TK>
__global__ void __launch_bounds__(256) k_gemm(const GemmArgs g)
{
    constexpr int LK = TKT + 8;          // padded row of a staged tile (bf16)
    constexpr int KS = TKT / 32;         // 32-wide k slices per staged tile
    __shared__ __align__(16) bf16_t sA[TM * LK];
    __shared__ __align__(16) bf16_t sB[TN * LK];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int ks = g.ksplit > 1 ? g.ksplit : 1;
    const int kc = (int)blockIdx.z % ks, mem = (int)blockIdx.z / ks;
    const int kbeg = ks > 1 ? kc * g.kchunk : 0, kend = ks > 1 ? kbeg + g.kchunk : g.K;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const bool rowsum = TA && EPI == EPI_STORE && g.bias_part != nullptr && blockIdx.x == 0;
    float bsum = 0.0f;
    const bf16_t *A = g.A + g.a_mstride * mem;
    const bf16_t *B = g.B + g.b_mstride * mem;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    // LDS tiles are row-major (row = m of A, n of B) with k along the row; the
    // 16-byte units of 8 k are XOR-swizzled by the row's group of 8, so that the
    // transposing writes below spread over all banks (the fragment reads stay
    // conflict-free: a unit is still read whole).
    auto lds = [](int row, int k) { return row * LK + ((((k >> 3) ^ ((row >> 3) & (TKT / 8 - 1)))) << 3) + (k & 7); };
    for (int k0 = kbeg; k0 < kend; k0 += TKT) {
        // ---- stage A (64 x TKT) and B (TKT x 64, stored n-major) ----
        // An operand whose rows run along k arrives in 16-byte units of 8 k: thread t
        // loads unit t % 4 of row t / 4 for each 32-wide k slice.  A transposed operand
        // (rows along m or n) arrives in units of 8 rows at one k: with TKT >= 64 thread
        // t loads rows 8 (t % 8) .. + 7 at the KS consecutive k = KS (t / 8) + r and
        // writes them transposed (KS k of a row in one write), else one k per thread
        // and eight 2-byte writes.
        uint4 va[KS], vb[KS];
#pragma unroll
        for (int sl = 0; sl < KS; ++sl) {
            const int kb = k0 + 32 * sl;
            va[sl] = make_uint4(0u, 0u, 0u, 0u);
            if (!TA) {
                const int r = t >> 2, kq = (t & 3) * 8;
                if (m0 + r < g.M) va[sl] = *reinterpret_cast<const uint4 *>(A + (uint64_t)(m0 + r) * g.lda + kb + kq);
            } else {
                const int kk = KS > 1 ? KS * (t >> 3) + sl : (t >> 3), mc = (t & 7) * 8;
                if (m0 + mc < g.M)
                    va[sl] = *reinterpret_cast<const uint4 *>(A + (uint64_t)(KS > 1 ? k0 + kk : kb + kk) * g.lda + m0 + mc);
            }
            if (!TB) {
                const int c = t >> 2, kq = (t & 3) * 8;
                vb[sl] = *reinterpret_cast<const uint4 *>(B + (uint64_t)(n0 + c) * g.ldb + kb + kq);
            } else {
                const int kk = KS > 1 ? KS * (t >> 3) + sl : (t >> 3), nc = (t & 7) * 8;
                vb[sl] = *reinterpret_cast<const uint4 *>(B + (uint64_t)(KS > 1 ? k0 + kk : kb + kk) * g.ldb + n0 + nc);
            }
        }
        // rows 8 (t % 8) + i of a transposed operand, k = KS (t / 8) .. + KS - 1
        auto put_transposed = [&](bf16_t *sT, const uint4 (&v)[KS]) {
            const int rc = (t & 7) * 8, kq = KS * (t >> 3);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                uint32_t w[KS / 2 > 0 ? KS / 2 : 1];
#pragma unroll
                for (int r = 0; r < KS / 2; ++r) {
                    // element i of k = kq + 2r (low half) and of k = kq + 2r + 1 (high half)
                    const uint32_t lo = reinterpret_cast<const uint32_t *>(&v[2 * r])[i >> 1];
                    const uint32_t hi = reinterpret_cast<const uint32_t *>(&v[2 * r + 1])[i >> 1];
                    w[r] = (i & 1) ? ((lo >> 16) | (hi & 0xFFFF0000u)) : ((lo & 0xFFFFu) | (hi << 16));
                }
                if constexpr (KS == 4)
                    *reinterpret_cast<uint2 *>(&sT[lds(rc + i, kq)]) = uint2{w[0], w[1]};
                else
                    *reinterpret_cast<uint32_t *>(&sT[lds(rc + i, kq)]) = w[0];
            }
        };
        if constexpr (TA && KS > 1) {
            put_transposed(sA, va);
        } else {
#pragma unroll
            for (int sl = 0; sl < KS; ++sl) {
                if (!TA) {
                    const int r = t >> 2, kq = (t & 3) * 8;
                    *reinterpret_cast<uint4 *>(&sA[lds(r, 32 * sl + kq)]) = va[sl];
                } else {
                    const int kk = t >> 3, mc = (t & 7) * 8;
                    const bf16_t *e = reinterpret_cast<const bf16_t *>(&va[sl]);
#pragma unroll
                    for (int i = 0; i < 8; ++i) sA[lds(mc + i, 32 * sl + kk)] = e[i];
                }
            }
        }
        if constexpr (TB && KS > 1) {
            put_transposed(sB, vb);
        } else {
#pragma unroll
            for (int sl = 0; sl < KS; ++sl) {
                if (!TB) {
                    const int c = t >> 2, kq = (t & 3) * 8;
                    *reinterpret_cast<uint4 *>(&sB[lds(c, 32 * sl + kq)]) = vb[sl];
                } else {
                    const int kk = t >> 3, nc = (t & 7) * 8;
                    const bf16_t *e = reinterpret_cast<const bf16_t *>(&vb[sl]);
#pragma unroll
                    for (int i = 0; i < 8; ++i) sB[lds(nc + i, 32 * sl + kk)] = e[i];
                }
            }
        }
        __syncthreads();
        // ---- 2 x 2 MFMA 16x16x32 per wave and k slice: lane holds row/col lane%16,
        //      k 8*(lane/16).. of the slice ----
        const int fr = lane & 15, fk = (lane >> 4) * 8;
#pragma unroll
        for (int sl = 0; sl < KS; ++sl) {
            bf16x8 af[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                af[i] = *reinterpret_cast<const bf16x8 *>(&sA[lds(wm + 16 * i + fr, 32 * sl + fk)]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8 *>(&sB[lds(wn + 16 * j + fr, 32 * sl + fk)]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        if (rowsum) {                    // row t/4 of the A tile, a quarter of its k
#pragma unroll
            for (int i = 0; i < TKT / 4; ++i) bsum += bf2f(sA[lds(t >> 2, (t & 3) * (TKT / 4) + i)]);
        }
        __syncthreads();
    }
    if (rowsum) {
        bsum += __shfl_xor(bsum, 1, 64);
        bsum += __shfl_xor(bsum, 2, 64);
        if ((t & 3) == 0 && m0 + (t >> 2) < g.M)
            g.bias_part[(uint64_t)kc * g.bias_kstride + (uint64_t)mem * H + m0 + (t >> 2)] = bsum;
    }

    // ---- epilogue: acc[i][j][e] is C[row 4*(lane/16)+e][col lane%16] of tile (i, j) ----
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + 16 * j + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
                if (m >= g.M) continue;
                const float v = acc[i][j][e];
                const uint64_t o = g.out_kstride * kc + g.out_mstride * mem + (uint64_t)m * g.ldc + n;
                if constexpr (EPI == EPI_FWD) {
                    const float z = v + g.bias[g.bias_mstride * mem + n];
                    if (g.zout) g.zout[g.zout_mstride * mem + (uint64_t)m * g.ldc + n] = z;
                    g.out_bf[o] = f2bf(gelu(z));
                } else if constexpr (EPI == EPI_DGRAD) {
                    const float z = g.zin[g.zin_mstride * mem + (uint64_t)m * g.ldz + n];
                    g.out_bf[o] = f2bf(v * gelu_grad(z));
                } else {
                    g.out_f[o] = v;
                }
            }
        }
    }
}

} // namespace mlp
} // namespace bm
