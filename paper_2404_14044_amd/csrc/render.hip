// Decode and composite the samples (Sec. 3.4, Eq. 2).
//
// One wave per chunk of RPW consecutive rays.  The wave packs the chunk's
// samples densely into tiles of 16, and for each tile:
//   1. aggregates the features of every sample's K neighbours with
//      inverse-distance weights (FP32): lane l handles sample l % 16 and
//      feature slice 8 (l / 16) .. +8, reading 32 contiguous bytes per neighbour;
//   2. runs the 32 -> 64 -> 64 -> 4 decoder on matrix cores with the sample
//      batch as the N dimension (H^T = W X^T): BF16 operands with
//      v_mfma_f32_16x16x32_bf16, or FP32 operands with v_mfma_f32_16x16x4f32,
//      FP32 accumulation either way.  Each layer's output registers are the
//      next layer's B operand directly: the contraction index is permuted
//      consistently in the weights instead of moving activations;
//   3. stores (sigmoid rgb, softplus sigma) per sample in LDS.
// Then lane r composites ray r of the chunk front to back in FP32.
#include <type_traits>

#include "hp_device.hpp"
#include "hp_kernels.hpp"

namespace hp {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int RPW = 32;  // rays per wave

__device__ __forceinline__ uint32_t bf16_bits_rne(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ bf16x8 pack_bf16x8(const float *v)
{
    union {
        uint32_t u[4];
        bf16x8 b;
    } r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.u[i] = bf16_bits_rne(v[2 * i]) | (bf16_bits_rne(v[2 * i + 1]) << 16);
    return r.b;
}

// Hidden-feature index that lane l's element e feeds at contraction block kb
// of a 64-wide layer input: the previous layer's output block 2 kb + e / 4,
// row 4 (l / 16) + e % 4.
__device__ __forceinline__ int hid_index(int kb, int l, int e)
{
    return 32 * kb + 16 * (e >> 2) + 4 * (l >> 4) + (e & 3);
}

__device__ __forceinline__ float softplus_f(float x)
{
    return __builtin_fmaxf(x, 0.0f) + log1pf(expf(-__builtin_fabsf(x)));
}

__device__ __forceinline__ float sigmoid_f(float x) { return 1.0f / (1.0f + expf(-x)); }

struct Tile {
    int n;         // samples in the tile (<= 16)
    int ray[16];   // chunk-local ray of each sample
};

// Aggregated feature slice (8 floats) of sample `row` for lane slice q.
__device__ __forceinline__ void idw_slice(const RenderArgs &a, int64_t row, int q, float *f)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = 0.0f;
    float wsum = 0.0f;
    for (int k = 0; k < a.K; ++k) {
        const int idx = a.knn_idx[row * a.K + k];
        if (idx < 0) break;
        const float d = a.knn_dist[row * a.K + k];
        const float w = 1.0f / (d > a.eps_idw ? d : a.eps_idw);
        const float4 *src = reinterpret_cast<const float4 *>(a.feat + (int64_t)idx * HP_FEAT_DIM + 8 * q);
        const float4 x0 = src[0], x1 = src[1];
        f[0] = fma_rn(w, x0.x, f[0]);
        f[1] = fma_rn(w, x0.y, f[1]);
        f[2] = fma_rn(w, x0.z, f[2]);
        f[3] = fma_rn(w, x0.w, f[3]);
        f[4] = fma_rn(w, x1.x, f[4]);
        f[5] = fma_rn(w, x1.y, f[5]);
        f[6] = fma_rn(w, x1.z, f[6]);
        f[7] = fma_rn(w, x1.w, f[7]);
        wsum += w;
    }
    const float inv = wsum > 0.0f ? 1.0f / wsum : 0.0f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] *= inv;
}

// ---------------------------------------------------------------------------
// decoder on one tile of 16 samples; returns o[0..3] of sample l (lanes 0..15)
// ---------------------------------------------------------------------------
struct MlpBf16 {
    bf16x8 w1[4];      // [out block]
    bf16x8 w2[4][2];   // [out block][k block]
    bf16x8 w3[2];      // [k block]
    float b1[4][4], b2[4][4], b3[4];
};

__device__ __forceinline__ void load_mlp_bf16(const RenderArgs &a, MlpBf16 &m)
{
    const int l = lane_id();
    const int r = l & 15, q = l >> 4;
    float tmp[8];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
        for (int e = 0; e < 8; ++e) tmp[e] = a.W1[(16 * ob + r) * HP_FEAT_DIM + 8 * q + e];
        m.w1[ob] = pack_bf16x8(tmp);
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
            for (int e = 0; e < 8; ++e) tmp[e] = a.W2[(16 * ob + r) * HP_HIDDEN + hid_index(kb, l, e)];
            m.w2[ob][kb] = pack_bf16x8(tmp);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            m.b1[ob][e] = a.b1[16 * ob + 4 * q + e];
            m.b2[ob][e] = a.b2[16 * ob + 4 * q + e];
        }
    }
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
        for (int e = 0; e < 8; ++e) tmp[e] = (r < 4) ? a.W3[r * HP_HIDDEN + hid_index(kb, l, e)] : 0.0f;
        m.w3[kb] = pack_bf16x8(tmp);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) m.b3[e] = (4 * q + e < 4) ? a.b3[4 * q + e] : 0.0f;
}

__device__ __forceinline__ f32x4 decode_bf16(const MlpBf16 &m, const float *f)
{
    const bf16x8 x = pack_bf16x8(f);
    f32x4 h1[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = {m.b1[ob][0], m.b1[ob][1], m.b1[ob][2], m.b1[ob][3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.w1[ob], x, acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = __builtin_fmaxf(acc[e], 0.0f);
        h1[ob] = acc;
    }
    bf16x8 x2[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        float t8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t8[e] = h1[2 * kb + (e >> 2)][e & 3];
        x2[kb] = pack_bf16x8(t8);
    }
    f32x4 h2[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = {m.b2[ob][0], m.b2[ob][1], m.b2[ob][2], m.b2[ob][3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.w2[ob][0], x2[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.w2[ob][1], x2[1], acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = __builtin_fmaxf(acc[e], 0.0f);
        h2[ob] = acc;
    }
    bf16x8 x3[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        float t8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t8[e] = h2[2 * kb + (e >> 2)][e & 3];
        x3[kb] = pack_bf16x8(t8);
    }
    f32x4 o = {m.b3[0], m.b3[1], m.b3[2], m.b3[3]};
    o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.w3[0], x3[0], o, 0, 0, 0);
    o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.w3[1], x3[1], o, 0, 0, 0);
    return o;
}

// FP32: v_mfma_f32_16x16x4f32, lane l supplies contraction row l / 16 of
// each 4-deep step.  Layer 1 step ks takes feature 8 (l / 16) + ks; layer 2
// and 3 step (ob, e) take hidden feature 16 ob + 4 (l / 16) + e.
struct MlpF32 {
    float w1[4][8];    // [out block][step]
    float w2[4][16];   // [out block][step]
    float w3[16];
    float b1[4][4], b2[4][4], b3[4];
};

__device__ __forceinline__ void load_mlp_f32(const RenderArgs &a, MlpF32 &m)
{
    const int l = lane_id();
    const int r = l & 15, q = l >> 4;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) m.w1[ob][ks] = a.W1[(16 * ob + r) * HP_FEAT_DIM + 8 * q + ks];
#pragma unroll
        for (int st = 0; st < 16; ++st)
            m.w2[ob][st] = a.W2[(16 * ob + r) * HP_HIDDEN + 16 * (st >> 2) + 4 * q + (st & 3)];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            m.b1[ob][e] = a.b1[16 * ob + 4 * q + e];
            m.b2[ob][e] = a.b2[16 * ob + 4 * q + e];
        }
    }
#pragma unroll
    for (int st = 0; st < 16; ++st)
        m.w3[st] = (r < 4) ? a.W3[r * HP_HIDDEN + 16 * (st >> 2) + 4 * q + (st & 3)] : 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) m.b3[e] = (4 * q + e < 4) ? a.b3[4 * q + e] : 0.0f;
}

__device__ __forceinline__ f32x4 decode_f32(const MlpF32 &m, const float *f)
{
    f32x4 h1[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = {m.b1[ob][0], m.b1[ob][1], m.b1[ob][2], m.b1[ob][3]};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(m.w1[ob][ks], f[ks], acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = __builtin_fmaxf(acc[e], 0.0f);
        h1[ob] = acc;
    }
    f32x4 h2[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = {m.b2[ob][0], m.b2[ob][1], m.b2[ob][2], m.b2[ob][3]};
#pragma unroll
        for (int st = 0; st < 16; ++st)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(m.w2[ob][st], h1[st >> 2][st & 3], acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = __builtin_fmaxf(acc[e], 0.0f);
        h2[ob] = acc;
    }
    f32x4 o = {m.b3[0], m.b3[1], m.b3[2], m.b3[3]};
#pragma unroll
    for (int st = 0; st < 16; ++st)
        o = __builtin_amdgcn_mfma_f32_16x16x4f32(m.w3[st], h2[st >> 2][st & 3], o, 0, 0, 0);
    return o;
}

template <int PREC>
__global__ void __launch_bounds__(WAVE) k_render(RenderArgs a)
{
    extern __shared__ float4 sh_out[];  // [RPW * S] (rgb, sigma) per sample
    __shared__ int sh_pre[RPW + 1];
    const int l = lane_id();
    const int64_t ray0 = (int64_t)blockIdx.x * RPW;
    if (ray0 >= a.n_rays) return;
    const int nr = (a.n_rays - ray0) < RPW ? (int)(a.n_rays - ray0) : RPW;

    // prefix of sample counts over the chunk
    const int ns = (l < nr) ? a.n_sel[ray0 + l] : 0;
    const int inc = wave_incl_scan_i32(ns);
    if (l < RPW) sh_pre[l] = inc - ns;
    const int total = readlane_i32(inc, WAVE - 1);
    if (l == 0) sh_pre[RPW] = total;
    __syncthreads();

    if (total > 0) {
        typename std::conditional<PREC == HP_BF16, MlpBf16, MlpF32>::type mlp;
        if constexpr (PREC == HP_BF16) load_mlp_bf16(a, mlp);
        else load_mlp_f32(a, mlp);
        const int r16 = l & 15, q = l >> 4;
        for (int s0 = 0; s0 < total; s0 += 16) {
            const int sidx = s0 + r16;
            const bool valid = sidx < total;
            float f[8];
            int cr = 0, cs = 0;
            if (valid) {
                int lo = 0, hi = nr;  // chunk-local ray: last with pre <= sidx
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (sh_pre[mid] <= sidx) lo = mid;
                    else hi = mid;
                }
                cr = lo;
                cs = sidx - sh_pre[lo];
                idw_slice(a, (ray0 + cr) * a.S + cs, q, f);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) f[e] = 0.0f;
            }
            f32x4 o;
            if constexpr (PREC == HP_BF16) o = decode_bf16(mlp, f);
            else o = decode_f32(mlp, f);
            if (q == 0 && valid)
                sh_out[sidx] = make_float4(sigmoid_f(o[0]), sigmoid_f(o[1]), sigmoid_f(o[2]),
                                           softplus_f(o[3]));
        }
    }
    __syncthreads();
    if (l < nr) {
        const int64_t ray = ray0 + l;
        const int base = sh_pre[l];
        float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, dep = 0.0f, ws = 0.0f;
        for (int s = 0; s < ns; ++s) {
            const float4 v = sh_out[base + s];
            const float t = a.t[ray * a.S + s];
            const float delta = (s + 1 < ns) ? a.t[ray * a.S + s + 1] - t : a.delta_last;
            const float e = expf(-v.w * delta);
            const float w = T * (1.0f - e);
            cr = fma_rn(w, v.x, cr);
            cg = fma_rn(w, v.y, cg);
            cb = fma_rn(w, v.z, cb);
            dep = fma_rn(w, t, dep);
            ws += w;
            T *= e;
        }
        const float rest = 1.0f - ws;
        a.rgb[3 * ray + 0] = fma_rn(rest, a.bg[0], cr);
        a.rgb[3 * ray + 1] = fma_rn(rest, a.bg[1], cg);
        a.rgb[3 * ray + 2] = fma_rn(rest, a.bg[2], cb);
        if (a.depth) a.depth[ray] = dep;
        if (a.acc) a.acc[ray] = ws;
    }
}

hipError_t launch_render(const RenderArgs &a, int precision, hipStream_t s)
{
    const int64_t blocks = (a.n_rays + RPW - 1) / RPW;
    if (blocks == 0) return hipSuccess;
    const size_t shmem = (size_t)RPW * a.S * sizeof(float4);
    if (precision == HP_BF16)
        k_render<HP_BF16><<<dim3((unsigned)blocks), dim3(WAVE), shmem, s>>>(a);
    else
        k_render<HP_FP32><<<dim3((unsigned)blocks), dim3(WAVE), shmem, s>>>(a);
    return hipGetLastError();
}

}  // namespace hp
