// Gradient of the render (Sec. 3.4, Eq. 2) with respect to the point
// features and the decoder parameters.
//
// One 64-lane workgroup per ray, persistent over rays like the forward search.
// For each ray the search and the primary-surface sampling are recomputed
// from the table (samples depend on geometry only), the decoder is replayed
// (BF16 or FP32 on MFMA) to recover its activations, and the gradient flows
//   compositing (sequential, FP32) -> decoder outputs
//   decoder backward (FP32, VALU; weights FP32)   -> aggregated features
//   inverse-distance aggregation                   -> point features (atomics)
// Decoder-parameter gradients are accumulated per workgroup in registers and
// written to a per-workgroup slice of the workspace; a second kernel sums the
// slices in a fixed order into the caller's gradient arrays.
#include <type_traits>

#include "hp_backward.hpp"

namespace hp {

constexpr int NPAR = HP_HIDDEN * HP_FEAT_DIM + HP_HIDDEN + HP_HIDDEN * HP_HIDDEN + HP_HIDDEN +
                     4 * HP_HIDDEN + 4;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + HP_HIDDEN * HP_FEAT_DIM;
constexpr int OFF_W2 = OFF_B1 + HP_HIDDEN;
constexpr int OFF_B2 = OFF_W2 + HP_HIDDEN * HP_HIDDEN;
constexpr int OFF_W3 = OFF_B2 + HP_HIDDEN;
constexpr int OFF_B3 = OFF_W3 + 4 * HP_HIDDEN;
constexpr int BWD_BLOCKS = 2048;

template <int KT>
struct BwdLds {
    SearchLds s;
    float smp_t[HP_MAX_SAMPLES];
    int32_t smp_idx[HP_MAX_SAMPLES][KT];
    float smp_dist[HP_MAX_SAMPLES][KT];
    float O[HP_MAX_SAMPLES][4];    // decoder outputs
    float DO[HP_MAX_SAMPLES][4];   // dL/d(decoder outputs)
    float F[16][HP_FEAT_DIM];      // tile: aggregated features
    float H1[16][HP_HIDDEN];       // tile: layer-1 activations, then their gradients
    float H2[16][HP_HIDDEN];       // tile: layer-2 activations, then their gradients
    float gpar[NPAR];              // this workgroup's decoder-parameter gradients
};

// Aggregated feature slice (8 floats, features 8 q .. 8 q + 7) of sample s.
template <int KT>
__device__ __forceinline__ void idw_slice_lds(const BwdLds<KT> &sh, const float *feat, int K,
                                              float eps_idw, int s, int q, float *f)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = 0.0f;
    float wsum = 0.0f;
    for (int k = 0; k < K; ++k) {
        const int idx = sh.smp_idx[s][k];
        if (idx < 0) break;
        const float d = sh.smp_dist[s][k];
        const float w = 1.0f / (d > eps_idw ? d : eps_idw);
        const float4 *src = reinterpret_cast<const float4 *>(feat + (int64_t)idx * HP_FEAT_DIM + 8 * q);
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

template <int KT, int PREC>
__device__ __forceinline__ void backward_body(const BwdArgs &A)
{
    __shared__ BwdLds<KT> sh;
    const SearchCtx &c = A.c;
    const int l = lane_id();
    const int r16 = l & 15, q = l >> 4;

    using Mlp = typename std::conditional<PREC == HP_BF16, MlpBf16, MlpF32>::type;
    auto load_mlp = [&](Mlp &m) {
        if constexpr (PREC == HP_BF16) load_mlp_bf16(A.w, m);
        else load_mlp_f32(A.w, m);
    };
    // decoder-parameter gradients: lane l owns column l of dW2 and dW3, rows
    // 32 (l >> 5) .. +31 of column l & 31 of dW1, and entry l of db1, db2
    for (int i = l; i < NPAR; i += WAVE) sh.gpar[i] = 0.0f;
    float gW3[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f;

    const int64_t n_chunks = (c.n_rays + c.chunk - 1) / c.chunk;
    for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
        const int64_t r1 = min((ch + 1) * c.chunk, c.n_rays);
        for (int64_t ray = ch * c.chunk; ray < r1; ++ray) {
            const float g0 = A.grad_rgb[3 * ray], g1 = A.grad_rgb[3 * ray + 1],
                        g2 = A.grad_rgb[3 * ray + 2];
            if (g0 == 0.0f && g1 == 0.0f && g2 == 0.0f) continue;  // no gradient through this ray
            const RayGeom g = ray_geometry(c, ray);
            uint64_t top;
            int count;
            search_neighbours(c, g, sh.s, top, count);
            const int m = count < c.M ? count : c.M;
            int prim;
            const int n = walk_candidates<KT>(
                c, g, sh.s, top, m, prim,
                [&](int s, int qq, float tj, const uint64_t(&kd)[KT], int kc) {
                    if (qq == 0) sh.smp_t[s] = tj;
#pragma unroll
                    for (int k = 0; k < KT; ++k) {
                        if ((k & 3) == qq) {
                            const bool v = k < kc;
                            sh.smp_idx[s][k] = v ? (int32_t)(uint32_t)kd[k] : -1;
                            sh.smp_dist[s][k] =
                                v ? __builtin_sqrtf(__uint_as_float((uint32_t)(kd[k] >> 32))) : 0.0f;
                        }
                    }
                });
            lds_sync();
            if (n == 0) continue;

            // pass A: decoder outputs of every sample
            Mlp mlp;
            load_mlp(mlp);
            for (int t0 = 0; t0 < n; t0 += 16) {
                const int s = t0 + r16;
                float f[8];
                if (s < n) idw_slice_lds(sh, A.feat, c.K, A.eps_idw, s, q, f);
                else
#pragma unroll
                    for (int e = 0; e < 8; ++e) f[e] = 0.0f;
                f32x4 o;
                if constexpr (PREC == HP_BF16) o = decode_bf16(mlp, f);
                else o = decode_f32(mlp, f);
                if (q == 0 && s < n) {
                    sh.O[s][0] = o[0];
                    sh.O[s][1] = o[1];
                    sh.O[s][2] = o[2];
                    sh.O[s][3] = o[3];
                }
            }
            lds_sync();

            // compositing backward (Eq. 2), sequential in sample order
            if (l == 0) {
                float T = 1.0f;
                float *Ts = &sh.F[0][0];  // scratch until pass B
                for (int j = 0; j < n; ++j) {
                    Ts[j] = T;
                    const float sg = softplus_f(sh.O[j][3]);
                    const float dl = (j + 1 < n) ? sh.smp_t[j + 1] - sh.smp_t[j] : A.delta_last;
                    T *= expf(-sg * dl);
                }
                float U0 = 0.0f, U1 = 0.0f, U2 = 0.0f, P = 1.0f;
                for (int j = n - 1; j >= 0; --j) {
                    const float c0 = sigmoid_f(sh.O[j][0]), c1 = sigmoid_f(sh.O[j][1]),
                                c2 = sigmoid_f(sh.O[j][2]);
                    const float sg = softplus_f(sh.O[j][3]);
                    const float dl = (j + 1 < n) ? sh.smp_t[j + 1] - sh.smp_t[j] : A.delta_last;
                    const float e = expf(-sg * dl);
                    const float a = 1.0f - e;
                    const float Tj = Ts[j];
                    const float dLda = g0 * (Tj * (c0 - U0) - A.bg[0] * Tj * P) +
                                       g1 * (Tj * (c1 - U1) - A.bg[1] * Tj * P) +
                                       g2 * (Tj * (c2 - U2) - A.bg[2] * Tj * P);
                    const float ws = Tj * a;
                    sh.DO[j][0] = g0 * ws * c0 * (1.0f - c0);
                    sh.DO[j][1] = g1 * ws * c1 * (1.0f - c1);
                    sh.DO[j][2] = g2 * ws * c2 * (1.0f - c2);
                    sh.DO[j][3] = dLda * dl * e * sigmoid_f(sh.O[j][3]);
                    U0 = a * c0 + e * U0;
                    U1 = a * c1 + e * U1;
                    U2 = a * c2 + e * U2;
                    P = e * P;
                }
            }
            lds_sync();

            // pass B: per tile, replay the decoder keeping activations, then backward
            for (int t0 = 0; t0 < n; t0 += 16) {
                const int nt = min(16, n - t0);
                {
                    const int s = t0 + r16;
                    float f[8];
                    if (s < n) idw_slice_lds(sh, A.feat, c.K, A.eps_idw, s, q, f);
                    else
#pragma unroll
                        for (int e = 0; e < 8; ++e) f[e] = 0.0f;
                    f32x4 h1[4], h2[4];
                    Mlp mlp2;
                    load_mlp(mlp2);
                    if constexpr (PREC == HP_BF16) decode_bf16(mlp2, f, h1, h2);
                    else decode_f32(mlp2, f, h1, h2);
#pragma unroll
                    for (int e = 0; e < 8; ++e) sh.F[r16][8 * q + e] = f[e];
#pragma unroll
                    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            sh.H1[r16][16 * ob + 4 * q + e] = h1[ob][e];
                            sh.H2[r16][16 * ob + 4 * q + e] = h2[ob][e];
                        }
                }
                lds_sync();
                // output layer: lane l is hidden unit l of layer 2
                {
                    const float w30 = A.w.W3[0 * HP_HIDDEN + l], w31 = A.w.W3[1 * HP_HIDDEN + l],
                                w32 = A.w.W3[2 * HP_HIDDEN + l], w33 = A.w.W3[3 * HP_HIDDEN + l];
                    for (int s = 0; s < nt; ++s) {
                        const float d0 = sh.DO[t0 + s][0], d1 = sh.DO[t0 + s][1],
                                    d2 = sh.DO[t0 + s][2], d3 = sh.DO[t0 + s][3];
                        const float h = sh.H2[s][l];
                        gW3[0] = fma_rn(d0, h, gW3[0]);
                        gW3[1] = fma_rn(d1, h, gW3[1]);
                        gW3[2] = fma_rn(d2, h, gW3[2]);
                        gW3[3] = fma_rn(d3, h, gW3[3]);
                        float dp = w30 * d0;
                        dp = fma_rn(w31, d1, dp);
                        dp = fma_rn(w32, d2, dp);
                        dp = fma_rn(w33, d3, dp);
                        const float dh = h > 0.0f ? dp : 0.0f;
                        sh.H2[s][l] = dh;  // activation no longer needed
                        gb2 += dh;
                        if (l < 4) gb3 += sh.DO[t0 + s][l];
                    }
                }
                lds_sync();
                // hidden layer 2 -> 1: lane l is hidden unit l of layer 1
                {
                    float acc[16];
                    float h1v[16];
#pragma unroll
                    for (int s = 0; s < 16; ++s) {
                        acc[s] = 0.0f;
                        h1v[s] = (s < nt) ? sh.H1[s][l] : 0.0f;
                    }
#pragma unroll 4
                    for (int o2 = 0; o2 < HP_HIDDEN; ++o2) {
                        const float w = A.w.W2[o2 * HP_HIDDEN + l];
                        float gw = 0.0f;
#pragma unroll
                        for (int s = 0; s < 16; ++s) {
                            const float d = (s < nt) ? sh.H2[s][o2] : 0.0f;
                            acc[s] = fma_rn(w, d, acc[s]);
                            gw = fma_rn(d, h1v[s], gw);
                        }
                        sh.gpar[OFF_W2 + o2 * HP_HIDDEN + l] += gw;
                    }
#pragma unroll
                    for (int s = 0; s < 16; ++s) {
                        const float dh = (s < nt && h1v[s] > 0.0f) ? acc[s] : 0.0f;
                        if (s < nt) sh.H1[s][l] = dh;
                        gb1 += dh;
                    }
                }
                lds_sync();
                // layer 1 -> aggregated features, and dW1
                {
                    const int cc = l & 31, half = l >> 5;
                    float df[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) df[i] = 0.0f;
#pragma unroll 4
                    for (int i = 0; i < HP_HIDDEN; ++i) {
                        const float w = A.w.W1[i * HP_FEAT_DIM + cc];
#pragma unroll
                        for (int si = 0; si < 8; ++si) {
                            const int s = 8 * half + si;
                            df[si] = fma_rn(w, (s < nt) ? sh.H1[s][i] : 0.0f, df[si]);
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 32; ++i) {
                        float gw = 0.0f;
                        for (int s = 0; s < nt; ++s) gw = fma_rn(sh.H1[s][32 * half + i], sh.F[s][cc], gw);
                        sh.gpar[OFF_W1 + (32 * half + i) * HP_FEAT_DIM + cc] += gw;
                    }
                    // aggregation backward: d feat[idx_k][cc] += (w_k / sum w) df
#pragma unroll
                    for (int si = 0; si < 8; ++si) {
                        const int s = 8 * half + si;
                        if (s >= nt) break;
                        float wsum = 0.0f;
                        for (int k = 0; k < c.K; ++k) {
                            if (sh.smp_idx[t0 + s][k] < 0) break;
                            const float d = sh.smp_dist[t0 + s][k];
                            wsum += 1.0f / (d > A.eps_idw ? d : A.eps_idw);
                        }
                        const float inv = 1.0f / wsum;
                        for (int k = 0; k < c.K; ++k) {
                            const int idx = sh.smp_idx[t0 + s][k];
                            if (idx < 0) break;
                            const float d = sh.smp_dist[t0 + s][k];
                            const float wk = (1.0f / (d > A.eps_idw ? d : A.eps_idw)) * inv;
                            atomicAdd(&A.grad_feat[(int64_t)idx * HP_FEAT_DIM + cc], wk * df[si]);
                        }
                    }
                }
                lds_sync();
            }
        }
    }

    // this workgroup's parameter gradients -> its workspace slice
#pragma unroll
    for (int k = 0; k < 4; ++k) sh.gpar[OFF_W3 + k * HP_HIDDEN + l] = gW3[k];
    sh.gpar[OFF_B1 + l] = gb1;
    sh.gpar[OFF_B2 + l] = gb2;
    if (l < 4) sh.gpar[OFF_B3 + l] = gb3;
    lds_sync();
    float *P = A.partial + (int64_t)blockIdx.x * NPAR;
    for (int i = l; i < NPAR; i += WAVE) P[i] = sh.gpar[i];
}

template <int KT, int PREC>
__global__ void __launch_bounds__(WAVE) k_render_backward(BwdArgs A)
{
    backward_body<KT, PREC>(A);
}

// Sum the per-workgroup slices in workgroup order and add to the gradients.
__global__ void __launch_bounds__(256) k_reduce_partials(const float *__restrict__ partial, int nblk,
                                                         float *gW1, float *gb1, float *gW2,
                                                         float *gb2, float *gW3, float *gb3)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAR) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * NPAR + i];
    float *dst;
    int j;
    if (i < OFF_B1) { dst = gW1; j = i - OFF_W1; }
    else if (i < OFF_W2) { dst = gb1; j = i - OFF_B1; }
    else if (i < OFF_B2) { dst = gW2; j = i - OFF_W2; }
    else if (i < OFF_W3) { dst = gb2; j = i - OFF_B2; }
    else if (i < OFF_B3) { dst = gW3; j = i - OFF_W3; }
    else { dst = gb3; j = i - OFF_B3; }
    dst[j] += s;
}

size_t backward_workspace_bytes() { return (size_t)BWD_BLOCKS * NPAR * sizeof(float); }

hipError_t launch_backward(const BwdArgs &A, int kt, int precision, const MlpGrad &gm, hipStream_t s)
{
    const int64_t chunks = (A.c.n_rays + A.c.chunk - 1) / A.c.chunk;
    const int nblk = (int)(chunks < BWD_BLOCKS ? (chunks > 0 ? chunks : 1) : BWD_BLOCKS);
    const dim3 grid(nblk), block(WAVE);
#define HP_BWD(KTV)                                                                 \
    do {                                                                            \
        if (precision == HP_BF16) k_render_backward<KTV, HP_BF16><<<grid, block, 0, s>>>(A); \
        else k_render_backward<KTV, HP_FP32><<<grid, block, 0, s>>>(A);             \
    } while (0)
    switch (kt) {
    case 4: HP_BWD(4); break;
    case 8: HP_BWD(8); break;
    case 16: HP_BWD(16); break;
    default: HP_BWD(32); break;
    }
#undef HP_BWD
    k_reduce_partials<<<(NPAR + 255) / 256, 256, 0, s>>>(A.partial, nblk, gm.W1, gm.b1, gm.W2,
                                                        gm.b2, gm.W3, gm.b3);
    return hipGetLastError();
}

}  // namespace hp
