// Gradient of the render (Sec. 3.4, Eq. 2) with respect to the point
// features and the decoder parameters, given the samples of every ray.
//
// The samples depend on geometry only, so the caller either keeps the
// forward pass's samples or recomputes them with the forward search kernel
// (hp_render_backward does the latter into its workspace).  This kernel then
// mirrors the render: one wave per chunk of consecutive rays, the chunk's
// samples packed densely into tiles of 16.
//   pass A   inverse-distance aggregation and decoder (BF16 or FP32 on MFMA)
//            -> raw decoder outputs of every sample, kept in LDS;
//   composite backward (Eq. 2), one lane per ray, FP32: the transmittance in
//            front of each sample forward, then the suffix sums of colour and
//            transmittance backward -> dL/d(decoder outputs), in place;
//   pass B   per tile: the decoder is replayed keeping its activations, the
//            gradient flows back through it on FP32 matrix cores to the
//            aggregated features, and through the aggregation to the point
//            features with atomics.
// With the BF16 decoder every rounding of a decoder operand (weights,
// aggregated feature, hidden activations) counts as adding a fixed offset:
// the backward products use the rounded operands (as FP32 values) and the
// ReLU masks use the unrounded pre-activations, so the result is the exact
// gradient of the BF16 forward with its rounding offsets held fixed.
// Decoder-parameter gradients are accumulated per workgroup in a zeroed slice of
// the workspace with global atomics (L2 atomics on whole lines are much faster
// here than LDS float atomics); a second kernel sums the slices in order into
// the caller's gradient arrays.
#include <type_traits>

#include "hp_backward.hpp"
#include "hp_search.hpp"  // wave sorts

namespace hp {

constexpr int NPAR = HP_HIDDEN * HP_FEAT_DIM + HP_HIDDEN + HP_HIDDEN * HP_HIDDEN + HP_HIDDEN +
                     4 * HP_HIDDEN + 4;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + HP_HIDDEN * HP_FEAT_DIM;
constexpr int OFF_W2 = OFF_B1 + HP_HIDDEN;
constexpr int OFF_B2 = OFF_W2 + HP_HIDDEN * HP_HIDDEN;
constexpr int OFF_W3 = OFF_B2 + HP_HIDDEN;
constexpr int OFF_B3 = OFF_W3 + 4 * HP_HIDDEN;
// Floats between workgroup gradient slices: whole 128-byte lines, so that a
// row's atomics never straddle a line (unaligned slices measured 1.3x slower).
constexpr int SSTRIDE = (NPAR + 31) / 32 * 32;

// One wave's LDS.
struct BwdWave {
    float4 o[BWD_CHUNK];            // raw decoder outputs, then their gradients
    float T[BWD_CHUNK];             // transmittance in front of each sample
    int32_t pre[WAVE + 1];          // sample prefix over the chunk's rays
    int64_t row[16];                // tile: sample row (ray * S + s), -1 = padding
    float inv[16];                  // tile: 1 / sum of the inverse-distance weights
    float4 w[16];                   // tile: four inverse-distance weights per sample
    float F[16][HP_FEAT_DIM];       // tile: aggregated features [sample][feature]
    float H1T[HP_HIDDEN][16];       // tile: layer-1 activations, then their gradients
    float H2T[HP_HIDDEN][16];       // tile: layer-2 activations, then their gradients
};

// a tile's neighbour indices and weights fit in the layer-2 area they reuse
static_assert(2 * 16 * HP_MAX_K <= HP_HIDDEN * 16, "neighbour staging exceeds its LDS area");

// Aggregated feature slice (features 8 q .. 8 q + 7) of sample row `row`;
// the same arithmetic as the render (neighbours four at a time, the
// sample's four lanes sharing the weights through `sw`, summed in
// order).  Returns 1 / sum of the weights.
__device__ __forceinline__ float idw_slice_bwd(const BwdArgs &A, int64_t row, int q, float4 &sw, float *f)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = 0.0f;
    float wsum = 0.0f;
    const int32_t *ki = A.knn_idx + row * A.K;
    const float *kd = A.knn_dist + row * A.K;
    const bool vec = nbr_vec_ok(A.knn_idx, A.knn_dist, A.K);
    for (int k0 = 0; k0 < A.K; k0 += 4) {
        int idx[4];
        float d[4], w[4];
        float4 x0[4], x1[4];
        load_nbr4(ki, kd, k0, A.K, vec, idx, d);
        {
            // the sample's four lanes share the four weights, one division each
            const float dq = q == 0 ? d[0] : q == 1 ? d[1] : q == 2 ? d[2] : d[3];
            wave_lds_sync();  // the previous four weights are read
            reinterpret_cast<float *>(&sw)[q] = 1.0f / (dq > A.eps_idw ? dq : A.eps_idw);
            wave_lds_sync();
            const float4 wv = sw;
            w[0] = wv.x, w[1] = wv.y, w[2] = wv.z, w[3] = wv.w;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (idx[j] >= 0) {
                const float4 *src =
                    reinterpret_cast<const float4 *>(A.feat + (int64_t)idx[j] * HP_FEAT_DIM + 8 * q);
                x0[j] = src[0];
                x1[j] = src[1];
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (idx[j] >= 0) {
                f[0] = fma_rn(w[j], x0[j].x, f[0]);
                f[1] = fma_rn(w[j], x0[j].y, f[1]);
                f[2] = fma_rn(w[j], x0[j].z, f[2]);
                f[3] = fma_rn(w[j], x0[j].w, f[3]);
                f[4] = fma_rn(w[j], x1[j].x, f[4]);
                f[5] = fma_rn(w[j], x1[j].y, f[5]);
                f[6] = fma_rn(w[j], x1[j].z, f[6]);
                f[7] = fma_rn(w[j], x1[j].w, f[7]);
                wsum += w[j];
            }
        }
        if (idx[3] < 0) break;
    }
    const float inv = wsum > 0.0f ? 1.0f / wsum : 0.0f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] *= inv;
    return inv;
}

// Chunk-local (ray, sample) of packed sample sidx: the last ray whose prefix
// is <= sidx.
__device__ __forceinline__ int64_t sample_row(const BwdWave &sh, const BwdArgs &A, int64_t ray0,
                                              int nr, int sidx)
{
    int lo = 0, hi = nr;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sh.pre[mid] <= sidx) lo = mid;
        else hi = mid;
    }
    return (ray0 + lo) * A.S + (sidx - sh.pre[lo]);
}

template <int PREC>
__global__ void __launch_bounds__(WAVE *BWD_WAVES) k_render_backward(BwdArgs A)
{
    __shared__ BwdWave waves[BWD_WAVES];
    // FP32 weight images for the backward products, shared by the workgroup:
    // imgW2[(o1 4 + o2) 64 + lane].e = W2[16 o2 + 4 q + e][16 o1 + r],
    // imgW1[(cb 4 + o1) 64 + lane].e = W1[16 o1 + 4 q + e][16 cb + r]
    // (the A operands of dZ2 W2 and dZ1 W1 in the C layout's unit order)
    __shared__ float4 imgW2[16 * WAVE], imgW1[8 * WAVE];
    __shared__ float sW3[4 * HP_HIDDEN];
    const int wave = threadIdx.x >> 6;
    BwdWave &sh = waves[wave];
    // decoder-parameter gradients: the workgroup's zeroed workspace slice,
    // accumulated with global atomics by its eight waves (one slice per
    // workgroup is 0.84 MB per XCD, resident in its L2)
    float *const gpar = A.partial + (int64_t)blockIdx.x * SSTRIDE;
    const int l = lane_id();
    const int r16 = l & 15, q = l >> 4;

    using Mlp = typename std::conditional<PREC == HP_BF16, MlpBf16, MlpF32>::type;
    auto load_mlp = [&](Mlp &m) {
        if constexpr (PREC == HP_BF16) load_mlp_bf16_image(*A.wimg, m);
        else load_mlp_f32(A.w, m);
    };
    // a value as the decoder consumes it (bfloat16-rounded with the BF16 decoder)
    auto opnd = [](float w) { return PREC == HP_BF16 ? bf16_round(w) : w; };
    for (int i = threadIdx.x; i < 16 * WAVE; i += blockDim.x) {
        const int ln = i % WAVE, blk = i / WAVE, o1 = blk >> 2, o2 = blk & 3;
        const int r = ln & 15, qq = ln >> 4;
        const float *w = A.w.W2 + (16 * o2 + 4 * qq) * HP_HIDDEN + 16 * o1 + r;
        imgW2[i] = make_float4(opnd(w[0]), opnd(w[HP_HIDDEN]), opnd(w[2 * HP_HIDDEN]), opnd(w[3 * HP_HIDDEN]));
    }
    for (int i = threadIdx.x; i < 8 * WAVE; i += blockDim.x) {
        const int ln = i % WAVE, blk = i / WAVE, cb = blk >> 2, o1 = blk & 3;
        const int r = ln & 15, qq = ln >> 4;
        const float *w = A.w.W1 + (16 * o1 + 4 * qq) * HP_FEAT_DIM + 16 * cb + r;
        imgW1[i] = make_float4(opnd(w[0]), opnd(w[HP_FEAT_DIM]), opnd(w[2 * HP_FEAT_DIM]),
                               opnd(w[3 * HP_FEAT_DIM]));
    }
    for (int i = threadIdx.x; i < 4 * HP_HIDDEN; i += blockDim.x) sW3[i] = opnd(A.w.W3[i]);
    __syncthreads();
    // lane l: column l of dW3, entry l of db1 and db2, entry l < 4 of db3
    float gW3[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f;

    // chunks of consecutive rays are taken from a work counter, one per
    // wave at a time: a chunk's cost follows its sample count, which varies
    // from none (background) to rpw * S, so a fixed deal would leave the
    // launch waiting on the waves that drew the busiest chunks
    const int64_t n_chunks = (A.n_rays + A.rpw - 1) / A.rpw;
    for (;;) {
        int taken = 0;
        if (l == 0) taken = atomicAdd(A.queue, 1);
        const int64_t ch = __builtin_amdgcn_readfirstlane(taken);
        if (ch >= n_chunks) break;
        const int64_t ray0 = ch * A.rpw;
        const int nr = (A.n_rays - ray0) < A.rpw ? (int)(A.n_rays - ray0) : A.rpw;
        float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
        int ns = 0;
        if (l < nr) {
            const int64_t ray = ray0 + l;
            g0 = A.grad_rgb[3 * ray];
            g1 = A.grad_rgb[3 * ray + 1];
            g2 = A.grad_rgb[3 * ray + 2];
            // a ray without incoming gradient contributes nothing
            // (a count beyond the sample cap would index past the ray's rows)
            if (g0 != 0.0f || g1 != 0.0f || g2 != 0.0f) ns = min(max(A.n_sel[ray], 0), A.S);
        }
        const int inc = wave_incl_scan_i32(ns);
        sh.pre[l] = inc - ns;
        const int total = readlane_i32(inc, WAVE - 1);
        if (l == 0) sh.pre[WAVE] = total;
        wave_lds_sync();
        if (total == 0) continue;

        // pass A: raw decoder outputs of every sample (the weights are
        // reloaded per tile after its aggregation, cache hits, so that they
        // hold no registers while the feature rows are in flight)
        {
            Mlp mlp;
            for (int s0 = 0; s0 < total; s0 += 16) {
                const int sidx = s0 + r16;
                float f[8];
                if (sidx < total) idw_slice_bwd(A, sample_row(sh, A, ray0, nr, sidx), q, sh.w[r16], f);
                else
#pragma unroll
                    for (int e = 0; e < 8; ++e) f[e] = 0.0f;
                f32x4 o;
                __asm__ volatile("" ::: "memory");
                load_mlp(mlp);
                if constexpr (PREC == HP_BF16) o = decode_bf16(mlp, f);
                else o = decode_f32(mlp, f);
                if (q == 0 && sidx < total) sh.o[sidx] = make_float4(o[0], o[1], o[2], o[3]);
            }
        }
        wave_lds_sync();

        // compositing backward (Eq. 2): lane r walks ray r of the chunk
        if (ns > 0) {
            const int64_t ray = ray0 + l;
            const int base = sh.pre[l];
            const float *tr = A.t + ray * A.S;
            float T = 1.0f;
            for (int j = 0; j < ns; ++j) {
                sh.T[base + j] = T;
                const float sg = softplus_f(sh.o[base + j].w);
                const float dl = (j + 1 < ns) ? tr[j + 1] - tr[j] : A.delta_last;
                T *= expf(-sg * dl);
            }
            // U: colour composited behind sample j relative to T_{j+1};
            // P: transmittance through everything behind j (background weight)
            float U0 = 0.0f, U1 = 0.0f, U2 = 0.0f, P = 1.0f;
            for (int j = ns - 1; j >= 0; --j) {
                const float4 o = sh.o[base + j];
                const float c0 = sigmoid_f(o.x), c1 = sigmoid_f(o.y), c2 = sigmoid_f(o.z);
                const float sg = softplus_f(o.w);
                const float dl = (j + 1 < ns) ? tr[j + 1] - tr[j] : A.delta_last;
                const float e = expf(-sg * dl);
                const float a = 1.0f - e;
                const float Tj = sh.T[base + j];
                const float dLda = g0 * (Tj * (c0 - U0) - A.bg[0] * Tj * P) +
                                   g1 * (Tj * (c1 - U1) - A.bg[1] * Tj * P) +
                                   g2 * (Tj * (c2 - U2) - A.bg[2] * Tj * P);
                const float ws = Tj * a;
                sh.o[base + j] = make_float4(g0 * ws * c0 * (1.0f - c0), g1 * ws * c1 * (1.0f - c1),
                                             g2 * ws * c2 * (1.0f - c2), dLda * dl * e * sigmoid_f(o.w));
                U0 = a * c0 + e * U0;
                U1 = a * c1 + e * U1;
                U2 = a * c2 + e * U2;
                P = e * P;
            }
        }
        wave_lds_sync();

        // pass B: per tile, replay the decoder keeping its activations, then
        // run the decoder backward on FP32 MFMA (v_mfma_f32_16x16x4f32, lane
        // l = 16 q + r supplies A[r][q] and B[q][r] and holds D[4 q + e][r]).
        // Activation gradients chain through the C layout like the forward
        // (unit 16 b + 4 q + e of sample r), with the contraction index
        // permuted in the weight images.  The weight gradients contract over
        // the tile's samples, so their operands come from transposed LDS
        // images [unit][TP(s)], TP(s) = 4 (s mod 4) + s / 4, where a lane's
        // four samples q, q + 4, q + 8, q + 12 are one 16-byte read.
        const int ps = 4 * (r16 & 3) + (r16 >> 2);  // TP(r16)
        float *const FT = &sh.F[0][0];  // [feature][TP(s)], later [s][feature]
        for (int s0 = 0; s0 < total; s0 += 16) {
            const int nt = (total - s0) < 16 ? total - s0 : 16;
            const int sidx = s0 + r16;
            const bool valid = sidx < total;
            f32x4 h1[4], h2[4];
            int64_t row = -1;
            {
                float f[8];
                float inv = 0.0f;
                if (valid) {
                    row = sample_row(sh, A, ray0, nr, sidx);
                    inv = idw_slice_bwd(A, row, q, sh.w[r16], f);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) f[e] = 0.0f;
                }
                Mlp mlp;
                // reload the weights here (cache hits) rather than keep them
                // live across the whole backward
                __asm__ volatile("" ::: "memory");
                load_mlp(mlp);
                if constexpr (PREC == HP_BF16) decode_bf16(mlp, f, h1, h2);
                else decode_f32(mlp, f, h1, h2);
                if (q == 0) {
                    sh.row[r16] = row;
                    sh.inv[r16] = inv;
                }
                // the weight gradients contract the activations as the next
                // layer consumed them (bfloat16-rounded with the BF16 decoder);
                // the registers keep the unrounded values for the ReLU masks
#pragma unroll
                for (int ob = 0; ob < 4; ++ob)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (!valid) {
                            h1[ob][e] = 0.0f;
                            h2[ob][e] = 0.0f;
                        }
                        sh.H1T[16 * ob + 4 * q + e][ps] = opnd(h1[ob][e]);
                        sh.H2T[16 * ob + 4 * q + e][ps] = opnd(h2[ob][e]);
                    }
#pragma unroll
                for (int e = 0; e < 8; ++e) FT[(8 * q + e) * 16 + ps] = opnd(f[e]);
            }
            // the tile's neighbour lists, fetched now (all loads independent,
            // in flight during the products) and staged in LDS after them
            // lane (r16, q): entries q, q + 4, ... of sample r16
            constexpr int PF = HP_MAX_K / 4;
            int32_t pf_i[PF];
            float pf_d[PF];
            {
                const int64_t prow = row;
#pragma unroll
                for (int m = 0; m < PF; ++m) {
                    const int k = q + 4 * m;
                    pf_i[m] = -1;
                    pf_d[m] = 0.0f;
                    if (prow >= 0 && k < A.K) {
                        pf_i[m] = A.knn_idx[prow * A.K + k];
                        pf_d[m] = A.knn_dist[prow * A.K + k];
                    }
                }
            }
            wave_lds_sync();
            // output layer: dW3 and db3 on the VALU, lane l = hidden unit l
            {
                float hrow[16];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float4 v = *reinterpret_cast<const float4 *>(&sh.H2T[l][4 * k]);
                    hrow[4 * k] = v.x;
                    hrow[4 * k + 1] = v.y;
                    hrow[4 * k + 2] = v.z;
                    hrow[4 * k + 3] = v.w;
                }
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    if (s < nt) {
                        const float4 d = sh.o[s0 + s];
                        const float h = hrow[4 * (s & 3) + (s >> 2)];
                        gW3[0] = fma_rn(d.x, h, gW3[0]);
                        gW3[1] = fma_rn(d.y, h, gW3[1]);
                        gW3[2] = fma_rn(d.z, h, gW3[2]);
                        gW3[3] = fma_rn(d.w, h, gW3[3]);
                        if (l < 4) gb3 += (l == 0) ? d.x : (l == 1) ? d.y : (l == 2) ? d.z : d.w;
                    }
                }
            }
            // dZ2 = (dO W3) masked by layer 2's ReLU: A = W3[q][unit], B = dO[s][q]
            f32x4 dz2[4];
            {
                float dOq = 0.0f;
                if (valid) {
                    const float4 d = sh.o[sidx];
                    dOq = q == 0 ? d.x : (q == 1 ? d.y : (q == 2 ? d.z : d.w));
                }
#pragma unroll
                for (int ob = 0; ob < 4; ++ob) {
                    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(sW3[q * HP_HIDDEN + 16 * ob + r16], dOq, acc, 0, 0, 0);
#pragma unroll
                    for (int e = 0; e < 4; ++e) dz2[ob][e] = h2[ob][e] > 0.0f ? acc[e] : 0.0f;
                }
            }
            wave_lds_sync();  // H2T (activations) fully read
#pragma unroll
            for (int ob = 0; ob < 4; ++ob)
#pragma unroll
                for (int e = 0; e < 4; ++e) sh.H2T[16 * ob + 4 * q + e][ps] = dz2[ob][e];
            wave_lds_sync();
            // db2 (lane l = unit l) and dW2 += dZ2^T H1 over the tile's samples
            {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float4 v = *reinterpret_cast<const float4 *>(&sh.H2T[l][4 * k]);
                    gb2 += v.x;
                    gb2 += v.y;
                    gb2 += v.z;
                    gb2 += v.w;
                }
                float4 b1[4];
#pragma unroll
                for (int ob = 0; ob < 4; ++ob)
                    b1[ob] = *reinterpret_cast<const float4 *>(&sh.H1T[16 * ob + r16][4 * q]);
                // block (o2, o1): lane holds dW2[16 o2 + 4 q + e][16 o1 + r16]
#pragma unroll 1
                for (int o2 = 0; o2 < 4; ++o2) {
                    const float4 a2 = *reinterpret_cast<const float4 *>(&sh.H2T[16 * o2 + r16][4 * q]);
#pragma unroll
                    for (int o1 = 0; o1 < 4; ++o1) {
                        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a2.x, b1[o1].x, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a2.y, b1[o1].y, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a2.z, b1[o1].z, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a2.w, b1[o1].w, acc, 0, 0, 0);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            atomicAdd(&gpar[OFF_W2 + (16 * o2 + 4 * q + e) * HP_HIDDEN + 16 * o1 + r16], acc[e]);
                    }
                }
            }
            // dZ1 = (dZ2 W2) masked by layer 1's ReLU; step (ob2, e) contracts
            // unit 16 ob2 + 4 q + e of layer 2
            f32x4 dz1[4];
#pragma unroll
            for (int o1 = 0; o1 < 4; ++o1) {
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int o2 = 0; o2 < 4; ++o2) {
                    const float4 w = imgW2[(o1 * 4 + o2) * WAVE + l];
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.x, dz2[o2][0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.y, dz2[o2][1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.z, dz2[o2][2], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w, dz2[o2][3], acc, 0, 0, 0);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) dz1[o1][e] = h1[o1][e] > 0.0f ? acc[e] : 0.0f;
            }
            wave_lds_sync();  // H1T (activations) fully read
#pragma unroll
            for (int ob = 0; ob < 4; ++ob)
#pragma unroll
                for (int e = 0; e < 4; ++e) sh.H1T[16 * ob + 4 * q + e][ps] = dz1[ob][e];
            wave_lds_sync();
            // db1 (lane l = unit l) and dW1 += dZ1^T F over the tile's samples
            {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float4 v = *reinterpret_cast<const float4 *>(&sh.H1T[l][4 * k]);
                    gb1 += v.x;
                    gb1 += v.y;
                    gb1 += v.z;
                    gb1 += v.w;
                }
                float4 bf[2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    bf[cb] = *reinterpret_cast<const float4 *>(&FT[(16 * cb + r16) * 16 + 4 * q]);
                // block (o1, cb): lane holds dW1[16 o1 + 4 q + e][16 cb + r16]
#pragma unroll 1
                for (int o1 = 0; o1 < 4; ++o1) {
                    const float4 a1 = *reinterpret_cast<const float4 *>(&sh.H1T[16 * o1 + r16][4 * q]);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, bf[cb].x, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.y, bf[cb].y, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.z, bf[cb].z, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.w, bf[cb].w, acc, 0, 0, 0);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            atomicAdd(&gpar[OFF_W1 + (16 * o1 + 4 * q + e) * HP_FEAT_DIM + 16 * cb + r16], acc[e]);
                    }
                }
            }
            // dF = dZ1 W1 (gradient of the aggregated features), written as
            // [sample][feature] over the feature image once dW1 has read it
            f32x4 dF[2];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int o1 = 0; o1 < 4; ++o1) {
                    const float4 w = imgW1[(cb * 4 + o1) * WAVE + l];
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.x, dz1[o1][0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.y, dz1[o1][1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.z, dz1[o1][2], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w, dz1[o1][3], acc, 0, 0, 0);
                }
                dF[cb] = acc;
            }
            wave_lds_sync();  // the feature image fully read
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
                *reinterpret_cast<float4 *>(&sh.F[r16][16 * cb + 4 * q]) =
                    make_float4(dF[cb][0], dF[cb][1], dF[cb][2], dF[cb][3]);
            // stage (index, normalised weight) of every neighbour of the tile
            // in the layer-2 area, now dead: [sample][K] each
            int32_t *const s_idx = reinterpret_cast<int32_t *>(&sh.H2T[0][0]);
            float *const s_w = &sh.H2T[0][0] + 16 * HP_MAX_K;
            {
                const float pinv = sh.inv[r16];
#pragma unroll
                for (int m = 0; m < PF; ++m) {
                    const int k = q + 4 * m;
                    if (k < A.K) {
                        const float d = pf_d[m];
                        s_idx[r16 * A.K + k] = pf_i[m];
                        s_w[r16 * A.K + k] =
                            pf_i[m] >= 0 ? (1.0f / (d > A.eps_idw ? d : A.eps_idw)) * pinv : 0.0f;
                    }
                }
            }
            wave_lds_sync();
            // aggregation backward: d feat[idx_k][cc] += (w_k / sum w) dF[s][cc].
            // Consecutive samples share most neighbours, so with K <= 8 the
            // tile's (neighbour, sample) pairs are sorted by neighbour and each
            // distinct neighbour gets one atomic per channel (the atomics, not
            // the arithmetic, bound this pass).
            if (A.K <= 8) {
                // key: neighbour index << 32 | s << 3 | k (~0: none); 128 pairs,
                // elements l and 64 + l on lane l
                uint64_t x0 = ~0ull, x1 = ~0ull;
                {
                    const int sa = l / A.K, ka = l - sa * A.K;
                    const int sb = (l + WAVE) / A.K, kb = l + WAVE - sb * A.K;
                    if (sa < nt) {
                        const int idx = s_idx[sa * A.K + ka];
                        if (idx >= 0) x0 = ((uint64_t)(uint32_t)idx << 32) | (uint32_t)(sa << 3 | ka);
                    }
                    if (sb < nt) {
                        const int idx = s_idx[sb * A.K + kb];
                        if (idx >= 0) x1 = ((uint64_t)(uint32_t)idx << 32) | (uint32_t)(sb << 3 | kb);
                    }
                }
                // 128-key bitonic sort: ascending and descending halves, then
                // the lane-wise half-cleaner and both halves sorted
                x0 = wave_sort_fast(x0);
                x1 = wave_sort_desc(x1);
                {
                    const uint64_t lo = umin64(x0, x1), hi = umax64(x0, x1);
                    x0 = wave_merge_low_fast(lo, ~0ull);
                    x1 = wave_merge_low_fast(hi, ~0ull);
                }
                // segment heads: the first pair of every distinct neighbour.
                // Layer-2 area (1024 words): s_idx [0, 128), sorted keys
                // [256, 512), s_w [512, 640), segment starts [640, 769)
                static_assert(16 * HP_MAX_K >= 512 && HP_HIDDEN * 16 >= 769, "pair staging layout");
                uint64_t *const srt = reinterpret_cast<uint64_t *>(&sh.H2T[0][0] + 256);
                int32_t *const seg = reinterpret_cast<int32_t *>(&sh.H2T[0][0] + 640);
                const uint32_t i0 = (uint32_t)(x0 >> 32), i1 = (uint32_t)(x1 >> 32);
                const uint32_t p0 = (uint32_t)__shfl_up((int)i0, 1, WAVE);
                const uint32_t p1 = l == 0 ? (uint32_t)readlane_i32((int)i0, WAVE - 1)
                                           : (uint32_t)__shfl_up((int)i1, 1, WAVE);
                const bool h0 = x0 != ~0ull && (l == 0 || p0 != i0);
                const bool h1 = x1 != ~0ull && p1 != i1;
                const uint64_t m0 = ballot(h0), m1 = ballot(h1);
                const int nv = popc64(ballot(x0 != ~0ull)) + popc64(ballot(x1 != ~0ull));
                const int u0 = popc64(m0), nu = u0 + popc64(m1);
                srt[l] = x0;
                srt[WAVE + l] = x1;
                if (h0) seg[rank_below(m0)] = l;
                if (h1) seg[u0 + rank_below(m1)] = WAVE + l;
                if (l == 0) seg[nu] = nv;
                wave_lds_sync();
                // lane (cc, half): distinct neighbours half, half + 2, ...
                const int cc = l & 31, half = l >> 5;
                for (int j = half; j < nu; j += 2) {
                    const int e0 = seg[j], e1 = seg[j + 1];
                    float g = 0.0f;
                    for (int e = e0; e < e1; ++e) {
                        const uint32_t sk = (uint32_t)srt[e];
                        const int ss = (int)(sk >> 3), kk = (int)(sk & 7u);
                        g = fma_rn(s_w[ss * A.K + kk], sh.F[ss][cc], g);
                    }
                    const uint32_t idx = (uint32_t)(srt[e0] >> 32);
                    atomicAdd(&A.grad_feat[(int64_t)idx * HP_FEAT_DIM + cc], g);
                }
            } else {
                // lane l is feature l & 31 of samples 8 (l >> 5) .. +7
                const int cc = l & 31, half = l >> 5;
#pragma unroll
                for (int si = 0; si < 8; ++si) {
                    const int s = 8 * half + si;
                    if (s >= nt) break;
                    const float df = sh.F[s][cc];
                    for (int k = 0; k < A.K; ++k) {
                        const int idx = s_idx[s * A.K + k];
                        if (idx < 0) break;
                        atomicAdd(&A.grad_feat[(int64_t)idx * HP_FEAT_DIM + cc], s_w[s * A.K + k] * df);
                    }
                }
            }
            wave_lds_sync();
        }
    }

    // this workgroup's parameter gradients -> its workspace slice
#pragma unroll
    for (int k = 0; k < 4; ++k) atomicAdd(&gpar[OFF_W3 + k * HP_HIDDEN + l], gW3[k]);
    atomicAdd(&gpar[OFF_B1 + l], gb1);
    atomicAdd(&gpar[OFF_B2 + l], gb2);
    if (l < 4) atomicAdd(&gpar[OFF_B3 + l], gb3);
}

__global__ void __launch_bounds__(256) k_zero_f32(float *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Sum the per-workgroup slices and add to the gradients, in a fixed order: each of
// RED_G thread groups sums a contiguous range of slices in order, then the
// group sums are added in group order.  (One thread per parameter walking
// every slice would leave the chip idle: there are only 6,532 parameters.)
constexpr int RED_P = 64;  // parameters per workgroup
constexpr int RED_G = 16;  // slice ranges per parameter

__global__ void __launch_bounds__(RED_P * RED_G) k_reduce_partials(const float *__restrict__ partial,
                                                                  int nslice, float *gW1, float *gb1,
                                                                  float *gW2, float *gb2, float *gW3,
                                                                  float *gb3)
{
    __shared__ float sh[RED_G][RED_P];
    const int p = threadIdx.x % RED_P, grp = threadIdx.x / RED_P;
    const int i = blockIdx.x * RED_P + p;
    const int per = (nslice + RED_G - 1) / RED_G;
    const int b0 = grp * per, b1 = min(nslice, b0 + per);
    float s = 0.0f;
    if (i < NPAR) {
#pragma unroll 8
        for (int b = b0; b < b1; ++b) s += partial[(int64_t)b * SSTRIDE + i];
    }
    sh[grp][p] = s;
    __syncthreads();
    if (grp != 0 || i >= NPAR) return;
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < RED_G; ++k) t += sh[k][p];
    float *dst;
    int j;
    if (i < OFF_B1) { dst = gW1; j = i - OFF_W1; }
    else if (i < OFF_W2) { dst = gb1; j = i - OFF_B1; }
    else if (i < OFF_B2) { dst = gW2; j = i - OFF_W2; }
    else if (i < OFF_W3) { dst = gb2; j = i - OFF_B2; }
    else if (i < OFF_B3) { dst = gW3; j = i - OFF_W3; }
    else { dst = gb3; j = i - OFF_B3; }
    dst[j] += t;
}

// the slices, one 256-byte line for the work counter, then the packed BF16
// decoder
constexpr size_t WIMG_BYTES = (sizeof(MlpBf16Shared) + 255) / 256 * 256;

size_t backward_partial_bytes()
{
    return (size_t)BWD_MAX_BLOCKS * SSTRIDE * sizeof(float) + 256 + WIMG_BYTES;
}

static int32_t *queue_of(float *partial)
{
    return reinterpret_cast<int32_t *>(partial + (size_t)BWD_MAX_BLOCKS * SSTRIDE);
}

static MlpBf16Shared *wimg_of(float *partial)
{
    return reinterpret_cast<MlpBf16Shared *>(reinterpret_cast<char *>(queue_of(partial)) + 256);
}

__global__ void __launch_bounds__(256) k_pack_mlp_bf16(MlpWeights w, MlpBf16Shared *img)
{
    store_mlp_bf16_shared(w, *img, threadIdx.x / WAVE, blockDim.x / WAVE);
}

int backward_slices()
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // one workgroup fills a CU's LDS: a persistent grid of one per CU
    return cus < BWD_MAX_BLOCKS ? (cus > 0 ? cus : 1) : BWD_MAX_BLOCKS;
}

int backward_rays_per_wave(int S)
{
    const int r = BWD_CHUNK / (S > 0 ? S : 1);
    return r > WAVE ? WAVE : r;
}

hipError_t backward_zero(float *partial, hipStream_t s)
{
    const int64_t nzero = (int64_t)backward_slices() * SSTRIDE;
    k_zero_f32<<<dim3((unsigned)((nzero + 255) / 256)), 256, 0, s>>>(partial, nzero);
    return hipGetLastError();
}

hipError_t backward_accumulate(const BwdArgs &args, int precision, hipStream_t s)
{
    if (args.n_rays == 0) return hipSuccess;
    BwdArgs A = args;
    A.queue = queue_of(A.partial);
    A.wimg = wimg_of(A.partial);
    // (a fill kernel, not a memset: callers may capture this in a graph)
    k_zero_f32<<<1, 64, 0, s>>>(reinterpret_cast<float *>(A.queue), 1);
    if (precision == HP_BF16) k_pack_mlp_bf16<<<1, 256, 0, s>>>(A.w, wimg_of(A.partial));
    const int64_t chunks = (A.n_rays + A.rpw - 1) / A.rpw;
    int64_t nblk = (chunks + BWD_WAVES - 1) / BWD_WAVES;
    const int64_t nslice = backward_slices();
    if (nblk > nslice) nblk = nslice;
    if (nblk < 1) nblk = 1;
    if (precision == HP_BF16)
        k_render_backward<HP_BF16><<<dim3((unsigned)nblk), dim3(WAVE * BWD_WAVES), 0, s>>>(A);
    else
        k_render_backward<HP_FP32><<<dim3((unsigned)nblk), dim3(WAVE * BWD_WAVES), 0, s>>>(A);
    return hipGetLastError();
}

hipError_t backward_reduce(const float *partial, const MlpGrad &gm, hipStream_t s)
{
    k_reduce_partials<<<(NPAR + RED_P - 1) / RED_P, RED_P * RED_G, 0, s>>>(
        partial, backward_slices(), gm.W1, gm.b1, gm.W2, gm.b2, gm.W3, gm.b3);
    return hipGetLastError();
}

}  // namespace hp
