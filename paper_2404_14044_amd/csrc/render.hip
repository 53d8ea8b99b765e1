// Decode and composite the samples (Sec. 3.4, Eq. 2).
//
// One wave per chunk of RPW consecutive rays (16 by default): eight waves
// per workgroup, one chunk each, with the decoder weights packed once per
// workgroup into the LDS (k_render_shared); the persistent grid and chunks
// too large for that: one wave per workgroup with the weights in its
// registers (render_body).  The wave packs the chunk's
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
#include "hp_mlp.hpp"

namespace hp {

// Aggregated feature slice (8 floats) of sample `row` for lane slice q.
// Neighbours are taken four at a time so that their index, distance and
// feature loads are in flight together; the sample's four lanes divide for
// one of the four weights each and share them through the LDS (`sh_w`, the
// sample's slot); the sums run in neighbour order (the lists are padded with
// -1 only at their end).
__device__ __forceinline__ void idw_slice(const RenderArgs &a, int64_t row, int q, float4 &sh_w, float *f)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = 0.0f;
    float wsum = 0.0f;
    const int32_t *ki = a.knn_idx + row * a.K;
    const float *kd = a.knn_dist + row * a.K;
    const bool vec = nbr_vec_ok(a.knn_idx, a.knn_dist, a.K);
    for (int k0 = 0; k0 < a.K; k0 += 4) {
        int idx[4];
        float d[4], w[4];
        float4 x0[4], x1[4];
        load_nbr4(ki, kd, k0, a.K, vec, idx, d);
        {
            // the sample's four lanes share the four weights, one division each
            const float dq = q == 0 ? d[0] : q == 1 ? d[1] : q == 2 ? d[2] : d[3];
            wave_lds_sync();  // the previous four weights are read
            reinterpret_cast<float *>(&sh_w)[q] = 1.0f / (dq > a.eps_idw ? dq : a.eps_idw);
            wave_lds_sync();
            const float4 wv = sh_w;
            w[0] = wv.x, w[1] = wv.y, w[2] = wv.z, w[3] = wv.w;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (idx[j] >= 0) {
                const float4 *src =
                    reinterpret_cast<const float4 *>(a.feat + (int64_t)idx[j] * HP_FEAT_DIM + 8 * q);
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
}

// Sample-count prefix of the chunk of RPW consecutive rays at ray0: sh_pre[r]
// = first sample of chunk ray r, sh_pre[RPW] = the chunk's samples.  Returns
// the lane's own ray's count (lane r < the chunk's rays) and the total.
struct ChunkCounts {
    int nr, ns, total;
};

template <int RPW>
__device__ __forceinline__ ChunkCounts chunk_prefix(const RenderArgs &a, int64_t ray0, int *sh_pre)
{
    const int l = lane_id();
    ChunkCounts c;
    c.nr = (a.n_rays - ray0) < RPW ? (int)(a.n_rays - ray0) : RPW;
    // (a count beyond the sample cap would index past the ray's rows and the
    // chunk's LDS)
    c.ns = (l < c.nr) ? min(max(a.n_sel[ray0 + l], 0), a.S) : 0;
    const int inc = wave_incl_scan_i32(c.ns);
    if (l < RPW) sh_pre[l] = inc - c.ns;
    c.total = readlane_i32(inc, WAVE - 1);
    if (l == 0) sh_pre[RPW] = c.total;
    wave_lds_sync();
    return c;
}

// The chunk's samples in tiles of 16: aggregate, decode (`decode`: the
// decoder on one tile's aggregated slices), activations; then each ray
// composited by its lane.  Only this wave touches sh_out, sh_pre and sh_w.
template <int RPW, typename Decode>
__device__ __forceinline__ void chunk_body(const RenderArgs &a, int64_t ray0, const ChunkCounts &c,
                                           Decode decode, float4 *sh_out, const int *sh_pre,
                                           float4 *sh_w)
{
    const int l = lane_id();
    const int nr = c.nr, ns = c.ns, total = c.total;
    const int r16 = l & 15, q = l >> 4;
    const auto activate = [&](const f32x4 &o, int sidx, bool valid) {
        // the four outputs of a sample sit in its q = 0 lane; each lane of
        // the sample takes one of them through the LDS, so the activations
        // run on all lanes instead of a quarter of them
        if (q == 0 && valid) sh_out[sidx] = make_float4(o[0], o[1], o[2], o[3]);
        wave_lds_sync();
        if (valid) {
            float *out = reinterpret_cast<float *>(&sh_out[sidx]) + q;
            const float x = *out;
            *out = q < 3 ? sigmoid_f(x) : softplus_f(x);
        }
    };
    for (int s0 = 0; s0 < total; s0 += 16) {
        const int sidx = s0 + r16;
        const bool valid = sidx < total;
        float f[8];
        if (valid) {
            int lo = 0, hi = nr;  // chunk-local ray: last with pre <= sidx
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sh_pre[mid] <= sidx) lo = mid;
                else hi = mid;
            }
            idw_slice(a, (ray0 + lo) * a.S + (sidx - sh_pre[lo]), q, sh_w[r16], f);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) f[e] = 0.0f;
        }
        activate(decode(f), sidx, valid);
    }
    wave_lds_sync();
    if (l < nr) {
        const int64_t ray = ray0 + l;
        const int base = sh_pre[l];
        float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, dep = 0.0f, ws = 0.0f;
        const float *tr = a.t + ray * a.S;
        float t = ns > 0 ? tr[0] : 0.0f;
        for (int s = 0; s < ns; ++s) {
            const float4 v = sh_out[base + s];
            // the next depth is loaded whether or not it exists (the last
            // sample reloads its own), so no load waits behind a branch
            const float tn = tr[s + 1 < ns ? s + 1 : s];
            const float delta = (s + 1 < ns) ? tn - t : a.delta_last;
            const float e = expf(-v.w * delta);
            const float w = T * (1.0f - e);
            cr = fma_rn(w, v.x, cr);
            cg = fma_rn(w, v.y, cg);
            cb = fma_rn(w, v.z, cb);
            dep = fma_rn(w, t, dep);
            ws += w;
            T *= e;
            t = tn;
        }
        const float rest = 1.0f - ws;
        a.rgb[3 * ray + 0] = fma_rn(rest, a.bg[0], cr);
        a.rgb[3 * ray + 1] = fma_rn(rest, a.bg[1], cg);
        a.rgb[3 * ray + 2] = fma_rn(rest, a.bg[2], cb);
        if (a.depth) a.depth[ray] = dep;
        if (a.acc) a.acc[ray] = ws;
    }
}

// One chunk with the decoder weights in the wave's registers: loaded here
// unless `loaded` says an earlier chunk left them there (BF16).
template <int PREC, int RPW, typename Mlp>
__device__ __forceinline__ void render_chunk(const RenderArgs &a, int64_t ray0, Mlp &mlp,
                                             bool &loaded, float4 *sh_out, int *sh_pre,
                                             float4 *sh_w)
{
    const ChunkCounts c = chunk_prefix<RPW>(a, ray0, sh_pre);
    if (c.total > 0 && (PREC != HP_BF16 || !loaded)) {
        const MlpWeights wts{a.W1, a.b1, a.W2, a.b2, a.W3, a.b3};
        if constexpr (PREC == HP_BF16) load_mlp_bf16(wts, mlp);
        else load_mlp_f32(wts, mlp);
        loaded = true;
    }
    chunk_body<RPW>(a, ray0, c, [&](const float *f) -> f32x4 {
        if constexpr (PREC == HP_BF16) return decode_bf16(mlp, f);
        else return decode_f32(mlp, f);
    }, sh_out, sh_pre, sh_w);
}

// Render grid.  By default one workgroup (one wave) per chunk, so the
// hardware dispatcher balances chunks with many samples against empty ones.
// The persistent form (render_blocks = G) has workgroup b take chunks b,
// b + G, b + 2G, ... and load the decoder weights at most once (BF16); the
// autotuner chooses between them.  Neither changes a result: every ray is
// composited by one lane from its own samples, and each sample's decoder
// column is independent of the tile it is packed in.
template <int PREC, int RPW, bool PERSIST>
__device__ __forceinline__ void render_body(const RenderArgs &a)
{
    extern __shared__ float4 sh_out[];  // [RPW * S] (rgb, sigma) per sample
    __shared__ int sh_pre[RPW + 1];
    __shared__ float4 sh_w[16];  // inverse-distance weights of a tile's samples
    typename std::conditional<PREC == HP_BF16, MlpBf16, MlpF32>::type mlp;
    bool loaded = false;
    const int64_t n_chunks = (a.n_rays + RPW - 1) / RPW;
    if constexpr (!PERSIST) {
        if ((int64_t)blockIdx.x < n_chunks)
            render_chunk<PREC, RPW>(a, (int64_t)blockIdx.x * RPW, mlp, loaded, sh_out, sh_pre, sh_w);
    } else {
        for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
            render_chunk<PREC, RPW>(a, ch * RPW, mlp, loaded, sh_out, sh_pre, sh_w);
            wave_lds_sync();  // this chunk's compositing read sh_pre / sh_out
        }
    }
}

// BF16 fits three waves per SIMD; the FP32 decoder's operands need more registers.
template <int RPW, bool PERSIST>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_render_bf16(RenderArgs a)
{
    render_body<HP_BF16, RPW, PERSIST>(a);
}

template <int RPW, bool PERSIST>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_render_fp32(RenderArgs a)
{
    render_body<HP_FP32, RPW, PERSIST>(a);
}

// Decoder weights in the LDS: a workgroup of SHARED_WAVES waves takes as
// many consecutive chunks, one per wave, and packs the weights once for all
// of them (only if one of its chunks has samples).  Without the weights in
// registers a wave needs about half as many, so more waves share a SIMD and
// hide the latency of the feature gathers.
constexpr int SHARED_WAVES = 8;
// its chunks' sample outputs must fit beside the weights: three (BF16) or two
// (FP32) workgroups per CU at 16 rays x 16 samples per chunk
constexpr size_t SHARED_DYN_MAX = 32768;

template <int PREC, int RPW>
__global__ void __launch_bounds__(WAVE *SHARED_WAVES) k_render_shared(RenderArgs a)
{
    extern __shared__ float4 sh_dyn[];  // [SHARED_WAVES][RPW * S] (rgb, sigma) per sample
    __shared__ typename std::conditional<PREC == HP_BF16, MlpBf16Shared, MlpF32Shared>::type mw;
    __shared__ int sh_pre[SHARED_WAVES][RPW + 1];
    __shared__ float4 sh_w[SHARED_WAVES][16];
    __shared__ int busy;
    const int w = threadIdx.x / WAVE;
    const int64_t n_chunks = (a.n_rays + RPW - 1) / RPW;
    const int64_t chunk = (int64_t)blockIdx.x * SHARED_WAVES + w;
    const bool live = chunk < n_chunks;
    if (threadIdx.x == 0) busy = 0;
    __syncthreads();
    ChunkCounts c{0, 0, 0};
    if (live) c = chunk_prefix<RPW>(a, chunk * RPW, sh_pre[w]);
    if (lane_id() == 0 && c.total > 0) busy = 1;
    __syncthreads();
    if (busy) {
        const MlpWeights wts{a.W1, a.b1, a.W2, a.b2, a.W3, a.b3};
        if constexpr (PREC == HP_BF16) store_mlp_bf16_shared(wts, mw, w, SHARED_WAVES);
        else store_mlp_f32_shared(wts, mw, w, SHARED_WAVES);
    }
    __syncthreads();
    if (!live) return;
    chunk_body<RPW>(a, chunk * RPW, c, [&](const float *f) -> f32x4 {
        if constexpr (PREC == HP_BF16) return decode_bf16(mw, f);
        else return decode_f32(mw, f);
    }, sh_dyn + (size_t)w * RPW * a.S, sh_pre[w], sh_w[w]);
}

template <int RPW>
static void launch_render_rpw(const RenderArgs &a, int precision, int64_t blocks, bool persist,
                              hipStream_t s)
{
    const size_t shmem = (size_t)RPW * a.S * sizeof(float4);
    const dim3 grid((unsigned)blocks), block(WAVE);
    const int64_t chunks = (a.n_rays + RPW - 1) / RPW;
    const unsigned g = (unsigned)((chunks + SHARED_WAVES - 1) / SHARED_WAVES);
    const bool shared = !persist && shmem * SHARED_WAVES <= SHARED_DYN_MAX;
    const size_t shm = shmem * SHARED_WAVES;
    if (precision == HP_BF16) {
        if (shared) k_render_shared<HP_BF16, RPW><<<g, WAVE * SHARED_WAVES, shm, s>>>(a);
        else if (persist) k_render_bf16<RPW, true><<<grid, block, shmem, s>>>(a);
        else k_render_bf16<RPW, false><<<grid, block, shmem, s>>>(a);
    } else {
        if (shared) k_render_shared<HP_FP32, RPW><<<g, WAVE * SHARED_WAVES, shm, s>>>(a);
        else if (persist) k_render_fp32<RPW, true><<<grid, block, shmem, s>>>(a);
        else k_render_fp32<RPW, false><<<grid, block, shmem, s>>>(a);
    }
}

hipError_t launch_render(const RenderArgs &a, int precision, hipStream_t s)
{
    const int rpw = a.rpw == 32 || a.rpw == 64 ? a.rpw : 16;
    const int64_t chunks = (a.n_rays + rpw - 1) / rpw;
    if (chunks == 0) return hipSuccess;
    const bool persist = a.blocks > 0 && a.blocks < chunks;
    const int64_t blocks = persist ? a.blocks : chunks;
    if (rpw == 16) launch_render_rpw<16>(a, precision, blocks, persist, s);
    else if (rpw == 64) launch_render_rpw<64>(a, precision, blocks, persist, s);
    else launch_render_rpw<32>(a, precision, blocks, persist, s);
    return hipGetLastError();
}

}  // namespace hp
