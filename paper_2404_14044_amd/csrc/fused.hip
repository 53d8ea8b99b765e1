// Search, sampling and rendering in one kernel (Sec. 3.2-3.4): the samples of
// a ray never leave the workgroup.  One wave per ray, persistent over
// XCD-banded chunks like the forward search: the search and the candidate
// walk (or the uniform sampler) emit each sample's t and nearest neighbours
// into LDS, then the wave aggregates the features of its (at most 16)
// samples as one MFMA tile, decodes them and composites the ray.  Every
// operation and its order are those of hp_search_sample followed by
// hp_render, so the outputs are identical; what is saved is the sample
// arrays' round trip through HBM and a launch.
#include <type_traits>

#include "hp_kernels.hpp"
#include "hp_mlp.hpp"
#include "hp_search.hpp"

namespace hp {

constexpr int FUSED_S = 16;  // samples per ray the fused kernel holds (one tile)

template <int KT>
struct FusedLds {
    SearchLds s;
    float t[FUSED_S];
    int32_t idx[FUSED_S][KT];
    float dist[FUSED_S][KT];
    float4 out[FUSED_S];  // (sigmoid rgb, softplus sigma) per sample
};

template <int KT, int PREC, bool MS>
__device__ __forceinline__ void fused_body(const SearchCtx &c, const FusedArgs &a)
{
    __shared__ FusedLds<KT> sh;
    const int l = lane_id();
    const int r16 = l & 15, q = l >> 4;
    for_each_ray_banded(c, sh.s.rs, [&](int64_t ray, const RayGeom &g) {
        uint64_t top;
        int count;
        search_neighbours(c, g, sh.s, top, count);
        const int m = count < c.M ? count : c.M;
        int prim;
        auto emit = [&](int s, int qq, float tj, const uint64_t(&kd)[KT], const float(&dq)[KT / 4],
                        int kc) {
            if (qq == 0) sh.t[s] = tj;
#pragma unroll
            for (int e = 0; e < KT / 4; ++e) {
                const int k = 4 * e + qq;
                const bool v = k < kc && k < c.K;
                sh.idx[s][k] = v ? (int32_t)(uint32_t)quad_entry<KT>(kd, e) : -1;
                sh.dist[s][k] = v ? dq[e] : 0.0f;
            }
        };
        int n;
        if constexpr (MS) n = uniform_samples<KT>(c, g, sh.s, top, count, prim, emit);
        else n = walk_candidates<KT>(c, g, sh.s, top, m, prim, emit);
        lds_sync();
        if (n > 0) {
            // aggregation (lane: sample r16, features 8 q .. 8 q + 7), as the render
            float f[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) f[e] = 0.0f;
            if (r16 < n) {
                // neighbours four at a time, summed in order (as the render)
                float wsum = 0.0f;
                for (int k0 = 0; k0 < c.K; k0 += 4) {
                    int idx[4];
                    float w[4];
                    float4 x0[4], x1[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const bool in = k0 + j < c.K;
                        idx[j] = in ? sh.idx[r16][k0 + j] : -1;
                        const float d = in ? sh.dist[r16][k0 + j] : 1.0f;
                        w[j] = 1.0f / (d > a.eps_idw ? d : a.eps_idw);
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (idx[j] >= 0) {
                            const float4 *src = reinterpret_cast<const float4 *>(
                                a.feat + (int64_t)idx[j] * HP_FEAT_DIM + 8 * q);
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
            f32x4 o;
            // load the weights here (cache hits) rather than keep them live
            // across the search
            __asm__ volatile("" ::: "memory");
            if constexpr (PREC == HP_BF16) {
                MlpBf16 mlp;
                load_mlp_bf16(a.w, mlp);
                o = decode_bf16(mlp, f);
            } else {
                MlpF32 mlp;
                load_mlp_f32(a.w, mlp);
                o = decode_f32(mlp, f);
            }
            if (q == 0 && r16 < n)
                sh.out[r16] = make_float4(sigmoid_f(o[0]), sigmoid_f(o[1]), sigmoid_f(o[2]),
                                          softplus_f(o[3]));
            lds_sync();
        }
        if (l == 0) {
            float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, dep = 0.0f, ws = 0.0f;
            for (int s = 0; s < n; ++s) {
                const float4 v = sh.out[s];
                const float t = sh.t[s];
                const float delta = (s + 1 < n) ? sh.t[s + 1] - t : a.delta_last;
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
            if (a.n_sel) a.n_sel[ray] = n;
        }
        lds_sync();
    }, [&](int64_t ray) {
        // (one lane) a ray with no point near it: the composite of no sample
        a.rgb[3 * ray + 0] = fma_rn(1.0f, a.bg[0], 0.0f);
        a.rgb[3 * ray + 1] = fma_rn(1.0f, a.bg[1], 0.0f);
        a.rgb[3 * ray + 2] = fma_rn(1.0f, a.bg[2], 0.0f);
        if (a.depth) a.depth[ray] = 0.0f;
        if (a.acc) a.acc[ray] = 0.0f;
        if (a.n_sel) a.n_sel[ray] = 0;
    });
}

// The decoder's weights live in registers (as in the render), which with the
// search's state needs about 240 VGPRs: 2 waves per SIMD.
template <int KT, int PREC, bool MS>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_fused(SearchCtx c, FusedArgs a)
{
    fused_body<KT, PREC, MS>(c, a);
}

int fused_max_samples() { return FUSED_S; }

template <int KT, int PREC>
static void launch_fused_kp(const SearchCtx &c, const FusedArgs &a, dim3 grid, hipStream_t s)
{
    if (c.sampler == HP_SAMPLER_MS) k_fused<KT, PREC, true><<<grid, dim3(WAVE), 0, s>>>(c, a);
    else k_fused<KT, PREC, false><<<grid, dim3(WAVE), 0, s>>>(c, a);
}

template <int KT>
static void launch_fused_k(const SearchCtx &c, const FusedArgs &a, int precision, dim3 grid,
                           hipStream_t s)
{
    if (precision == HP_BF16) launch_fused_kp<KT, HP_BF16>(c, a, grid, s);
    else launch_fused_kp<KT, HP_FP32>(c, a, grid, s);
}

hipError_t launch_fused(const SearchCtx &c, const FusedArgs &a, int kt, int precision, hipStream_t s)
{
    const int64_t blocks = banded_grid(c, c.blocks > 0 ? c.blocks : DEFAULT_SEARCH_BLOCKS);
    if (blocks == 0) return hipSuccess;
    const dim3 grid((unsigned)blocks);
    if (kt == 4) launch_fused_k<4>(c, a, precision, grid, s);
    else if (kt == 8) launch_fused_k<8>(c, a, precision, grid, s);
    else launch_fused_k<16>(c, a, precision, grid, s);
    return hipGetLastError();
}

}  // namespace hp
