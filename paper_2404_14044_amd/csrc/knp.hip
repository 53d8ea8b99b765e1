// K-NP extraction and image-based blending (Sec. 3.1, Eq. 1): the K points
// nearest to each ray among its neighbours, found by the same hashed-point
// search with the kept list ordered by (squared distance to the ray, index),
// blended with geometric weights w_i = 1 / max(e_i, eps), normalised.
//
// One 64-lane workgroup per ray, persistent over XCD-banded chunks like the
// forward search: lane i < K holds the i-th nearest point, gathers its
// colour, and the wave reduces the weighted sums with a fixed butterfly.
#include "hp_kernels.hpp"
#include "hp_search.hpp"

namespace hp {

__device__ __forceinline__ float wave_sum_f32(float v)
{
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_knp(SearchCtx c, KnpArgs a)
{
    __shared__ SearchLds sh;
    const int l = lane_id();
    for_each_ray_banded(c, sh.rs, [&](int64_t ray, const RayGeom &g) {
        uint64_t top;
        int count;
        search_neighbours<true>(c, g, sh, top, count);
        const int kk = count < a.K ? count : a.K;
        const bool mine = l < kk;
        const int idx = mine ? (int)(uint32_t)top : -1;
        const float e = mine ? __builtin_sqrtf(__uint_as_float((uint32_t)(top >> 32))) : 0.0f;
        float w = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
        if (mine) {
            w = 1.0f / (e > a.eps_idw ? e : a.eps_idw);
            const float *col = a.colors + 3 * (int64_t)idx;
            c0 = w * col[0];
            c1 = w * col[1];
            c2 = w * col[2];
        }
        const float ws = wave_sum_f32(w);
        c0 = wave_sum_f32(c0);
        c1 = wave_sum_f32(c1);
        c2 = wave_sum_f32(c2);
        if (l == 0) {
            a.rgb[3 * ray + 0] = kk ? c0 / ws : a.bg[0];
            a.rgb[3 * ray + 1] = kk ? c1 / ws : a.bg[1];
            a.rgb[3 * ray + 2] = kk ? c2 / ws : a.bg[2];
            if (a.cnt) a.cnt[ray] = kk;
        }
        if (a.idx && l < a.K) {
            a.idx[ray * a.K + l] = idx;
            a.dist[ray * a.K + l] = e;
        }
        lds_sync();
    }, [&](int64_t ray) {
        // (one lane) a ray with no point near it: background, no point
        a.rgb[3 * ray + 0] = a.bg[0];
        a.rgb[3 * ray + 1] = a.bg[1];
        a.rgb[3 * ray + 2] = a.bg[2];
        if (a.cnt) a.cnt[ray] = 0;
        if (a.idx) {
            for (int i = 0; i < a.K; ++i) {
                a.idx[ray * a.K + i] = -1;
                a.dist[ray * a.K + i] = 0.0f;
            }
        }
    });
}

hipError_t launch_knp(const SearchCtx &c, const KnpArgs &a, hipStream_t s)
{
    const int64_t blocks = banded_grid(c, c.blocks > 0 ? c.blocks : DEFAULT_SEARCH_BLOCKS);
    if (blocks == 0) return hipSuccess;
    k_knp<<<dim3((unsigned)blocks), dim3(WAVE), 0, s>>>(c, a);
    return hipGetLastError();
}

}  // namespace hp
