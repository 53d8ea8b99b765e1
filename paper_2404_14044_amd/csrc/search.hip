// Forward search + sampling kernel: one 64-lane workgroup per ray, persistent
// over XCD-banded chunks of rays (for_each_ray_banded).
#include "hp_kernels.hpp"
#include "hp_search.hpp"

namespace hp {

template <int KT, bool MS>
__device__ __forceinline__ void search_sample_body(const SearchCtx &c, const SampleOut &o)
{
    __shared__ SearchLds sh;
    const int l = lane_id();
    for_each_ray_banded(c, sh.rs, [&](int64_t gray, const RayGeom &g) {
        const int64_t ray = gray - c.ray0;  // row of the outputs
        uint64_t top;
        int count;
        search_neighbours(c, g, sh, top, count);
        const int m = count < c.M ? count : c.M;
        const int64_t rbase = ray * c.S;
        int prim;
        auto emit = [&](int s, int q, float tj, const uint64_t(&kd)[KT], const float(&dq)[KT / 4],
                        int kc) {
            // the candidate's four lanes share the row: lane q writes k = q, q + 4, ...
            const int64_t row = rbase + s;
            if (q == 0) o.t[row] = tj;
#pragma unroll
            for (int e = 0; e < KT / 4; ++e) {
                const int k = 4 * e + q;
                if (k < c.K) {
                    const bool v = k < kc;
                    o.knn_idx[row * c.K + k] = v ? (int32_t)(uint32_t)quad_entry<KT>(kd, e) : -1;
                    o.knn_dist[row * c.K + k] = v ? dq[e] : 0.0f;
                }
            }
        };
        int nsel;
        if constexpr (MS) nsel = uniform_samples<KT>(c, g, sh, top, count, prim, emit);
        else nsel = walk_candidates<KT>(c, g, sh, top, m, prim, emit);
        if (l == 0) {
            o.n_sel[ray] = nsel;
            o.n_nbr[ray] = m;
            o.flags[ray] = (count > c.M) ? 1u : 0u;
            o.primary[ray] = prim;
        }
        const float tj = __uint_as_float((uint32_t)(top >> 32));
        const int idxj = (int)(uint32_t)top;
        if (o.nbr_idx && l < c.M) {
            o.nbr_idx[ray * c.M + l] = l < m ? idxj : -1;
            o.nbr_t[ray * c.M + l] = l < m ? tj : 0.0f;
        }
        lds_sync();
    }, [&](int64_t gray) {
        // (one lane) a ray with no point near it: no neighbour, no sample
        const int64_t ray = gray - c.ray0;
        o.n_sel[ray] = 0;
        o.n_nbr[ray] = 0;
        o.flags[ray] = 0u;
        o.primary[ray] = -1;
        if (o.nbr_idx) {
            for (int i = 0; i < c.M; ++i) {
                o.nbr_idx[ray * c.M + i] = -1;
                o.nbr_t[ray * c.M + i] = 0.0f;
            }
        }
    });
}

// 6 waves per SIMD where the nearest-neighbour lists are short (80 VGPRs,
// fewer spills than at 8; with the default grid of many more workgroups
// than fit at once, 6 measured 3% faster than 8, and 7, 5 or 4 slower).
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_search_sample_k4(SearchCtx c, SampleOut o) { search_sample_body<4, false>(c, o); }
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_search_sample_k8(SearchCtx c, SampleOut o) { search_sample_body<8, false>(c, o); }
// 16-entry lists: 5 waves per SIMD (room view 9% faster than 4, 3 slower)
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(5, 8)))
k_search_sample_k16(SearchCtx c, SampleOut o) { search_sample_body<16, false>(c, o); }
__global__ void __launch_bounds__(WAVE) k_search_sample_k32(SearchCtx c, SampleOut o)
{
    search_sample_body<32, false>(c, o);
}

// The same search with the uniform multi-surface sampler.
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_search_ms_k4(SearchCtx c, SampleOut o) { search_sample_body<4, true>(c, o); }
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_search_ms_k8(SearchCtx c, SampleOut o) { search_sample_body<8, true>(c, o); }
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_search_ms_k16(SearchCtx c, SampleOut o) { search_sample_body<16, true>(c, o); }
__global__ void __launch_bounds__(WAVE) k_search_ms_k32(SearchCtx c, SampleOut o)
{
    search_sample_body<32, true>(c, o);
}

hipError_t launch_search_sample(const SearchCtx &c, const SampleOut &o, int kt, hipStream_t s)
{
    const int64_t blocks = banded_grid(c, c.blocks > 0 ? c.blocks : DEFAULT_SEARCH_BLOCKS);
    if (blocks == 0) return hipSuccess;
    const dim3 grid((unsigned)blocks), block(WAVE);
    if (c.sampler == HP_SAMPLER_MS) {
        switch (kt) {
        case 4: k_search_ms_k4<<<grid, block, 0, s>>>(c, o); break;
        case 8: k_search_ms_k8<<<grid, block, 0, s>>>(c, o); break;
        case 16: k_search_ms_k16<<<grid, block, 0, s>>>(c, o); break;
        default: k_search_ms_k32<<<grid, block, 0, s>>>(c, o); break;
        }
        return hipGetLastError();
    }
    switch (kt) {
    case 4: k_search_sample_k4<<<grid, block, 0, s>>>(c, o); break;
    case 8: k_search_sample_k8<<<grid, block, 0, s>>>(c, o); break;
    case 16: k_search_sample_k16<<<grid, block, 0, s>>>(c, o); break;
    default: k_search_sample_k32<<<grid, block, 0, s>>>(c, o); break;
    }
    return hipGetLastError();
}

}  // namespace hp
