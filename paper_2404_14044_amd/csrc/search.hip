// Forward search + sampling kernel: one 64-lane workgroup per ray.
#include "hp_kernels.hpp"
#include "hp_search.hpp"

namespace hp {

// Ray handled by this workgroup.  Consecutive workgroup ids go to different
// XCDs (round robin over 8); give each XCD a contiguous band of rays so the
// rays sharing table buckets also share an L2.
__device__ __forceinline__ int64_t xcd_ray(int64_t n_rays)
{
    const int64_t bid = blockIdx.x;
    const int64_t per = gridDim.x >> 3;
    return (bid & 7) * per + (bid >> 3);
}

template <int KT>
__global__ void __launch_bounds__(WAVE) k_search_sample(SearchCtx c, SampleOut o)
{
    __shared__ SearchLds sh;
    const int64_t ray = xcd_ray(c.n_rays);
    if (ray >= c.n_rays) return;
    const int l = lane_id();
    const RayGeom g = ray_geometry(c, ray);
    uint64_t top;
    int count;
    search_neighbours(c, g, sh, top, count);
    const int m = count < c.M ? count : c.M;
    float tj, alpha;
    int idxj, kc, nsel;
    uint64_t kd[KT], selmask;
    walk_candidates<KT>(c, g, sh, top, m, tj, idxj, kd, kc, alpha, selmask, nsel);

    if (l == 0) {
        o.n_sel[ray] = nsel;
        o.n_nbr[ray] = m;
        o.flags[ray] = (count > c.M) ? 1u : 0u;
    }
    const int first = selmask ? __builtin_ctzll(selmask) : 0;
    const int prim = readlane_i32(idxj, first);
    if (l == 0) o.primary[ray] = selmask ? prim : -1;
    if ((selmask >> l) & 1ull) {
        const int s = popc64(selmask & ((1ull << l) - 1ull));
        const int64_t row = ray * c.S + s;
        o.t[row] = tj;
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (k < c.K) {
                const bool v = k < kc;
                o.knn_idx[row * c.K + k] = v ? (int32_t)(uint32_t)kd[k] : -1;
                o.knn_dist[row * c.K + k] =
                    v ? __builtin_sqrtf(__uint_as_float((uint32_t)(kd[k] >> 32))) : 0.0f;
            }
        }
    }
    if (o.nbr_idx && l < c.M) {
        o.nbr_idx[ray * c.M + l] = l < m ? idxj : -1;
        o.nbr_t[ray * c.M + l] = l < m ? tj : 0.0f;
    }
}

hipError_t launch_search_sample(const SearchCtx &c, const SampleOut &o, int kt, hipStream_t s)
{
    int64_t blocks = (c.n_rays + 7) / 8 * 8;
    if (blocks == 0) return hipSuccess;
    const dim3 grid((unsigned)blocks), block(WAVE);
    switch (kt) {
    case 4: k_search_sample<4><<<grid, block, 0, s>>>(c, o); break;
    case 8: k_search_sample<8><<<grid, block, 0, s>>>(c, o); break;
    case 16: k_search_sample<16><<<grid, block, 0, s>>>(c, o); break;
    default: k_search_sample<32><<<grid, block, 0, s>>>(c, o); break;
    }
    return hipGetLastError();
}

}  // namespace hp
