// Launch interfaces of the HashPoint kernels (host side of the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hashpoint.h"
#include "hp_mlp.hpp"

namespace hp {

struct ViewK;
struct ViewSet;
struct SearchCtx;

struct SampleOut {
    int32_t *n_sel, *primary, *n_nbr;
    uint32_t *flags;
    float *t;
    int32_t *knn_idx;
    float *knn_dist;
    int32_t *nbr_idx;
    float *nbr_t;
};

struct RenderArgs {
    const int32_t *n_sel;
    const float *t;
    const int32_t *knn_idx;
    const float *knn_dist;
    int64_t n_rays;
    const float *feat;
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    int32_t K, S;
    float eps_idw, delta_last;
    float bg[3];
    float *rgb, *depth, *acc;
    int32_t rpw;     // rays per render chunk (16, 32 or 64)
    int32_t blocks;  // render grid, 0 = one workgroup per chunk
};

struct TableWs;

// table build
hipError_t launch_build(const float *xyz, int64_t n, const ViewSet &vs, int64_t n_buckets,
                        int64_t n_cells, const TableWs &tw, hipStream_t s);

hipError_t launch_search_sample(const SearchCtx &c, const SampleOut &o, int kt, hipStream_t s);

hipError_t launch_render(const RenderArgs &a, int precision, hipStream_t s);

struct KnpArgs {
    const float *colors;  // n x 3
    int32_t K;
    float eps_idw;
    float bg[3];
    float *rgb;     // R x 3
    int32_t *cnt;   // R, nullable
    int32_t *idx;   // R x K, nullable (with dist)
    float *dist;    // R x K
};

hipError_t launch_knp(const SearchCtx &c, const KnpArgs &a, hipStream_t s);

struct FusedArgs {
    const float *feat;
    MlpWeights w;
    float eps_idw, delta_last;
    float bg[3];
    float *rgb, *depth, *acc;  // depth, acc nullable
    int32_t *n_sel;            // nullable
    int32_t K;
};

int fused_max_samples();
hipError_t launch_exp_neg(const float *x, float *y, int64_t n, hipStream_t s);
hipError_t launch_bf16_round(const float *x, float *y, int64_t n, hipStream_t s);
hipError_t launch_fused(const SearchCtx &c, const FusedArgs &a, int kt, int precision, hipStream_t s);

}  // namespace hp
