// Launch interface of the render backward pass.
#pragma once

#include "hp_kernels.hpp"
#include "hp_mlp.hpp"

namespace hp {

constexpr int BWD_WAVES = 8;          // waves per workgroup (one workgroup per CU)
constexpr int BWD_CHUNK = 256;        // samples one wave holds at once
constexpr int BWD_MAX_BLOCKS = 256;   // bound on the persistent grid (one gradient slice each)

struct MlpGrad {
    float *W1, *b1, *W2, *b2, *W3, *b3;
};

struct BwdArgs {
    const int32_t *n_sel;
    const float *t;
    const int32_t *knn_idx;
    const float *knn_dist;
    int64_t n_rays;
    int32_t K, S, rpw;  // rpw: rays per wave chunk, rpw * S <= BWD_CHUNK
    const float *feat;
    MlpWeights w;
    float eps_idw, delta_last;
    float bg[3];
    const float *grad_rgb;
    float *grad_feat;
    float *partial;  // per-workgroup decoder-gradient slices
    int32_t *queue;  // work counter of one accumulate launch (zeroed before it)
    const MlpBf16Shared *wimg;  // the BF16 decoder packed per lane (after the counter)
};

// Decoder-gradient slices: one per workgroup of the backward grid, which is
// at most backward_slices() workgroups for any number of rays, followed by
// the work counter of the accumulate launches and the BF16 decoder's
// fragments packed per lane (read by every tile's decode instead of loading
// and converting the FP32 weights each time).
size_t backward_partial_bytes();
int backward_slices();
int backward_rays_per_wave(int S);
// The three steps of a gradient: zero the slices, accumulate any number of
// ray chunks into them (and into the feature gradient), then add the slices
// in a fixed order to the caller's decoder gradients.
hipError_t backward_zero(float *partial, hipStream_t s);
hipError_t backward_accumulate(const BwdArgs &A, int precision, hipStream_t s);
hipError_t backward_reduce(const float *partial, const MlpGrad &gm, hipStream_t s);

}  // namespace hp
