// Launch interface of the render backward pass.
#pragma once

#include "hp_kernels.hpp"
#include "hp_mlp.hpp"
#include "hp_search.hpp"

namespace hp {

struct MlpGrad {
    float *W1, *b1, *W2, *b2, *W3, *b3;
};

struct BwdArgs {
    SearchCtx c;
    const float *feat;
    MlpWeights w;
    float eps_idw, delta_last;
    float bg[3];
    const float *grad_rgb;
    float *grad_feat;
    float *partial;  // per-workgroup decoder-gradient slices
};

size_t backward_workspace_bytes();
hipError_t launch_backward(const BwdArgs &A, int kt, int precision, const MlpGrad &gm, hipStream_t s);

}  // namespace hp
