// Device evaluation of the binary32 exponential that decides which
// candidates become samples (alpha = gamma exp(-d^2 / beta^2), Sec. 3.3), so
// that its bits can be compared with any other implementation of the same
// operation sequence.
#include "hp_device.hpp"
#include "hp_kernels.hpp"
#include "hp_mlp.hpp"

namespace hp {

__global__ void __launch_bounds__(256) k_exp_neg(const float *__restrict__ x, float *__restrict__ y,
                                                 int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = exp_neg(x[i]);
}

hipError_t launch_exp_neg(const float *x, float *y, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    k_exp_neg<<<dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s>>>(x, y, n);
    return hipGetLastError();
}

// Device rounding of binary32 values to bfloat16, the operation the BF16
// decoder applies to its operands (R22), for bit-for-bit comparison.
__global__ void __launch_bounds__(256) k_bf16_round(const float *__restrict__ x, float *__restrict__ y,
                                                    int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = bf16_round(x[i]);
}

hipError_t launch_bf16_round(const float *x, float *y, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    k_bf16_round<<<dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s>>>(x, y, n);
    return hipGetLastError();
}

}  // namespace hp
