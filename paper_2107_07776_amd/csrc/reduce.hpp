// Device-side block reductions shared by the kernels (256-thread blocks).
#pragma once

#include <hip/hip_runtime.h>

namespace trbdg {
namespace red {

constexpr int BS = 256;

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Block-wide sum over a 256-thread block; the result is valid in thread 0.
// Every thread of the block must call it.
__device__ inline double block_sum(double v) {
    __shared__ double s_part[BS / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) s_part[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) r += s_part[i];
    __syncthreads();
    return r;
}

}  // namespace red
}  // namespace trbdg
