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

__device__ inline double load_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True in every thread of the block that arrives last (ticket from an atomic
// counter).  The caller resets the counter to zero when it is done.
__device__ inline bool last_block(unsigned* counter) {
    __shared__ bool s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned t = atomicAdd(counter, 1u);
        s_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last;
}

// Sum of G partials partial[k * G + b] added in block order; valid in thread 0.
__device__ inline double sum_partials(const double* partial, int G, int k) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < G; b += (int)blockDim.x) acc += load_coherent(partial + (size_t)k * G + b);
    return block_sum(acc);
}

}  // namespace red
}  // namespace trbdg
