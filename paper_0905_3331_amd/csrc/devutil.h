// devutil.h -- device helpers shared by the kernel files.
#pragma once
#include <hip/hip_runtime.h>

namespace tmq {

// Sum over a block (blockDim.x a multiple of 64, at most 1024), result valid in
// thread 0.  Fixed combination order, so the result is reproducible.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) s += sh[i];
    return s;
}

__device__ __forceinline__ double block_max(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) s = fmax(s, sh[i]);
    return s;
}

}  // namespace tmq
