// Deterministic block reductions (fixed shuffle tree inside each wave, then
// waves summed in index order by thread 0).
#pragma once
#include <hip/hip_runtime.h>

namespace paro {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// Sum over the block; the result is valid in thread 0 and also returned to
// every thread (broadcast through red[0]).  red: __shared__ double[NT/64].
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < NT / 64; ++i) s += red[i];
        red[0] = s;
    }
    __syncthreads();
    s = red[0];
    __syncthreads();
    return s;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double *red)
{
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = red[0];
        for (int i = 1; i < NT / 64; ++i) s = fmax(s, red[i]);
        red[0] = s;
    }
    __syncthreads();
    double s = red[0];
    __syncthreads();
    return s;
}

}  // namespace paro
