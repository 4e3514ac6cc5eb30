// reduce.h -- deterministic reductions (fixed butterfly, fixed block order).
// A grid-wide sum is two-stage: each block of the producing kernel writes one
// float64 partial, and a later kernel on the same stream sums the partials in
// a fixed order (kernel boundaries make them visible without fences).
#pragma once

#include <hip/hip_runtime.h>

namespace eptv {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over a block of NT threads; the result is valid in every thread.
// `lds` must hold NT/64 doubles.  Contains __syncthreads().
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += lds[i];
    return r;
}

// Sum of part[i * stride], i < n, written by an earlier kernel, by a block of
// NT threads in a fixed order (valid in all threads).  `lds` holds NT/64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum_partials(const double* part, int n, int stride, double* lds)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) v += part[(size_t)i * stride];
    return block_sum<NT>(v, lds);
}

}  // namespace eptv
