// reduce.h -- deterministic block reductions (fixed butterfly + fixed wave order).
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

// Sum of part[0..n) in a fixed order by one block of 256 threads (valid in all threads).
__device__ __forceinline__ double block_sum_array(const double* part, int n, int stride, double* lds)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += part[(size_t)i * stride];
    return block_sum<256>(v, lds);
}

}  // namespace eptv
