// reduce.h -- deterministic reductions (fixed lane patterns, fixed block order).
// A grid-wide sum is two-stage: each block of the producing kernel writes one
// float64 partial, and a later kernel on the same stream sums the partials in
// a fixed order (kernel boundaries make them visible without fences).
#pragma once

#include <hip/hip_runtime.h>

namespace eptv {

// v + v of another lane of the same 16-lane row, by a DPP lane pattern (the
// two 32-bit halves moved separately).
template <int CTRL>
__device__ __forceinline__ double dpp_add_row(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return v + __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_of(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the wave's 64 lanes in a fixed order, valid in every lane: within
// each 16-lane row by DPP (the pair partner, the other pair of the quad, the
// other quad of the 8, the other 8 of the 16; a + b and b + a agree, so all
// lanes of a row hold the same bits), then the four rows' sums in order.
// Every lane must be active.
__device__ __forceinline__ double wave_sum(double v)
{
    v = dpp_add_row<0xb1>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add_row<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add_row<0x141>(v);  // row_half_mirror
    v = dpp_add_row<0x140>(v);  // row_mirror
    return (lane_of(v, 0) + lane_of(v, 16)) + (lane_of(v, 32) + lane_of(v, 48));
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
