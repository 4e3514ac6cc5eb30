// cgls_step.h -- the vector update of one CGLS step (App. I), shared by the
// one-slice launch, the batched launch and the one-slice launch that also
// forms the half-edge histogram of the step's result (sigma's first digit).
#pragma once

#include <hip/hip_runtime.h>

#include "eptv_internal.h"
#include "reduce.h"

namespace eptv {

constexpr int kAxpyBlock = 256;
constexpr int kAxpyPer = 4;

// Blocks of kAxpyBlock threads, kAxpyPer elements each, over n elements.
int axpy_blocks(size_t n);

// a_m = gamma_m / delta_m, or 0 once the iteration has broken down.  gamma_m
// comes from the backprojector's partials for m = 0, else from the value
// recorded by the previous s-update; delta_m from the projector's partials.
// Every block forms it the same way (the same sums in the same order); the
// block that passes `record` stores the step's scalars for later kernels.
__device__ __forceinline__ float cgls_step_a(DevState* st, int m, const double* part_bp, int n_bp,
                                             const double* part_proj, int n_proj, bool record, double* lds)
{
    const double g = m == 0 ? block_sum_partials<kAxpyBlock>(part_bp, n_bp, 1, lds) : st->gamma[m];
    const double d = block_sum_partials<kAxpyBlock>(part_proj, n_proj, 1, lds);
    const double g0 = m == 0 ? g : st->gamma0;
    const int was = m == 0 ? 1 : st->active[m - 1];
    const bool g_ok = g > 1e-30 * g0;
    const int active = was && g_ok && (d > 0.0);
    const float a = active ? (float)(g / d) : 0.0f;
    if (record && threadIdx.x == 0) {
        if (m == 0) {
            st->gamma[0] = g;
            st->gamma0 = g;
        }
        st->delta[m] = was && g_ok ? d : 0.0;  // a step stopped by gamma_m forms no delta_m
        st->a[m] = a;
        st->active[m] = active;
        if (active) st->cg_steps = m + 1;
    }
    return a;
}

// u = u_in + a_m s (image part, blocks below img_blocks) and r = r - a_m q
// (sinogram part, the blocks after them), one launch.  When part_res is given
// the sinogram blocks also emit ||r||^2.  A block's operands are loaded
// (unconditionally, at indices clamped into the vector) before a_m is formed,
// so the two memory round trips overlap.
__device__ __forceinline__ void cgls_axpy_block(DevState* st, int m, const double* part_bp, int n_bp,
                                                const double* part_proj, int n_proj, size_t n_img, size_t n_sino,
                                                int img_blocks, const float* u_in, float* u, const float* sdir,
                                                float* r, const float* q, double* part_res, int blk, double* lds)
{
    const bool img = blk < img_blocks;
    const size_t n = img ? n_img : n_sino;
    const float* xs = img ? sdir : q;  // the direction the step moves along
    const float* ys = img ? u_in : r;  // the vector it moves
    const size_t base = (size_t)(img ? blk : blk - img_blocks) * kAxpyBlock * kAxpyPer + threadIdx.x;
    float x[kAxpyPer], y[kAxpyPer];
#pragma unroll
    for (int e = 0; e < kAxpyPer; ++e) {
        const size_t i = min(base + (size_t)e * kAxpyBlock, n - 1);
        x[e] = xs[i];
        y[e] = ys[i];
    }
    const float a = cgls_step_a(st, m, part_bp, n_bp, part_proj, n_proj, blk == 0, lds);
    if (img) {
#pragma unroll
        for (int e = 0; e < kAxpyPer; ++e) {
            const size_t i = base + (size_t)e * kAxpyBlock;
            if (i < n_img) u[i] = fmaf(a, x[e], y[e]);
        }
    } else {
        double r2 = 0.0;
#pragma unroll
        for (int e = 0; e < kAxpyPer; ++e) {
            const size_t i = base + (size_t)e * kAxpyBlock;
            if (i < n_sino) {
                const float rv = fmaf(-a, x[e], y[e]);
                r[i] = rv;
                r2 += (double)rv * (double)rv;
            }
        }
        if (part_res) {
            r2 = block_sum<kAxpyBlock>(r2, lds);
            if (threadIdx.x == 0) part_res[blk - img_blocks] = r2;
        }
    }
}

}  // namespace eptv
