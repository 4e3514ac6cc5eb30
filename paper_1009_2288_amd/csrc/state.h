// state.h -- reset of the per-iteration device state and the close of an
// outer iteration, shared by the kernels that start a run, the one that closes
// each outer iteration, and the projector launch that can close the previous
// one in a block of its own.
#pragma once

#include "eptv_internal.h"
#include "reduce.h"

namespace eptv {

// Per-iteration records, the iteration counter, and the reset of the
// per-iteration state for the next iteration (histograms, CGLS step count,
// selection prefix, sigma), so no kernel of its own is needed.
__device__ __forceinline__ void reset_iteration_state(DevState* st, uint32_t* hist, float sigma_fixed)
{
    for (int i = threadIdx.x; i < 3 * kSelectBins; i += blockDim.x) hist[i] = 0u;
    if (threadIdx.x == 0) {
        st->cg_steps = 0;
        st->prefix = 0u;
        st->rank = st->rank0;
        st->sigma = sigma_fixed;
        st->inv_sigma2 = sigma_fixed >= 0.0f ? 1.0f / (sigma_fixed * sigma_fixed) : 0.0f;
    }
}

// Sum of part[0..n) in the order of a 256-thread block_sum_partials (thread i
// sums i, i + 256, ...; waves in order), by a block of NT >= 256 threads: the
// threads past 256 add zeros after the others, so the bits are the same
// whatever NT.  Valid in every thread; `lds` holds NT / 64 doubles.
template <int NT>
__device__ __forceinline__ double partials_sum256(const double* part, int n, double* lds)
{
    static_assert(NT >= 256 && NT % 64 == 0, "block shape");
    double v = 0.0;
    if (threadIdx.x < 256)
        for (int i = threadIdx.x; i < n; i += 256) v += part[i];
    return block_sum<NT>(v, lds);
}

// The close of an outer iteration by one block of NT threads: ||r||^2 from
// the last CGLS step's partials and the squared error to the reference from
// the RMSE partials (the RMSE kernel's, or the final P2 update's per tile),
// the iteration's records, the counter, and reset_iteration_state.
template <int NT>
__device__ __forceinline__ void iter_end_run(const IterEnd& e, double* lds)
{
    DevState* st = e.st;
    const double res = e.with_resid ? partials_sum256<NT>(e.part_res, e.n_res, lds) : 0.0;
    const double sq = e.with_rmse ? partials_sum256<NT>(e.part_rmse, e.n_rmse, lds) : 0.0;
    const int it = st->iter;
    // the CGLS scalars of the steps reached (gamma_m is recorded for every
    // step that the previous ones left active, including one it stopped)
    for (int m = threadIdx.x; m < e.M; m += NT) {
        const int reached = m == 0 || st->active[m - 1];
        if (e.st_gamma) e.st_gamma[(size_t)it * e.M + m] = reached ? st->gamma[m] : 0.0;
        if (e.st_delta) e.st_delta[(size_t)it * e.M + m] = reached ? st->delta[m] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (e.st_sigma) e.st_sigma[it] = st->sigma;
        if (e.st_steps) e.st_steps[it] = st->cg_steps;
        if (e.st_resid) e.st_resid[it] = res;
        if (e.with_rmse && e.st_rmse) e.st_rmse[it] = sqrt(sq / e.npix);
        st->iter = it + 1;
    }
    __syncthreads();
    reset_iteration_state(st, e.hist, e.sigma_fixed);
}

}  // namespace eptv
