// state.h -- reset of the per-iteration device state, shared by the kernels
// that start a run and the one that closes each outer iteration.
#pragma once

#include "eptv_internal.h"

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

// ||r||^2 from n_res partials, the squared error to the reference from
// n_rmse partials (the RMSE kernel's, or the final P2 update's per tile).

}  // namespace eptv
