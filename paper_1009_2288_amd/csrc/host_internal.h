// host_internal.h -- host-side helpers shared by the one-slice plan (plan.cpp)
// and the batch (batch.cpp).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "eptv_internal.h"
#include "tables.h"

struct eptv_plan_s {
    eptv::Plan p;
    std::mutex graph_mu;
    // page-locked host staging for reconstruct's small reads back (the RMSE
    // check, the per-iteration records): a copy into it needs no bounce
    // buffer of the runtime's.  Grown on demand; used under host_mu.
    std::mutex host_mu;
    void* host_buf = nullptr;
    size_t host_bytes = 0;
};

namespace eptv {

void set_last_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);
int reconstruct_impl(eptv_plan h, const eptv_params* q, const float* y, float* f, const float* f_ref,
                     const float* wx_in, const float* wy_in, int frozen, const int32_t* replay, void* ws,
                     size_t ws_bytes, eptv_stats* stats, void* stream, bool noalloc);

#define EPTV_HIP(call)                                            \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::eptv::hip_fail(e_, #call); \
    } while (0)

}  // namespace eptv
