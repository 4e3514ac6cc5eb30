// host_internal.h -- host-side helpers shared by the one-slice plan (plan.cpp)
// and the batch (batch.cpp).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "eptv_internal.h"

struct eptv_plan_s {
    eptv::Plan p;
    std::mutex graph_mu;
};

namespace eptv {

void set_last_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);
int validate_geometry(const eptv_geometry* g);
int check_params(const eptv_params* q);
uint32_t select_rank(const Plan& p, double q);
float t0_of(const eptv_params& q);
float sigma_init(const eptv_params& q);

#define EPTV_HIP(call)                                            \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::eptv::hip_fail(e_, #call); \
    } while (0)

}  // namespace eptv
