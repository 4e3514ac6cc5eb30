// noalloc.hip -- eptv_reconstruct_noalloc: eptv_reconstruct with its
// workspace in a fixed device array of the library, for callers that cannot
// allocate device memory.
//
// The array `scratch` is a file-scope __device__ object: every GPU the library
// runs on holds its own copy (kScratchBytes) from the code object's load until
// the process ends.  In host code its name is only a host-side stand-in, so
// the device address is looked up once per device with hipGetSymbolAddress
// and kept; the kernels receive that address exactly as they receive a
// caller's workspace.  All calls on one GPU share its copy: calls that overlap
// on one GPU (other streams, other threads) race on it.  The contents need no
// clearing: the iteration's first kernel resets the device state, and every
// other buffer is written before it is read, as with a caller's workspace.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host_internal.h"

// 32 MiB: the workspace of a 512 x 512 image (about 20 MiB) with room for
// hundreds of thousands of per-iteration records
static constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's copy of `scratch`.
int scratch_address(void** out)
{
    int dev = -1;
    EPTV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        eptv::set_last_error("eptv_reconstruct_noalloc: device ordinal " + std::to_string(dev) + " out of range");
        return EPTV_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return eptv::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) {
            eptv::set_last_error("hipGetSymbolAddress(scratch) returned a null address");
            return EPTV_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return EPTV_OK;
}

}  // namespace

extern "C" {

size_t eptv_noalloc_scratch_bytes(void) { return kScratchBytes; }

int eptv_reconstruct_noalloc(eptv_plan h, const eptv_params* q, const float* y, float* f, const float* f_ref,
                             eptv_stats* stats, void* stream)
{
    if (!h || !q) return EPTV_ERR_ARG;
    size_t need = 0;
    int rc = eptv_workspace_bytes(h, q, &need);
    if (rc != EPTV_OK) return rc;
    if (need > kScratchBytes) {
        eptv::set_last_error("eptv_reconstruct_noalloc: the workspace needs " + std::to_string(need) +
                             " bytes, more than the library's fixed " + std::to_string(kScratchBytes));
        return EPTV_ERR_WORKSPACE;
    }
    int dev = -1;
    EPTV_HIP(hipGetDevice(&dev));
    if (dev != h->p.device) {
        eptv::set_last_error("eptv_reconstruct_noalloc: the current device is not the plan's");
        return EPTV_ERR_ARG;
    }
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != EPTV_OK) return rc;
    return eptv::reconstruct_impl(h, q, y, f, f_ref, nullptr, nullptr, 0, nullptr, ws, kScratchBytes, stats, stream,
                                  true);
}

}  // extern "C"
