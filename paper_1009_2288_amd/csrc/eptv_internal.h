// eptv_internal.h -- plan layout, device state and kernel launchers of libeptv.
//
// Internal to the HIP library; the public contract is include/eptv.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/eptv.h"

namespace eptv {

// ---------------------------------------------------------------- rays
// Every ray is stored in "sweep form".  A ray that is closer to the x axis
// (|cos| >= |sin|) is swept column by column: in column k it enters at the
// continuous row coordinate e(k) = e0 + k*slope and leaves at e(k+1) (row
// units: 0 at the image bottom edge, 1 per pixel, |slope| <= 1).  A ray closer
// to the y axis is swept row by row with the roles of rows and columns
// exchanged.  e is held in 32.32 fixed point, E(k) = E0 + k*S, so stepping
// along the ray is exact integer arithmetic and a crossing of a row boundary is
// located to ~1e-10 pixel however shallow the ray.  The length of the ray
// inside cell (k, m) of its sweep, with lo/hi the smaller/larger of E(k),
// E(k+1), m0 = floor(lo), m1 = floor(hi) (m1 <= m0 + 1), is
//     S == 0:            wfull                   if m == m0
//     m0 == m1:          (hi - lo) * w32         if m == m0
//     m1 == m0 + 1:      (2^32 - frac(lo)) * w32 if m == m0,  frac(hi) * w32 if m == m1
// and 0 elsewhere, where w32 = 2^-32 d/|sin| (d/|cos| for row sweeps) is the
// length per fixed-point unit of row crossed and wfull = d/|cos| (d/|sin|) the
// length across a whole column (row).  Both the projector and the
// backprojector evaluate exactly this expression with the same integer and
// float operations, so their float32 matrices are transposes of each other.
struct RayTable {
    longlong2* d_fx = nullptr;  // [V*B] (E0, S)
    float2* d_w = nullptr;      // [V*B] (w32, +-wfull); wfull < 0 marks a row sweep
    int2* d_range = nullptr;    // [V*B] sweep range [k_lo, k_hi) that can meet the image
    float2* d_view = nullptr;   // [V] (cos theta, sin theta)
};

// Ray length in cross cell m of the sweep cell whose boundaries are at E(k) = ea
// and E(k+1) = eb (32.32 fixed point), given S = eb - ea.
__device__ __forceinline__ float chord_fx(long long ea, long long eb, long long S, int m, float w32, float wfull)
{
    const long long lo = S >= 0 ? ea : eb, hi = S >= 0 ? eb : ea;
    const int m0 = (int)(lo >> 32), m1 = (int)(hi >> 32);
    if (S == 0) return m == m0 ? wfull : 0.0f;
    const unsigned flo = (unsigned)lo, fhi = (unsigned)hi;
    if (m == m0) return (m1 == m0 ? (float)(fhi - flo) : 4294967296.0f - (float)flo) * w32;
    if (m == m1) return (float)fhi * w32;
    return 0.0f;
}

// ---------------------------------------------------------------- device state
constexpr int kMaxCgls = 64;
constexpr int kSelectBins = 2048;       // 11-bit radix digits
constexpr int kArmijoCand = 16;         // Armijo candidates evaluated per pass

struct DevState {
    // P1 (CGLS)
    double gamma[kMaxCgls + 1];  // ||P^T r||^2 before step m
    double delta[kMaxCgls];      // ||P s||^2 at step m
    double gamma0;
    float a[kMaxCgls], b[kMaxCgls];
    int cg_active;
    int cg_steps;
    double resid;
    // sigma selection
    uint32_t prefix;
    uint32_t rank;
    uint32_t rank0;
    float sigma;
    float inv_sigma2;
    // P2 (Armijo)
    double q0, gg;
    int decided;
    int k;
    float t;
    // bookkeeping
    int iter;
    double rmse_acc;
    int pad[8];
};

struct Plan {
    int nx = 0, ny = 0, V = 0, B = 0;
    double pixel = 0, dbeta = 0, bin_offset = 0, sad = 0, sdd = 0;
    std::vector<double> angles;
    long long nnz = 0;
    int device = 0;
    RayTable rays;
    hipStream_t cap_stream = nullptr;
    // cached graph of one outer iteration
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> gkey;
};

// ---------------------------------------------------------------- workspace
struct Workspace {
    float* fT;      // transposed image for the projector [nx][ny]
    float* u;       // CGLS iterate / v
    float* s;       // CGLS direction
    float* sT;      // its transposed copy
    float* z;       // backprojection P^T r
    float* g;       // P2 direction
    float* wx;      // x-edge weights [ny][nx+1]
    float* wy;      // y-edge weights [ny+1][nx]
    float* r;       // CGLS residual [V][B]
    float* q;       // P s [V][B]
    uint32_t* keys; // edge magnitude bit patterns [n_edges]
    uint32_t* hist; // [3][kSelectBins]
    double* part;   // per-block partial sums
    DevState* st;
    float* st_sigma;     // [K]
    int32_t* st_k;       // [K*T]
    int32_t* st_steps;   // [K]
    double* st_resid;    // [K]
    double* st_rmse;     // [K]
    size_t bytes;
};

size_t workspace_layout(const Plan& p, int K, int T, char* base, Workspace* w);

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return hipGetLastError().
size_t n_edges(const Plan& p);
int project_blocks(const Plan& p);
int image_tile_blocks(const Plan& p);
int armijo_blocks(const Plan& p);
int select_blocks(const Plan& p);

hipError_t launch_transpose(const float* src, float* dst, int nx, int ny, hipStream_t s);
hipError_t launch_fill(float* dst, size_t n, float value, hipStream_t s);
hipError_t launch_project(const Plan& p, const float* x, const float* xT, float alpha, float beta,
                          const float* c, float* q, double* partial, hipStream_t s);
hipError_t launch_backproject(const Plan& p, const float* r, float alpha, float beta, const float* c,
                              float* z, float* zT, double* partial, hipStream_t s);

// CGLS glue
hipError_t launch_state_init(DevState* st, uint32_t* hist, uint32_t rank, float sigma_fixed,
                             int zero_iter, hipStream_t s);
hipError_t launch_cgls_gamma(DevState* st, const double* part, int nparts, int m, hipStream_t s);
hipError_t launch_cgls_delta(DevState* st, const double* part, int nparts, int m, hipStream_t s);
hipError_t launch_cgls_axpy(const Plan& p, DevState* st, int m, const float* u_in, float* u,
                            const float* sdir, float* r, const float* q, double* part_r2, hipStream_t s);
hipError_t launch_cgls_resid(DevState* st, const double* part, int nparts, hipStream_t s);
hipError_t launch_cgls_supdate(const Plan& p, DevState* st, int m, const float* z, float* sdir,
                               float* sdirT, hipStream_t s);
hipError_t launch_gd_p1(const Plan& p, const float* f, const float* z, float step, float* u,
                        hipStream_t s);

// sigma
hipError_t launch_edges_hist(const Plan& p, const float* f, float eps2, uint32_t* keys,
                             uint32_t* hist0, hipStream_t s);
hipError_t launch_select_hist(const Plan& p, int pass, const uint32_t* keys, const DevState* st,
                              uint32_t* hist, hipStream_t s);
hipError_t launch_select_finalize(DevState* st, int pass, uint32_t* hist, float sigma_floor,
                                  hipStream_t s);
hipError_t launch_sigma_out(const DevState* st, float* out, hipStream_t s);

// P2
hipError_t launch_tv_grad(const Plan& p, const float* f, const float* v, float lambda,
                          const DevState* st, float sigma_direct, float eps2, float* g, float* wx,
                          float* wy, double* part, hipStream_t s);
hipError_t launch_grad_finalize(DevState* st, const double* part, int nparts, hipStream_t s);
hipError_t launch_armijo(const Plan& p, int pass, const float* f, const float* g, const float* v,
                         const float* wx, const float* wy, float lambda, float eps2, float t0,
                         float shrink, const DevState* st, double* part, hipStream_t s);
hipError_t launch_armijo_finalize(DevState* st, const double* part, int nparts, int pass,
                                  int max_bt, double c, double t0, double shrink, hipStream_t s);
hipError_t launch_p2_update(const Plan& p, const DevState* st, const float* fcur, const float* g,
                            float* fout, float* foutT, int clamp, int32_t* st_k, int step,
                            int T, hipStream_t s);
hipError_t launch_copy_clamp(const Plan& p, const float* src, float* dst, float* dstT, int clamp,
                             hipStream_t s);

// bookkeeping
hipError_t launch_rmse_part(const Plan& p, const float* f, const float* ref, double* part,
                            hipStream_t s);
hipError_t launch_iter_end(DevState* st, const double* rmse_part, double npix, int with_rmse,
                           float* st_sigma, int32_t* st_steps, double* st_resid, double* st_rmse,
                           hipStream_t s);

}  // namespace eptv
