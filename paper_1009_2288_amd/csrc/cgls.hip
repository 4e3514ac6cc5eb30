// cgls.hip -- the P1 data step (App. I: CGLS on min ||P u - y||^2 started at
// f^(k)) and per-iteration bookkeeping.
//
// CGLS keeps every scalar on the device: reductions of ||P^T r||^2 and
// ||P s||^2 are written as one float64 partial per block by the producing
// kernel (projector / backprojector epilogue), summed in a fixed order by a
// one-block finalise kernel, and read by the vector kernels that follow, so
// an outer iteration needs no host synchronisation and can be replayed as a
// graph.  Breakdown (||P s|| = 0, or ||P^T r||^2 <= 1e-30 of its first value)
// freezes the iterate for the remaining steps.
#include "eptv_internal.h"
#include "reduce.h"

namespace eptv {

__global__ void k_state_init(DevState* st, uint32_t* hist, uint32_t rank, float sigma_fixed, int zero_iter)
{
    const int t = threadIdx.x;
    for (int i = t; i < 3 * kSelectBins; i += blockDim.x) hist[i] = 0u;
    if (t == 0) {
        st->cg_active = 1;
        st->cg_steps = 0;
        st->resid = 0.0;
        st->prefix = 0u;
        st->rank = rank;
        st->rank0 = rank;
        st->sigma = sigma_fixed;
        st->inv_sigma2 = sigma_fixed >= 0.0f ? 1.0f / (sigma_fixed * sigma_fixed) : 0.0f;
        st->decided = 0;
        st->k = -1;
        st->t = 0.0f;
        if (zero_iter) st->iter = 0;
    }
}

hipError_t launch_state_init(DevState* st, uint32_t* hist, uint32_t rank, float sigma_fixed,
                             int zero_iter, hipStream_t s)
{
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(256), 0, s, st, hist, rank, sigma_fixed, zero_iter);
    return hipGetLastError();
}

// gamma_m = ||P^T r_m||^2 (m = 0: the initial residual, which also re-arms CGLS)
__global__ __launch_bounds__(256) void k_cgls_gamma(DevState* st, const double* part, int n, int m)
{
    __shared__ double lds[4];
    const double g = block_sum_array(part, n, 1, lds);
    if (threadIdx.x == 0) {
        st->gamma[m] = g;
        if (m == 0) {
            st->gamma0 = g;
            st->cg_active = 1;
            st->cg_steps = 0;
        } else {
            st->b[m - 1] = st->cg_active ? (float)(g / st->gamma[m - 1]) : 0.0f;
        }
    }
}

hipError_t launch_cgls_gamma(DevState* st, const double* part, int nparts, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_cgls_gamma, dim3(1), dim3(256), 0, s, st, part, nparts, m);
    return hipGetLastError();
}

// delta_m = ||P s_m||^2, a_m = gamma_m / delta_m
__global__ __launch_bounds__(256) void k_cgls_delta(DevState* st, const double* part, int n, int m)
{
    __shared__ double lds[4];
    const double d = block_sum_array(part, n, 1, lds);
    if (threadIdx.x == 0) {
        st->delta[m] = d;
        const double g = st->gamma[m];
        int active = st->cg_active && (g > 1e-30 * st->gamma0) && (d > 0.0);
        st->cg_active = active;
        st->a[m] = active ? (float)(g / d) : 0.0f;
        if (active) st->cg_steps = m + 1;
    }
}

hipError_t launch_cgls_delta(DevState* st, const double* part, int nparts, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_cgls_delta, dim3(1), dim3(256), 0, s, st, part, nparts, m);
    return hipGetLastError();
}

// u = u_in + a_m s (image part) and r = r - a_m q (sinogram part), one launch.
// When part_r2 is given the blocks covering the sinogram also emit ||r||^2.
constexpr int kAxpyBlock = 256;
constexpr int kAxpyPer = 4;

__global__ __launch_bounds__(kAxpyBlock) void k_cgls_axpy(const DevState* st, int m, size_t n_img, size_t n_sino,
                                                          int img_blocks, const float* u_in, float* u,
                                                          const float* sdir, float* r, const float* q,
                                                          double* part_r2)
{
    __shared__ double lds[4];
    const float a = st->a[m];
    if ((int)blockIdx.x < img_blocks) {
        const size_t base = (size_t)blockIdx.x * kAxpyBlock * kAxpyPer + threadIdx.x;
#pragma unroll
        for (int e = 0; e < kAxpyPer; ++e) {
            const size_t i = base + (size_t)e * kAxpyBlock;
            if (i < n_img) u[i] = fmaf(a, sdir[i], u_in[i]);
        }
    } else {
        const size_t base = (size_t)(blockIdx.x - img_blocks) * kAxpyBlock * kAxpyPer + threadIdx.x;
        double r2 = 0.0;
#pragma unroll
        for (int e = 0; e < kAxpyPer; ++e) {
            const size_t i = base + (size_t)e * kAxpyBlock;
            if (i < n_sino) {
                const float rv = fmaf(-a, q[i], r[i]);
                r[i] = rv;
                r2 += (double)rv * (double)rv;
            }
        }
        if (part_r2) {
            r2 = block_sum<kAxpyBlock>(r2, lds);
            if (threadIdx.x == 0) part_r2[blockIdx.x - img_blocks] = r2;
        }
    }
}

static int axpy_blocks(size_t n) { return (int)((n + kAxpyBlock * kAxpyPer - 1) / (kAxpyBlock * kAxpyPer)); }

hipError_t launch_cgls_axpy(const Plan& p, DevState* st, int m, const float* u_in, float* u,
                            const float* sdir, float* r, const float* q, double* part_r2, hipStream_t s)
{
    const size_t ni = (size_t)p.nx * p.ny, ns = (size_t)p.V * p.B;
    const int bi = axpy_blocks(ni), bs = axpy_blocks(ns);
    hipLaunchKernelGGL(k_cgls_axpy, dim3(bi + bs), dim3(kAxpyBlock), 0, s, st, m, ni, ns, bi, u_in, u,
                       sdir, r, q, part_r2);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_cgls_resid(DevState* st, const double* part, int n)
{
    __shared__ double lds[4];
    const double v = block_sum_array(part, n, 1, lds);
    if (threadIdx.x == 0) st->resid = v;
}

hipError_t launch_cgls_resid(DevState* st, const double* part, int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_cgls_resid, dim3(1), dim3(256), 0, s, st, part, nparts);
    return hipGetLastError();
}

// s = z + b_m s, written row-major and transposed (the projector reads both).
__global__ __launch_bounds__(256) void k_cgls_supdate(const DevState* st, int m, const float* __restrict__ z,
                                                      float* sdir, float* sdirT, int nx, int ny)
{
    __shared__ float t[32][33];
    const float bm = st->b[m];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int i = bx + tx, j = by + k;
        float v = 0.0f;
        if (i < nx && j < ny) {
            const size_t id = (size_t)j * nx + i;
            v = fmaf(bm, sdir[id], z[id]);
            sdir[id] = v;
        }
        t[k][tx] = v;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int i = bx + k, j = by + tx;
        if (i < nx && j < ny) sdirT[(size_t)i * ny + j] = t[tx][k];
    }
}

hipError_t launch_cgls_supdate(const Plan& p, DevState* st, int m, const float* z, float* sdir,
                               float* sdirT, hipStream_t s)
{
    dim3 grid((p.nx + 31) / 32, (p.ny + 31) / 32);
    hipLaunchKernelGGL(k_cgls_supdate, grid, dim3(256), 0, s, st, m, z, sdir, sdirT, p.nx, p.ny);
    return hipGetLastError();
}

// Gradient form of P1 (Eq. 8): v = f - mu/lambda P^T (P f - y) = f + step * P^T r.
__global__ void k_gd_p1(const float* f, const float* z, float step, float* u, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        u[i] = fmaf(step, z[i], f[i]);
}

hipError_t launch_gd_p1(const Plan& p, const float* f, const float* z, float step, float* u, hipStream_t s)
{
    const size_t n = (size_t)p.nx * p.ny;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_gd_p1, dim3(blocks), dim3(256), 0, s, f, z, step, u, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ bookkeeping
__global__ __launch_bounds__(256) void k_rmse_part(const float* f, const float* ref, size_t n, double* part)
{
    __shared__ double lds[4];
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double d = (double)f[i] - (double)ref[i];
        acc += d * d;
    }
    acc = block_sum<256>(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

constexpr int kRmseBlocks = 256;

hipError_t launch_rmse_part(const Plan& p, const float* f, const float* ref, double* part, hipStream_t s)
{
    hipLaunchKernelGGL(k_rmse_part, dim3(kRmseBlocks), dim3(256), 0, s, f, ref, (size_t)p.nx * p.ny, part);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_iter_end(DevState* st, const double* rpart, int n, int with_rmse,
                                                  double npix, float* st_sigma, int32_t* st_steps,
                                                  double* st_resid, double* st_rmse)
{
    __shared__ double lds[4];
    double e = 0.0;
    if (with_rmse) e = block_sum_array(rpart, n, 1, lds);
    if (threadIdx.x == 0) {
        const int it = st->iter;
        if (st_sigma) st_sigma[it] = st->sigma;
        if (st_steps) st_steps[it] = st->cg_steps;
        if (st_resid) st_resid[it] = st->resid;
        if (with_rmse && st_rmse) st_rmse[it] = sqrt(e / npix);
        st->iter = it + 1;
    }
}

hipError_t launch_iter_end(DevState* st, const double* rmse_part, double npix, int with_rmse,
                           float* st_sigma, int32_t* st_steps, double* st_resid, double* st_rmse,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(256), 0, s, st, rmse_part, kRmseBlocks, with_rmse, npix,
                       st_sigma, st_steps, st_resid, st_rmse);
    return hipGetLastError();
}

}  // namespace eptv
