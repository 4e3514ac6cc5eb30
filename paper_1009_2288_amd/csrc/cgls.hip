// cgls.hip -- the P1 data step (App. I: CGLS on min ||P u - y||^2 started at
// f^(k)) and per-iteration bookkeeping.
//
// CGLS keeps every scalar on the device.  The projector and the
// backprojector write one float64 partial of ||P s||^2 / ||P^T r||^2 per
// block; the vector kernel that needs the scalar sums those partials itself,
// in a fixed order, in every block (a few thousand loads from L2 per block),
// so no separate scalar kernel is launched and an outer iteration needs no
// host synchronisation.  Block 0 records the scalars for later kernels.
//
//   step m:  gamma_m = ||P^T r_m||^2, delta_m = ||P s_m||^2,
//            a_m = gamma_m / delta_m, u += a_m s, r -= a_m P s,
//            b_m = gamma_{m+1} / gamma_m, s = P^T r_{m+1} + b_m s.
// Breakdown (delta_m = 0, or gamma_m <= 1e-30 gamma_0) freezes the iterate for
// the remaining steps.
#include "eptv_internal.h"
#include "reduce.h"

namespace eptv {

__global__ void k_state_init(DevState* st, uint32_t* hist, uint32_t rank, float sigma_fixed, int zero_iter)
{
    const int t = threadIdx.x;
    for (int i = t; i < 3 * kSelectBins; i += blockDim.x) hist[i] = 0u;
    if (t == 0) {
        st->cg_steps = 0;
        st->prefix = 0u;
        st->rank = rank;
        st->sigma = sigma_fixed;
        st->inv_sigma2 = sigma_fixed >= 0.0f ? 1.0f / (sigma_fixed * sigma_fixed) : 0.0f;
        st->decided = 0;
        st->k = -1;
        st->t = 0.0f;
        if (zero_iter) st->iter = 0;
    }
}

hipError_t launch_state_init(DevState* st, uint32_t* hist, uint32_t rank, float sigma_fixed, int zero_iter,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(256), 0, s, st, hist, rank, sigma_fixed, zero_iter);
    return hipGetLastError();
}

int sino_blocks(const Plan& p) { return (int)(((size_t)p.V * p.B + 1023) / 1024); }

// u = u_in + a_m s (image part) and r = r - a_m q (sinogram part), one launch.
// Every block first forms a_m from gamma_m (the backprojector's partials for
// m = 0, else the value recorded by the previous s-update) and delta_m (the
// projector's partials).  When part_res is given the sinogram blocks also
// emit ||r||^2.
constexpr int kAxpyBlock = 256;
constexpr int kAxpyPer = 4;

__global__ __launch_bounds__(kAxpyBlock) void k_cgls_axpy(DevState* st, int m, const double* part_bp, int n_bp,
                                                          const double* part_proj, int n_proj, size_t n_img,
                                                          size_t n_sino, int img_blocks, const float* u_in,
                                                          float* u, const float* sdir, float* r, const float* q,
                                                          double* part_res)
{
    __shared__ double lds[4];
    const double g = m == 0 ? block_sum_partials<kAxpyBlock>(part_bp, n_bp, 1, lds) : st->gamma[m];
    const double d = block_sum_partials<kAxpyBlock>(part_proj, n_proj, 1, lds);
    const double g0 = m == 0 ? g : st->gamma0;
    const int was = m == 0 ? 1 : st->active[m - 1];
    const int active = was && (g > 1e-30 * g0) && (d > 0.0);
    const float a = active ? (float)(g / d) : 0.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (m == 0) {
            st->gamma[0] = g;
            st->gamma0 = g;
        }
        st->a[m] = a;
        st->active[m] = active;
        if (active) st->cg_steps = m + 1;
    }
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
        if (part_res) {
            r2 = block_sum<kAxpyBlock>(r2, lds);
            if (threadIdx.x == 0) part_res[blockIdx.x - img_blocks] = r2;
        }
    }
}

static int axpy_blocks(size_t n) { return (int)((n + kAxpyBlock * kAxpyPer - 1) / (kAxpyBlock * kAxpyPer)); }

hipError_t launch_cgls_axpy(const Plan& p, DevState* st, int m, const double* part_bp, const double* part_proj,
                            const float* u_in, float* u, const float* sdir, float* r, const float* q,
                            double* part_res, hipStream_t s)
{
    const size_t ni = (size_t)p.nx * p.ny, ns = (size_t)p.V * p.B;
    const int bi = axpy_blocks(ni), bs = axpy_blocks(ns);
    hipLaunchKernelGGL(k_cgls_axpy, dim3(bi + bs), dim3(kAxpyBlock), 0, s, st, m, part_bp, image_tile_blocks(p),
                       part_proj, project_blocks(p), ni, ns, bi, u_in, u, sdir, r, q, part_res);
    return hipGetLastError();
}

// s = z + b_m s, written row-major and transposed (the projector reads both);
// b_m = gamma_{m+1} / gamma_m with gamma_{m+1} summed from the backprojector's
// partials and recorded for step m+1.
__global__ __launch_bounds__(256) void k_cgls_supdate(DevState* st, int m, const double* part_bp, int n_bp,
                                                      const float* __restrict__ z, float* sdir, float* sdirT, int nx,
                                                      int ny)
{
    __shared__ float t[32][33];
    __shared__ double lds[4];
    const double gn = block_sum_partials<256>(part_bp, n_bp, 1, lds);
    const float bm = st->active[m] ? (float)(gn / st->gamma[m]) : 0.0f;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        st->gamma[m + 1] = gn;
        st->b[m] = bm;
    }
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

hipError_t launch_cgls_supdate(const Plan& p, DevState* st, int m, const double* part_bp, const float* z,
                               float* sdir, float* sdirT, hipStream_t s)
{
    dim3 grid((p.nx + 31) / 32, (p.ny + 31) / 32);
    hipLaunchKernelGGL(k_cgls_supdate, grid, dim3(256), 0, s, st, m, part_bp, image_tile_blocks(p), z, sdir, sdirT,
                       p.nx, p.ny);
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

hipError_t launch_rmse_part(const Plan& p, const float* f, const float* ref, double* part, hipStream_t s)
{
    hipLaunchKernelGGL(k_rmse_part, dim3(kRmseBlocks), dim3(256), 0, s, f, ref, (size_t)p.nx * p.ny, part);
    return hipGetLastError();
}

// Per-iteration records, then the iteration counter.
__global__ __launch_bounds__(256) void k_iter_end(DevState* st, const double* part_res, int n_res, int with_resid,
                                                  const double* part_rmse, int with_rmse, double npix,
                                                  float* st_sigma, int32_t* st_steps, double* st_resid,
                                                  double* st_rmse)
{
    __shared__ double lds[4];
    const double res = with_resid ? block_sum_partials<256>(part_res, n_res, 1, lds) : 0.0;
    const double e = with_rmse ? block_sum_partials<256>(part_rmse, kRmseBlocks, 1, lds) : 0.0;
    if (threadIdx.x == 0) {
        const int it = st->iter;
        if (st_sigma) st_sigma[it] = st->sigma;
        if (st_steps) st_steps[it] = st->cg_steps;
        if (st_resid) st_resid[it] = res;
        if (with_rmse && st_rmse) st_rmse[it] = sqrt(e / npix);
        st->iter = it + 1;
    }
}

hipError_t launch_iter_end(const Plan& p, DevState* st, const double* part_res, int with_resid,
                           const double* part_rmse, int with_rmse, float* st_sigma, int32_t* st_steps,
                           double* st_resid, double* st_rmse, hipStream_t s)
{
    hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(256), 0, s, st, part_res, sino_blocks(p), with_resid, part_rmse,
                       with_rmse, (double)p.nx * p.ny, st_sigma, st_steps, st_resid, st_rmse);
    return hipGetLastError();
}

}  // namespace eptv
