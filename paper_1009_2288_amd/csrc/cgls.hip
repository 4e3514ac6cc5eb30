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
#include "batch.h"
#include "eptv_internal.h"
#include "cgls_step.h"
#include "reduce.h"
#include "state.h"

namespace eptv {

__device__ __forceinline__ void reset_iteration_state(DevState* st, uint32_t* hist, float sigma_fixed);

__global__ void k_state_init(DevState* st, uint32_t* hist, uint32_t rank, float sigma_fixed, int zero_iter)
{
    if (threadIdx.x == 0) st->rank0 = rank;
    reset_iteration_state(st, hist, sigma_fixed);
    if (threadIdx.x == 0 && zero_iter) st->iter = 0;
}

hipError_t launch_state_init(DevState* st, uint32_t* hist, uint32_t rank, float sigma_fixed, int zero_iter,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(256), 0, s, st, hist, rank, sigma_fixed, zero_iter);
    return hipGetLastError();
}

int sino_blocks(const Plan& p) { return (int)(((size_t)p.V * p.B + 1023) / 1024); }

// One CGLS step's update, u = u_in + a_m s and r -= a_m q (cgls_axpy_block).
__global__ __launch_bounds__(kAxpyBlock) void k_cgls_axpy(DevState* st, int m, const double* part_bp, int n_bp,
                                                          const double* part_proj, int n_proj, size_t n_img,
                                                          size_t n_sino, int img_blocks, const float* u_in,
                                                          float* u, const float* sdir, float* r, const float* q,
                                                          double* part_res)
{
    __shared__ double lds[4];
    cgls_axpy_block(st, m, part_bp, n_bp, part_proj, n_proj, n_img, n_sino, img_blocks, u_in, u, sdir, r, q,
                    part_res, blockIdx.x, lds);
}

int axpy_blocks(size_t n) { return (int)((n + kAxpyBlock * kAxpyPer - 1) / (kAxpyBlock * kAxpyPer)); }

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
__device__ __forceinline__ void cgls_supdate_block(DevState* st, int m, const double* part_bp, int n_bp,
                                                   const float* __restrict__ z, float* sdir, float* sdirT, int nx,
                                                   int ny, int tbx, int tby, float (*t)[33], double* lds)
{
    // the tile's s and z are loaded (at positions clamped into the image)
    // before b_m is formed, so the two memory round trips overlap
    const int bx = tbx * 32, by = tby * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    float sv[4], zv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const size_t id = (size_t)min(by + ty + 8 * c, ny - 1) * nx + min(bx + tx, nx - 1);
        sv[c] = sdir[id];
        zv[c] = z[id];
    }
    const double gn = block_sum_partials<256>(part_bp, n_bp, 1, lds);
    const float bm = st->active[m] ? (float)(gn / st->gamma[m]) : 0.0f;
    if (tbx == 0 && tby == 0 && threadIdx.x == 0) {
        st->gamma[m + 1] = gn;
        st->b[m] = bm;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int k = ty + 8 * c;
        const int i = bx + tx, j = by + k;
        float v = 0.0f;
        if (i < nx && j < ny) {
            v = fmaf(bm, sv[c], zv[c]);
            sdir[(size_t)j * nx + i] = v;
        }
        t[k][tx] = v;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int i = bx + k, j = by + tx;
        if (i < nx && j < ny) sdirT[(size_t)i * ny + j] = t[tx][k];
    }
}

__global__ __launch_bounds__(256) void k_cgls_supdate(DevState* st, int m, const double* part_bp, int n_bp,
                                                      const float* __restrict__ z, float* sdir, float* sdirT, int nx,
                                                      int ny)
{
    __shared__ float t[32][33];
    __shared__ double lds[4];
    cgls_supdate_block(st, m, part_bp, n_bp, z, sdir, sdirT, nx, ny, blockIdx.x, blockIdx.y, t, lds);
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
__device__ __forceinline__ void gd_p1_block(const float* f, const float* z, float step, float* u, size_t n, int blk,
                                            int nblk)
{
    for (size_t i = (size_t)blk * 256 + threadIdx.x; i < n; i += (size_t)nblk * 256) u[i] = fmaf(step, z[i], f[i]);
}

__global__ __launch_bounds__(256) void k_gd_p1(const float* f, const float* z, float step, float* u, size_t n)
{
    gd_p1_block(f, z, step, u, n, blockIdx.x, gridDim.x);
}

hipError_t launch_gd_p1(const Plan& p, const float* f, const float* z, float step, float* u, hipStream_t s)
{
    const size_t n = (size_t)p.nx * p.ny;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_gd_p1, dim3(blocks), dim3(256), 0, s, f, z, step, u, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ bookkeeping
__device__ __forceinline__ void rmse_part_block(const float* f, const float* ref, size_t n, double* part, int blk,
                                                int nblk, double* lds)
{
    double acc = 0.0;
    for (size_t i = (size_t)blk * 256 + threadIdx.x; i < n; i += (size_t)nblk * 256) {
        const double d = (double)f[i] - (double)ref[i];
        acc += d * d;
    }
    acc = block_sum<256>(acc, lds);
    if (threadIdx.x == 0) part[blk] = acc;
}

__global__ __launch_bounds__(256) void k_rmse_part(const float* f, const float* ref, size_t n, double* part)
{
    __shared__ double lds[4];
    rmse_part_block(f, ref, n, part, blockIdx.x, gridDim.x, lds);
}

hipError_t launch_rmse_part(const Plan& p, const float* f, const float* ref, double* part, hipStream_t s)
{
    hipLaunchKernelGGL(k_rmse_part, dim3(kRmseBlocks), dim3(256), 0, s, f, ref, (size_t)p.nx * p.ny, part);
    return hipGetLastError();
}

IterEnd iter_end_args(const Plan& p, DevState* st, const double* part_res, int with_resid, const double* part_rmse,
                      int n_rmse, int with_rmse, float* st_sigma, int32_t* st_steps, double* st_resid, double* st_rmse,
                      int M, double* st_gamma, double* st_delta, uint32_t* hist, float sigma_fixed)
{
    IterEnd e;
    e.st = st;
    e.part_res = part_res;
    e.n_res = sino_blocks(p);
    e.with_resid = with_resid;
    e.part_rmse = part_rmse;
    e.n_rmse = n_rmse;
    e.with_rmse = with_rmse;
    e.npix = (double)p.nx * p.ny;
    e.st_sigma = st_sigma;
    e.st_steps = st_steps;
    e.st_resid = st_resid;
    e.st_rmse = st_rmse;
    e.M = M;
    e.st_gamma = st_gamma;
    e.st_delta = st_delta;
    e.hist = hist;
    e.sigma_fixed = sigma_fixed;
    return e;
}

__global__ __launch_bounds__(256) void k_iter_end(IterEnd e)
{
    __shared__ double lds[4];
    iter_end_run<256>(e, lds);
}

hipError_t launch_iter_end(const IterEnd& e, hipStream_t s)
{
    hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(256), 0, s, e);
    return hipGetLastError();
}

// The optional input check: one block walks the array and records whether any
// value is NaN or infinite, as the flag's new value (first array) or or-ed
// into it (later ones), so nothing has to be cleared before.
__global__ __launch_bounds__(1024) void k_scan_finite(const float* __restrict__ a, size_t n, DevState* st,
                                                      int accumulate)
{
    int bad = 0;
    for (size_t i = threadIdx.x; i < n; i += 1024) bad |= !__builtin_isfinite(a[i]);
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) st->nonfinite = (bad || (accumulate && st->nonfinite)) ? 1 : 0;
}

hipError_t launch_scan_finite(const float* a, size_t n, DevState* st, int accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_finite, dim3(1), dim3(1024), 0, s, a, n, st, accumulate);
    return hipGetLastError();
}

// ------------------------------------------------------------------ batched kernels (see batch.h)
__global__ __launch_bounds__(kAxpyBlock) void kb_cgls_axpy(const SliceDev* __restrict__ sl,
                                                           const int2* __restrict__ items, int n_items, int m,
                                                           int u_ins, int with_res)
{
    __shared__ double lds[4];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        __syncthreads();
        cgls_axpy_block(d.st, m, d.part[kPartBp], d.t16x * d.t16y, d.part[kPartProj], d.proj_gx * d.V,
                        (size_t)d.nx * d.ny, (size_t)d.V * d.B, d.axpy_img, d.buf[u_ins], d.buf[kBufU],
                        d.buf[kBufS], d.buf[kBufR], d.buf[kBufQ], with_res ? d.part[kPartRes] : nullptr, w.y, lds);
    }
}

hipError_t blaunch_cgls_axpy(const BatchDev& b, int m, int u_in, bool with_res, hipStream_t s)
{
    const int n = b.n_items[kShAxpy];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_cgls_axpy, dim3(b.grid[kShAxpy]), dim3(kAxpyBlock), 0, s, b.slices, b.items[kShAxpy], n, m,
                       u_in, (int)with_res);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_cgls_supdate(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                       int n_items, int m)
{
    __shared__ float t[32][33];
    __shared__ double lds[4];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        __syncthreads();
        cgls_supdate_block(d.st, m, d.part[kPartBp], d.t16x * d.t16y, d.buf[kBufZ], d.buf[kBufS], d.buf[kBufST], d.nx,
                           d.ny, w.y % d.t32x, w.y / d.t32x, t, lds);
    }
}

hipError_t blaunch_cgls_supdate(const BatchDev& b, int m, hipStream_t s)
{
    const int n = b.n_items[kShT32];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_cgls_supdate, dim3(b.grid[kShT32]), dim3(256), 0, s, b.slices, b.items[kShT32], n, m);
    return hipGetLastError();
}

// gradient form of P1 over 32x32 tiles: u = f + step z
__global__ __launch_bounds__(256) void kb_gd_p1(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                int n_items, float step)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        const int bx = (w.y % d.t32x) * 32, by = (w.y / d.t32x) * 32;
        const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
        for (int k = ty; k < 32; k += 8) {
            const int i = bx + tx, j = by + k;
            if (i < d.nx && j < d.ny) {
                const size_t id = (size_t)j * d.nx + i;
                d.buf[kBufU][id] = fmaf(step, d.buf[kBufZ][id], d.buf[kBufF][id]);
            }
        }
    }
}

hipError_t blaunch_gd_p1(const BatchDev& b, float step, hipStream_t s)
{
    const int n = b.n_items[kShT32];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_gd_p1, dim3(b.grid[kShT32]), dim3(256), 0, s, b.slices, b.items[kShT32], n, step);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_rmse_part(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                    int n_items, int fs)
{
    __shared__ double lds[4];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        if (!d.buf[kBufFRef]) continue;  // uniform per item
        __syncthreads();
        rmse_part_block(d.buf[fs], d.buf[kBufFRef], (size_t)d.nx * d.ny, d.part[kPartRmse], w.y, kRmseBlocks, lds);
    }
}

hipError_t blaunch_rmse_part(const BatchDev& b, int f, hipStream_t s)
{
    const int n = b.n_items[kShRmse];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_rmse_part, dim3(b.grid[kShRmse]), dim3(256), 0, s, b.slices, b.items[kShRmse], n, f);
    return hipGetLastError();
}

// one block per slice
// rmse_tiles: the squared errors come from the final update's 32 x 32 tiles
// (else from the RMSE kernel's kRmseBlocks partials)
__global__ __launch_bounds__(256) void kb_iter_end(const SliceDev* __restrict__ sl, int with_resid, int with_rmse,
                                                   int rmse_tiles, float sigma_fixed)
{
    __shared__ double lds[4];
    const SliceDev& d = sl[blockIdx.x];
    IterEnd e;
    e.st = d.st;
    e.part_res = d.part[kPartRes];
    e.n_res = d.axpy_sino;
    e.with_resid = with_resid;
    e.part_rmse = d.part[kPartRmse];
    e.n_rmse = rmse_tiles ? d.t32x * d.t32y : kRmseBlocks;
    e.with_rmse = with_rmse && d.buf[kBufFRef] != nullptr;
    e.npix = (double)d.nx * d.ny;
    e.st_sigma = d.st_sigma;
    e.st_steps = d.st_steps;
    e.st_resid = d.st_resid;
    e.st_rmse = d.st_rmse;
    e.M = d.cgls_iters;
    e.st_gamma = d.st_gamma;
    e.st_delta = d.st_delta;
    e.hist = d.hist;
    e.sigma_fixed = sigma_fixed;
    iter_end_run<256>(e, lds);
}

hipError_t blaunch_iter_end(const BatchDev& b, bool with_resid, bool with_rmse, bool rmse_tiles, float sigma_fixed,
                            hipStream_t s)
{
    hipLaunchKernelGGL(kb_iter_end, dim3(b.n), dim3(256), 0, s, b.slices, (int)with_resid, (int)with_rmse,
                       (int)rmse_tiles, sigma_fixed);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_state_init(const SliceDev* __restrict__ sl, float sigma_fixed, int zero_iter)
{
    const SliceDev& d = sl[blockIdx.x];
    if (threadIdx.x == 0) d.st->rank0 = d.rank;
    reset_iteration_state(d.st, d.hist, sigma_fixed);
    if (threadIdx.x == 0 && zero_iter) d.st->iter = 0;
}

hipError_t blaunch_state_init(const BatchDev& b, float sigma_fixed, int zero_iter, hipStream_t s)
{
    hipLaunchKernelGGL(kb_state_init, dim3(b.n), dim3(256), 0, s, b.slices, sigma_fixed, zero_iter);
    return hipGetLastError();
}

}  // namespace eptv
