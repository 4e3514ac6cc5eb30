// proj.hip -- forward projection P and its exact transpose P^T on gfx950.
//
// P (Sec. 2.1, Eq. 1): entry p_ij is the length of ray i inside pixel j.
// The projector is ray-driven, one lane per ray (Sec. 2.3): a wave holds 64
// consecutive detector bins of one view, so the output row q[v][b..b+63] is
// written with one coalesced store.  Each ray is swept along its dominant axis
// (see RayTable); the sweep is split into NSEG segments handled by the waves of
// a block and summed in LDS in a fixed order, and each wave evaluates four
// sweep cells at a time without branches so their loads are in flight together.  Rays swept column by column read
// the transposed image, so the 64 lanes of a wave, which sit in neighbouring
// rows of one column, touch contiguous memory in both sweep directions.
//
// P^T is computed per 16x16 pixel tile (Sec. 2.3: the tile's block owns its
// pixels, so the write conflicts of a ray-driven scatter cannot arise): the
// rays that can meet the tile are walked through it with the projector's own
// cell arithmetic, so the float32 P^T is exactly the transpose of the float32
// P (not the interpolating approximation of Eq. 11, which is provided
// separately).  Summation order is fixed; there are no atomics.
//
// Each kernel's per-block work is a __device__ function of the block's
// coordinates, shared by the one-slice kernels here and the batched kernels
// (batch.hip), which walk a list of (slice, block) items.
#include "batch.h"
#include "eptv_internal.h"
#include "tables.h"
#include "reduce.h"
#include "state.h"

namespace eptv {

// ------------------------------------------------------------------ projector
#ifndef EPTV_PROJ_SEG
#define EPTV_PROJ_SEG 16
#endif
constexpr int kProjSeg = EPTV_PROJ_SEG;  // sweep segments (waves) per block of 64 rays
constexpr int kProjUnroll = 4;           // sweep cells whose loads are issued together

// Contribution of one sweep cell: the (at most two) pixels the ray crosses in
// it, m0 and m0 + 1, neighbours along the line the image layout stores
// contiguously.  Both come from one 8-byte load at `b` = m0 clamped to
// [0, ncross - 2]; `s0` / `s1` say which half holds m0 / m0 + 1, and
// out-of-image pixels are weighted 0 (the load then stays inside the line).
struct CellTap {
    int b;
    bool s0, s1;  // true: the second float of the pair
    float a0, a1;
};

typedef float f32x2a4 __attribute__((ext_vector_type(2), aligned(4)));  // 4-byte aligned pair

__device__ __forceinline__ CellTap cell_tap(long long lo, const RayFx& R, float wfull, int ncross)
{
    const CellW w = cell_weights(lo, R.span, R.w32, wfull);
    const bool in0 = (unsigned)w.m0 < (unsigned)ncross;
    const bool in1 = (unsigned)(w.m0 + 1) < (unsigned)ncross;
    CellTap t;
    t.b = min(max(w.m0, 0), ncross - 2);
    t.s0 = w.m0 != t.b;
    t.s1 = w.m0 + 1 != t.b;
    t.a0 = in0 ? w.c0 : 0.0f;
    t.a1 = in1 ? w.c1 : 0.0f;
    return t;
}

template <int NSEG>
__device__ __forceinline__ void project_block(const RayFx* __restrict__ rays, const int2* __restrict__ range,
                                              const float* __restrict__ x, const float* __restrict__ xT, int nx,
                                              int ny, int B, float alpha, float beta, const float* c, float* q,
                                              double* partial, int bx, int v, int part_id, float (*red)[64],
                                              double* lds)
{
    const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int b = bx * 64 + lane;
    float acc = 0.0f, acc1 = 0.0f;
    if (b < B) {
        const int id = v * B + b;
        const RayFx R = rays[id];
        const int2 K = range[id];
        const bool rows = R.wfull < 0.0f;  // swept row by row: cells are rows of x
        const float wfull = fabsf(R.wfull);
        const float* img = rows ? x : xT;
        const int ncross = rows ? nx : ny;
        const int len = K.y - K.x;
        const int k0 = K.x + (int)(((long long)len * seg) / NSEG);
        const int k1 = K.x + (int)(((long long)len * (seg + 1)) / NSEG);
        long long lo = R.lo0 + (long long)k0 * R.step;
        const float* line = img + (size_t)k0 * ncross;
        int k = k0;
        for (; k + kProjUnroll <= k1; k += kProjUnroll) {
            CellTap t[kProjUnroll];
#pragma unroll
            for (int u = 0; u < kProjUnroll; ++u) {
                t[u] = cell_tap(lo, R, wfull, ncross);
                lo += R.step;
            }
            f32x2a4 pr[kProjUnroll];
#pragma unroll
            for (int u = 0; u < kProjUnroll; ++u)
                pr[u] = *reinterpret_cast<const f32x2a4*>(line + u * ncross + t[u].b);
#pragma unroll
            for (int u = 0; u < kProjUnroll; ++u) {
                acc = fmaf(t[u].a0, t[u].s0 ? pr[u].y : pr[u].x, acc);
                acc1 = fmaf(t[u].a1, t[u].s1 ? pr[u].y : pr[u].x, acc1);
            }
            line += (size_t)kProjUnroll * ncross;
        }
        for (; k < k1; ++k) {
            const CellTap t = cell_tap(lo, R, wfull, ncross);
            const f32x2a4 pv = *reinterpret_cast<const f32x2a4*>(line + t.b);
            acc = fmaf(t.a0, t.s0 ? pv.y : pv.x, acc);
            acc1 = fmaf(t.a1, t.s1 ? pv.y : pv.x, acc1);
            lo += R.step;
            line += ncross;
        }
    }
    red[seg][lane] = acc + acc1;
    __syncthreads();
    if (seg == 0) {
        float out = 0.0f;
        if (b < B) {
            float sum = red[0][lane];
#pragma unroll
            for (int i = 1; i < NSEG; ++i) sum += red[i][lane];
            const int id = v * B + b;
            out = alpha * sum;
            if (beta != 0.0f) out = fmaf(beta, c[id], out);
            q[id] = out;
        }
        if (partial) {
            const double s2 = wave_sum((double)out * (double)out);
            if (lane == 0) lds[0] = s2;
        }
    }
    if (partial) {
        __syncthreads();
        if (threadIdx.x == 0) partial[part_id] = lds[0];
    }
}

template <int NSEG>
__global__ __launch_bounds__(64 * NSEG) void k_project(const RayFx* __restrict__ rays,
                                                       const int2* __restrict__ range,
                                                       const float* __restrict__ x,
                                                       const float* __restrict__ xT, int nx, int ny,
                                                       int B, float alpha, float beta,
                                                       const float* c, float* q, double* partial)
{
    __shared__ float red[NSEG][64];
    __shared__ double lds[1];
    project_block<NSEG>(rays, range, x, xT, nx, ny, B, alpha, beta, c, q, partial, blockIdx.x, blockIdx.y,
                        blockIdx.y * gridDim.x + blockIdx.x, red, lds);
}

int project_blocks(const Plan& p) { return ((p.B + 63) / 64) * p.V; }

hipError_t launch_project(const Plan& p, const float* x, const float* xT, float alpha, float beta,
                          const float* c, float* q, double* partial, hipStream_t s)
{
    dim3 grid((p.B + 63) / 64, p.V);
    hipLaunchKernelGGL(k_project<kProjSeg>, grid, dim3(64 * kProjSeg), 0, s, p.rays.d_ray, p.rays.d_range, x, xT,
                       p.nx, p.ny, p.B, alpha, beta, c, q, partial);
    return hipGetLastError();
}

// ------------------------------------------------------------------ backprojector
constexpr int kTile = kBpTile;

// lo0 + ks * step for 0 <= ks < 2^15 and |step| <= 2^32: the low word of step
// in one 32x32->64 multiply-add, its high word (-1, 0 or 1) in a 24-bit one.
__device__ __forceinline__ long long cell_lo(const RayFx& R, int ks)
{
    const unsigned long long prod =
        (unsigned long long)(unsigned)ks * (unsigned)(unsigned long long)R.step + (unsigned long long)R.lo0;
    const int hi = (int)(prod >> 32) + __mul24(ks, (int)(R.step >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)prod);
}

// P^T r, exact transpose of k_project, computed tile by tile without write
// conflicts (the concern of Sec. 2.3) and without per-pixel arctangents.
// A block owns a 16x16 pixel tile.  The host lists, per tile, every ray that
// can meet it (views ascending, bins ascending); the block stages them in LDS
// in chunks and walks each through the tile's 16 sweep lines: thread
// (line, group) evaluates the ray's one or two cells on its sweep line with
// the projector's own fixed-point arithmetic (cell_weights) and adds c * r to
// the group's private accumulator tile.  The 16 lanes of a group take the
// same ray at the same time, and a ray's sweep lines own distinct pixels, so
// no two lanes ever update one accumulator entry; the per-pixel order (rays
// in list order, then the 16 groups in order) is fixed, so results are
// deterministic.
constexpr int kBpGroups = 16;
constexpr int kBpChunk = 256;

struct BpEntry {
    RayFx ray;
    int2 range;
    float r;
    float pad;
};

struct BpShared {
    BpEntry ent[kBpChunk];
    float acc[kBpGroups][kTile][kTile + 1];
    float tile[kTile][kTile + 1];
    double lds[4];
};

__device__ __forceinline__ void backproject_block(const RayFx* __restrict__ rays, const int2* __restrict__ range,
                                                  const int* __restrict__ list_off, const int* __restrict__ list,
                                                  const float* __restrict__ r, int nx, int ny, float alpha,
                                                  float beta, const float* c, float* z, float* zT, double* partial,
                                                  int bx, int by, int tile_id, BpShared& S)
{
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
    const int line = tx, grp = ty;  // the same split read as (sweep line, group)
    const int i0 = bx * kTile, j0 = by * kTile;
    for (int g = 0; g < kBpGroups; ++g) S.acc[g][ty][tx] = 0.0f;
    const int beg = list_off[tile_id], end = list_off[tile_id + 1];
    for (int base = beg; base < end; base += kBpChunk) {
        const int n = min(kBpChunk, end - base);
        __syncthreads();
        if ((int)threadIdx.x < n) {
            const int id = list[base + threadIdx.x];
            BpEntry e;
            e.ray = rays[id];
            e.range = range[id];
            e.r = r[id];
            e.pad = 0.0f;
            S.ent[threadIdx.x] = e;
        }
        __syncthreads();
        for (int k = grp; k < n; k += kBpGroups) {
            const BpEntry& e = S.ent[k];
            const bool rows = e.ray.wfull < 0.0f;  // swept row by row
            const int ks = (rows ? j0 : i0) + line;
            if (ks < e.range.x || ks >= e.range.y) continue;
            const CellW w = cell_weights(cell_lo(e.ray, ks), e.ray.span, e.ray.w32, fabsf(e.ray.wfull));
            const int m = w.m0 - (rows ? i0 : j0);
            if ((unsigned)m < (unsigned)kTile) {
                float& a = rows ? S.acc[grp][line][m] : S.acc[grp][m][line];
                a = fmaf(w.c0, e.r, a);
            }
            if ((unsigned)(m + 1) < (unsigned)kTile) {
                float& a = rows ? S.acc[grp][line][m + 1] : S.acc[grp][m + 1][line];
                a = fmaf(w.c1, e.r, a);
            }
        }
    }
    __syncthreads();
    const int i = i0 + tx, j = j0 + ty;
    const bool in = i < nx && j < ny;
    float sum = 0.0f;
#pragma unroll
    for (int g = 0; g < kBpGroups; ++g) sum += S.acc[g][ty][tx];
    float out = 0.0f;
    if (in) {
        const size_t id = (size_t)j * nx + i;
        out = alpha * sum;
        if (beta != 0.0f) out = fmaf(beta, c[id], out);
        z[id] = out;
    }
    if (zT) {
        S.tile[ty][tx] = out;
        __syncthreads();
        const int it = i0 + ty, jt = j0 + tx;
        if (it < nx && jt < ny) zT[(size_t)it * ny + jt] = S.tile[tx][ty];
    }
    if (partial) {
        const double s2 = block_sum<256>((double)out * (double)out, S.lds);
        if (threadIdx.x == 0) partial[tile_id] = s2;
    }
}

__global__ __launch_bounds__(256) void k_backproject(const RayFx* __restrict__ rays,
                                                     const int2* __restrict__ range,
                                                     const int* __restrict__ list_off,
                                                     const int* __restrict__ list,
                                                     const float* __restrict__ r, int nx, int ny,
                                                     float alpha, float beta, const float* c, float* z,
                                                     float* zT, double* partial)
{
    __shared__ BpShared S;
    backproject_block(rays, range, list_off, list, r, nx, ny, alpha, beta, c, z, zT, partial, blockIdx.x,
                      blockIdx.y, blockIdx.y * gridDim.x + blockIdx.x, S);
}

int image_tile_blocks(const Plan& p) { return ((p.nx + kTile - 1) / kTile) * ((p.ny + kTile - 1) / kTile); }

hipError_t launch_backproject(const Plan& p, const float* r, float alpha, float beta, const float* c,
                              float* z, float* zT, double* partial, hipStream_t s)
{
    dim3 grid((p.nx + kTile - 1) / kTile, (p.ny + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_backproject, grid, dim3(256), 0, s, p.rays.d_ray, p.rays.d_range, p.rays.d_list_off,
                       p.rays.d_list, r, p.nx, p.ny, alpha, beta, c, z, zT, partial);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Eq. 11 backprojector
// The paper's pixel-driven backprojector (Eq. 11, derived in App. III): per
// view, the pixel centre's angle beta* seen from the source picks a fractional
// bin, the sinogram is interpolated linearly there (bins beyond the detector
// read zero) and weighted by 1/l, l the source-to-pixel distance; the sum over
// views is scaled by d^2 / dbeta.  Only approximately the transpose of the
// projector.
//
// The interpolation weight moves by 1/dbeta per radian of beta*, so beta* must
// be right to far better than a float32 arctangent.  The bin angles are
// equally spaced and the same for every view, so with tau_b = tan(beta_b)
// (double, per bin) and rho = across/along = tan(beta*):
//   beta* - beta_b = atan((across - tau_b along) / (along + tau_b across)),
// a small angle (about one bin), whose arctangent is x - x^3/3 to 1e-15.
// The numerator is formed in double from double coordinates; a float32
// polynomial arctangent (error < 1.3e-7 rad) only guesses the bin, corrected
// by one if the fraction leaves [0, 1).
__device__ __forceinline__ float guess_atan(float t)
{
    // odd polynomial of degree 15 for atan on [0, 1], reflected above 1; the
    // coefficients are the near-minimax fit of Lawson's iteratively
    // reweighted least squares (fit_atan.py beside this file prints them),
    // 3.75e-8 rad at most in exact arithmetic
    const float a = fabsf(t);
    const bool big = a > 1.0f;
    const float u = big ? __builtin_amdgcn_rcpf(a) : a;
    const float u2 = u * u;
    float p = -4.054566622e-03f;
    p = fmaf(p, u2, 2.186295575e-02f);
    p = fmaf(p, u2, -5.591232369e-02f);
    p = fmaf(p, u2, 9.642197100e-02f);
    p = fmaf(p, u2, -1.390862946e-01f);
    p = fmaf(p, u2, 1.994656563e-01f);
    p = fmaf(p, u2, -3.332986078e-01f);
    p = fmaf(p, u2, 9.999993356e-01f);
    p *= u;
    p = big ? 1.5707963268f - p : p;
    return copysignf(p, t);
}

__global__ __launch_bounds__(256) void k_backproject_interp(const double2* __restrict__ view,
                                                            const double* __restrict__ tau,
                                                            const float* __restrict__ r, int nx, int ny, int V,
                                                            int B, double pixel, double sad, float inv_dbeta,
                                                            float bin_c, float scale, float beta, const float* c,
                                                            float* z, float* zT, double* partial)
{
    __shared__ float tile[kTile][kTile + 1];
    __shared__ double lds[4];
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
    const int i = blockIdx.x * kTile + tx, j = blockIdx.y * kTile + ty;
    const bool in = i < nx && j < ny;
    float acc = 0.0f;
    if (in) {
        const double cx = ((double)i + 0.5 - 0.5 * nx) * pixel;
        const double cy = ((double)j + 0.5 - 0.5 * ny) * pixel;
        for (int v = 0; v < V; ++v) {
            const double2 cs = view[v];
            // pixel centre in the frame of the view's central ray
            const double along = fma(cx, cs.x, fma(cy, cs.y, sad));
            const double across = fma(cy, cs.x, -cx * cs.y);
            const float alf = (float)along, acf = (float)across;
            int b0 = (int)floorf(fmaf(guess_atan(acf * __builtin_amdgcn_rcpf(alf)), inv_dbeta, bin_c));
            if (b0 < -1 || b0 > B - 1) continue;  // both bins beyond the detector
            const double tb = tau[b0 + 1];
            const float x = (float)fma(-tb, along, across) / (float)fma(tb, across, along);
            float a = (x - x * x * x * (1.0f / 3.0f)) * inv_dbeta;
            if (a < 0.0f) {
                --b0;
                a += 1.0f;
            } else if (a >= 1.0f) {
                ++b0;
                a -= 1.0f;
            }
            const float* rr = r + (size_t)v * B;
            const float y0 = (b0 >= 0 && b0 < B) ? rr[b0] : 0.0f;
            const float y1 = (b0 + 1 >= 0 && b0 + 1 < B) ? rr[b0 + 1] : 0.0f;
            const float inv_l = __builtin_amdgcn_rsqf(fmaf(alf, alf, acf * acf));
            acc = fmaf(fmaf(a, y1 - y0, y0), inv_l, acc);
        }
    }
    float out = 0.0f;
    if (in) {
        const size_t id = (size_t)j * nx + i;
        out = scale * acc;
        if (beta != 0.0f) out = fmaf(beta, c[id], out);
        z[id] = out;
    }
    if (zT) {
        tile[ty][tx] = out;
        __syncthreads();
        const int it = blockIdx.x * kTile + ty, jt = blockIdx.y * kTile + tx;
        if (it < nx && jt < ny) zT[(size_t)it * ny + jt] = tile[tx][ty];
    }
    if (partial) {
        const double s2 = block_sum<256>((double)out * (double)out, lds);
        if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s2;
    }
}

hipError_t launch_backproject_interp(const Plan& p, const float* r, float alpha, float beta, const float* c,
                                     float* z, float* zT, double* partial, hipStream_t s)
{
    const float scale = (float)((double)alpha * p.pixel * p.pixel / p.dbeta);
    dim3 grid((p.nx + kTile - 1) / kTile, (p.ny + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_backproject_interp, grid, dim3(256), 0, s, p.rays.d_view_d, p.rays.d_tau, r, p.nx, p.ny,
                       p.V, p.B, p.pixel, p.sad, (float)(1.0 / p.dbeta), (float)(0.5 * (p.B - 1) - p.bin_offset),
                       scale, beta, c, z, zT, partial);
    return hipGetLastError();
}

// ------------------------------------------------------------------ layout helpers
__device__ __forceinline__ void transpose_block(const float* __restrict__ src, float* __restrict__ dst, int nx,
                                                int ny, int tbx, int tby, float (*t)[33])
{
    const int bx = tbx * 32, by = tby * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int i = bx + tx, j = by + k;
        t[k][tx] = (i < nx && j < ny) ? src[(size_t)j * nx + i] : 0.0f;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int i = bx + k, j = by + tx;
        if (i < nx && j < ny) dst[(size_t)i * ny + j] = t[tx][k];
    }
}

__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ src, float* __restrict__ dst,
                                                   int nx, int ny)
{
    __shared__ float t[32][33];
    transpose_block(src, dst, nx, ny, blockIdx.x, blockIdx.y, t);
}

hipError_t launch_transpose(const float* src, float* dst, int nx, int ny, hipStream_t s)
{
    dim3 grid((nx + 31) / 32, (ny + 31) / 32);
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, src, dst, nx, ny);
    return hipGetLastError();
}

// The start of a reconstruction in one launch: the image zeroed (when asked)
// or else transposed into fT, each block one 32 x 32 tile, and the device
// state reset by block 0 (as k_state_init), so no separate kernels are needed.
__global__ __launch_bounds__(256) void k_recon_start(float* f, float* __restrict__ fT, int nx, int ny, int zero,
                                                     DevState* st, uint32_t* hist, uint32_t rank, float sigma_fixed)
{
    __shared__ float t[32][33];
    if (zero) {
        const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
        for (int k = ty; k < 32; k += 8) {
            const int i = blockIdx.x * 32 + tx, j = blockIdx.y * 32 + k;
            if (i < nx && j < ny) f[(size_t)j * nx + i] = 0.0f;
            const int it = blockIdx.x * 32 + k, jt = blockIdx.y * 32 + tx;
            if (it < nx && jt < ny) fT[(size_t)it * ny + jt] = 0.0f;
        }
    } else {
        transpose_block(f, fT, nx, ny, blockIdx.x, blockIdx.y, t);
    }
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        if (threadIdx.x == 0) st->rank0 = rank;
        reset_iteration_state(st, hist, sigma_fixed);
        if (threadIdx.x == 0) st->iter = 0;
    }
}

hipError_t launch_recon_start(float* f, float* fT, int nx, int ny, int zero, DevState* st, uint32_t* hist,
                              uint32_t rank, float sigma_fixed, hipStream_t s)
{
    dim3 grid((nx + 31) / 32, (ny + 31) / 32);
    hipLaunchKernelGGL(k_recon_start, grid, dim3(256), 0, s, f, fT, nx, ny, zero, st, hist, rank, sigma_fixed);
    return hipGetLastError();
}

__global__ void k_fill(float* dst, size_t n, float value)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = value;
}

hipError_t launch_fill(float* dst, size_t n, float value, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, dst, n, value);
    return hipGetLastError();
}

// ------------------------------------------------------------------ batched kernels
// Persistent grids over (slice, block) items; see batch.h.  Each item runs the
// one-slice kernel's block function; a barrier separates items because the
// block's LDS is reused.
template <int NSEG>
__global__ __launch_bounds__(64 * NSEG) void kb_project(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                        int n_items, int xs, int xTs, float alpha, float beta, int cs,
                                                        int outs, int parts)
{
    __shared__ float red[NSEG][64];
    __shared__ double lds[1];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        __syncthreads();
        project_block<NSEG>(d.rays, d.range, d.buf[xs], d.buf[xTs], d.nx, d.ny, d.B, alpha, beta, bsel(d, cs),
                            d.buf[outs], psel(d, parts), w.y % d.proj_gx, w.y / d.proj_gx, w.y, red, lds);
    }
}

hipError_t blaunch_project(const BatchDev& b, int x, int xT, float alpha, float beta, int c, int out, int part,
                           hipStream_t s)
{
    const int n = b.n_items[kShProj], g = b.grid[kShProj];
    if (n == 0) return hipSuccess;
    switch (b.proj_seg) {
    case 4:
        hipLaunchKernelGGL(kb_project<4>, dim3(g), dim3(256), 0, s, b.slices, b.items[kShProj], n, x, xT, alpha, beta,
                           c, out, part);
        break;
    case 8:
        hipLaunchKernelGGL(kb_project<8>, dim3(g), dim3(512), 0, s, b.slices, b.items[kShProj], n, x, xT, alpha, beta,
                           c, out, part);
        break;
    default:
        hipLaunchKernelGGL(kb_project<16>, dim3(g), dim3(1024), 0, s, b.slices, b.items[kShProj], n, x, xT, alpha,
                           beta, c, out, part);
        break;
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_backproject(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                      int n_items, int rs, float alpha, float beta, int cs, int zs,
                                                      int zTs, int parts)
{
    __shared__ BpShared S;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        __syncthreads();
        backproject_block(d.rays, d.range, d.list_off, d.list, d.buf[rs], d.nx, d.ny, alpha, beta, bsel(d, cs),
                          d.buf[zs], bsel(d, zTs), psel(d, parts), w.y % d.t16x, w.y / d.t16x, w.y, S);
    }
}

hipError_t blaunch_backproject(const BatchDev& b, int r, float alpha, float beta, int c, int z, int zT, int part,
                               hipStream_t s)
{
    const int n = b.n_items[kShT16];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_backproject, dim3(b.grid[kShT16]), dim3(256), 0, s, b.slices, b.items[kShT16], n, r, alpha,
                       beta, c, z, zT, part);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_transpose(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                    int n_items, int srcs, int dsts)
{
    __shared__ float t[32][33];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        __syncthreads();
        transpose_block(d.buf[srcs], d.buf[dsts], d.nx, d.ny, w.y % d.t32x, w.y / d.t32x, t);
    }
}

hipError_t blaunch_transpose(const BatchDev& b, int src, int dst, hipStream_t s)
{
    const int n = b.n_items[kShT32];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_transpose, dim3(b.grid[kShT32]), dim3(256), 0, s, b.slices, b.items[kShT32], n, src, dst);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_fill_zero(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                    int n_items, int dsts)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        const int bx = (w.y % d.t32x) * 32, by = (w.y / d.t32x) * 32;
        const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
        for (int k = ty; k < 32; k += 8) {
            const int i = bx + tx, j = by + k;
            if (i < d.nx && j < d.ny) d.buf[dsts][(size_t)j * d.nx + i] = 0.0f;
        }
    }
}

hipError_t blaunch_fill_zero(const BatchDev& b, int dst, hipStream_t s)
{
    const int n = b.n_items[kShT32];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_fill_zero, dim3(b.grid[kShT32]), dim3(256), 0, s, b.slices, b.items[kShT32], n, dst);
    return hipGetLastError();
}

}  // namespace eptv
