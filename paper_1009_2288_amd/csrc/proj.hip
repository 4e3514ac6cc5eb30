// proj.hip -- forward projection P and its exact transpose P^T on gfx950.
//
// P (Sec. 2.1, Eq. 1): entry p_ij is the length of ray i inside pixel j.
// The projector is ray-driven, one lane per ray (Sec. 2.3): a wave holds 64
// consecutive detector bins of one view, so the output row q[v][b..b+63] is
// written with one coalesced store.  Each ray is swept along its dominant axis
// (see RayTable); the sweep is split into NSEG segments handled by the waves of
// a block and summed in LDS in a fixed order.  Rays swept column by column read
// the transposed image, so the 64 lanes of a wave, which sit in neighbouring
// rows of one column, touch contiguous memory in both sweep directions.
//
// P^T is pixel-driven (Sec. 2.3: one thread per pixel avoids the write
// conflicts of a ray-driven scatter).  For every view a pixel finds the bins
// whose rays can meet it from its angular position seen from the source, and
// evaluates the same chord expression as the projector, so the float32 P^T is
// exactly the transpose of the float32 P (not the interpolating approximation
// of Eq. 11).  Views are summed in ascending order; there are no atomics.
#include "eptv_internal.h"
#include "reduce.h"

namespace eptv {

// ------------------------------------------------------------------ projector
template <int NSEG>
__global__ __launch_bounds__(64 * NSEG) void k_project(const longlong2* __restrict__ fx,
                                                       const float2* __restrict__ wt,
                                                       const int2* __restrict__ range,
                                                       const float* __restrict__ x,
                                                       const float* __restrict__ xT, int nx, int ny,
                                                       int B, float alpha, float beta,
                                                       const float* c, float* q, double* partial)
{
    __shared__ float red[NSEG][64];
    __shared__ double lds[1];
    const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int b = blockIdx.x * 64 + lane, v = blockIdx.y;
    float acc = 0.0f;
    if (b < B) {
        const int id = v * B + b;
        const longlong2 FX = fx[id];
        const float2 W = wt[id];
        const int2 K = range[id];
        const bool rows = W.y < 0.0f;  // swept row by row: cells are columns of x
        const float wfull = fabsf(W.y), w32 = W.x;
        const long long S = FX.y;
        const float* img = rows ? x : xT;
        const int ncross = rows ? nx : ny;
        const int len = K.y - K.x;
        const int k0 = K.x + (int)(((long long)len * seg) / NSEG);
        const int k1 = K.x + (int)(((long long)len * (seg + 1)) / NSEG);
        long long E = FX.x + (long long)k0 * S;
        for (int k = k0; k < k1; ++k) {
            const long long En = E + S;
            const long long lo = S >= 0 ? E : En, hi = S >= 0 ? En : E;
            const int m0 = (int)(lo >> 32), m1 = (int)(hi >> 32);
            const float* line = img + (size_t)k * ncross;
            if (S == 0) {
                if (m0 >= 0 && m0 < ncross) acc = fmaf(wfull, line[m0], acc);
            } else {
                const unsigned flo = (unsigned)lo, fhi = (unsigned)hi;
                if (m0 == m1) {
                    if (m0 >= 0 && m0 < ncross) acc = fmaf((float)(fhi - flo) * w32, line[m0], acc);
                } else {
                    if (m0 >= 0 && m0 < ncross) acc = fmaf((4294967296.0f - (float)flo) * w32, line[m0], acc);
                    if (fhi != 0u && m1 >= 0 && m1 < ncross) acc = fmaf((float)fhi * w32, line[m1], acc);
                }
            }
            E = En;
        }
    }
    red[seg][lane] = acc;
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
        if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = lds[0];
    }
}

constexpr int kProjSeg = 8;

int project_blocks(const Plan& p) { return ((p.B + 63) / 64) * p.V; }

hipError_t launch_project(const Plan& p, const float* x, const float* xT, float alpha, float beta,
                          const float* c, float* q, double* partial, hipStream_t s)
{
    dim3 grid((p.B + 63) / 64, p.V);
    hipLaunchKernelGGL(k_project<kProjSeg>, grid, dim3(64 * kProjSeg), 0, s, p.rays.d_fx, p.rays.d_w,
                       p.rays.d_range, x, xT, p.nx, p.ny, p.B, alpha, beta, c, q, partial);
    return hipGetLastError();
}

// ------------------------------------------------------------------ backprojector
struct BpConst {
    float pixel;      // d
    float sad;
    float inv_dbeta;
    float bin_c;      // (B-1)/2 - bin_offset: bin coordinate of beta = 0
    float rad;        // d / sqrt(2): radius of the circle around a pixel
    float margin;     // extra bins on each side (rounding of the bin search)
};

constexpr int kTile = 16;

__global__ __launch_bounds__(256) void k_backproject(const longlong2* __restrict__ fx,
                                                     const float2* __restrict__ wt,
                                                     const float2* __restrict__ view,
                                                     const float* __restrict__ r, int nx, int ny,
                                                     int V, int B, BpConst k, float alpha,
                                                     float beta, const float* c, float* z,
                                                     float* zT, double* partial)
{
    __shared__ float tile[kTile][kTile + 1];
    __shared__ double lds[4];
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
    const int i = blockIdx.x * kTile + tx, j = blockIdx.y * kTile + ty;
    const bool in = i < nx && j < ny;
    float acc = 0.0f;
    if (in) {
        const float cx = ((float)i + 0.5f - 0.5f * (float)nx) * k.pixel;
        const float cy = ((float)j + 0.5f - 0.5f * (float)ny) * k.pixel;
        const float rad2 = k.rad * k.rad;
        for (int v = 0; v < V; ++v) {
            const float2 cs = view[v];
            // position of the pixel centre in the frame of the view's central ray
            const float along = fmaf(cx, cs.x, fmaf(cy, cs.y, k.sad));
            const float across = fmaf(cy, cs.x, -cx * cs.y);
            const float bc = fmaf(atan2f(across, along), k.inv_dbeta, k.bin_c);
            // the pixel lies inside a circle of radius d/sqrt(2): its rays are
            // within asin(rad/l) <= rad / sqrt(l^2 - rad^2) of the centre's.
            const float hw = fmaf(k.rad * rsqrtf(along * along + across * across - rad2),
                                  k.inv_dbeta, k.margin);
            const int b0 = max((int)ceilf(bc - hw), 0);
            const int b1 = min((int)floorf(bc + hw), B - 1);
            const longlong2* fv = fx + (size_t)v * B;
            const float2* wv = wt + (size_t)v * B;
            const float* rr = r + (size_t)v * B;
            for (int b = b0; b <= b1; ++b) {
                const longlong2 FX = fv[b];
                const float2 W = wv[b];
                const bool rows = W.y < 0.0f;
                const int ks = rows ? j : i, m = rows ? i : j;
                const long long ea = FX.x + (long long)ks * FX.y;
                acc = fmaf(chord_fx(ea, ea + FX.y, FX.y, m, W.x, fabsf(W.y)), rr[b], acc);
            }
        }
    }
    float out = 0.0f;
    if (in) {
        const size_t id = (size_t)j * nx + i;
        out = alpha * acc;
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

int image_tile_blocks(const Plan& p) { return ((p.nx + kTile - 1) / kTile) * ((p.ny + kTile - 1) / kTile); }

hipError_t launch_backproject(const Plan& p, const float* r, float alpha, float beta, const float* c,
                              float* z, float* zT, double* partial, hipStream_t s)
{
    const double half_diag = 0.5 * p.pixel * std::sqrt((double)p.nx * p.nx + (double)p.ny * p.ny);
    const double dot_min = p.sad - half_diag;
    // rounding of the stored ray coordinates (far below 2^-22 (nx+ny) row units)
    // seen from the nearest pixel, plus a fixed 0.01 bin for the bin search itself.
    const double err = std::ldexp(1.0, -22) * (p.nx + p.ny) * p.pixel / (dot_min * p.dbeta);
    BpConst k;
    k.pixel = (float)p.pixel;
    k.sad = (float)p.sad;
    k.inv_dbeta = (float)(1.0 / p.dbeta);
    k.bin_c = (float)(0.5 * (p.B - 1) - p.bin_offset);
    k.rad = (float)(p.pixel * std::sqrt(0.5) * (1.0 + 1e-6));
    k.margin = (float)(0.01 + 4.0 * err);
    dim3 grid((p.nx + kTile - 1) / kTile, (p.ny + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_backproject, grid, dim3(256), 0, s, p.rays.d_fx, p.rays.d_w, p.rays.d_view, r, p.nx,
                       p.ny, p.V, p.B, k, alpha, beta, c, z, zT, partial);
    return hipGetLastError();
}

// ------------------------------------------------------------------ layout helpers
__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ src, float* __restrict__ dst,
                                                   int nx, int ny)
{
    __shared__ float t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
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

hipError_t launch_transpose(const float* src, float* dst, int nx, int ny, hipStream_t s)
{
    dim3 grid((nx + 31) / 32, (ny + 31) / 32);
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, src, dst, nx, ny);
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

}  // namespace eptv
