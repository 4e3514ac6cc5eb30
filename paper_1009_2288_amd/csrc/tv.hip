// tv.hip -- the P2 step: half-edge TV magnitudes and weights, the sigma order
// statistic, the descent direction and the Armijo line search.
//
// Half-edge magnitude of App. II Eq. A3 for the x-edge (i+1/2, j):
//   TV = sqrt((f[i+1,j]-f[i,j])^2 + 1/2 (m[j+1]-m[j])^2 + 1/2 (m[j]-m[j-1])^2 + eps^2),
//   m[k] = (f[i+1,k] + f[i,k]) / 2,
// y-edges with the roles of i and j exchanged, pixels outside the image zero
// (zero boundary condition below Eq. A1).  Weight w = exp(-TV^2/sigma^2)
// (Eq. 5 on the half-edge).  Direction (Eq. 9, variation by Eq. A2):
//   g = lambda (f - v) - [F(i+1/2,j) - F(i-1/2,j)] - [F(i,j+1/2) - F(i,j-1/2)],
//   F = w * (difference across the edge) / TV.
// Every kernel reads a pixel's 3x3 neighbourhood; each half-edge is owned by
// exactly one pixel (its left / lower pixel, or the border pixel for the
// edges on the left and bottom image border) for the energy sums.
#include "eptv_internal.h"
#include "reduce.h"

namespace eptv {

constexpr int kT = 16;  // 16 x 16 pixel tiles, one pixel per thread

__device__ __forceinline__ float pix(const float* f, int nx, int ny, int i, int j)
{
    return (i >= 0 && i < nx && j >= 0 && j < ny) ? f[(size_t)j * nx + i] : 0.0f;
}

// Magnitude of the half-edge between pixel values a and b, whose neighbouring
// pixel pairs on the two sides across the edge direction are (au, bu) and (ad, bd).
__device__ __forceinline__ float tv_edge(float a, float b, float au, float bu, float ad, float bd, float eps2)
{
    const float d = b - a;
    const float m0 = 0.5f * (a + b), mu = 0.5f * (au + bu), md = 0.5f * (ad + bd);
    const float t1 = mu - m0, t2 = m0 - md;
    return sqrtf(d * d + 0.5f * (t1 * t1) + 0.5f * (t2 * t2) + eps2);
}

// N[a][b] = f(i + a - 1, j + b - 1): a indexes x, b indexes y.
struct Nbhd {
    float n[3][3];
};

__device__ __forceinline__ void load_nbhd(const float* f, int nx, int ny, int i, int j, Nbhd& N)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) N.n[a][b] = pix(f, nx, ny, i + a - 1, j + b - 1);
}

__device__ __forceinline__ float tv_right(const Nbhd& N, float e2)
{
    return tv_edge(N.n[1][1], N.n[2][1], N.n[1][2], N.n[2][2], N.n[1][0], N.n[2][0], e2);
}
__device__ __forceinline__ float tv_left(const Nbhd& N, float e2)
{
    return tv_edge(N.n[0][1], N.n[1][1], N.n[0][2], N.n[1][2], N.n[0][0], N.n[1][0], e2);
}
__device__ __forceinline__ float tv_up(const Nbhd& N, float e2)
{
    return tv_edge(N.n[1][1], N.n[1][2], N.n[2][1], N.n[2][2], N.n[0][1], N.n[0][2], e2);
}
__device__ __forceinline__ float tv_down(const Nbhd& N, float e2)
{
    return tv_edge(N.n[1][0], N.n[1][1], N.n[2][0], N.n[2][1], N.n[0][0], N.n[0][1], e2);
}

size_t n_edges(const Plan& p) { return (size_t)p.ny * (p.nx + 1) + (size_t)(p.ny + 1) * p.nx; }

// ------------------------------------------------------------------ sigma: magnitudes + first digit
// Edge index: x-edge (i+1/2, j) -> j*(nx+1) + i+1; y-edge (i, j+1/2) -> ny*(nx+1) + (j+1)*nx + i.
// Magnitudes are non-negative floats, so their bit patterns order like the values.
__global__ __launch_bounds__(256) void k_edges_hist(const float* __restrict__ f, int nx, int ny, float eps2,
                                                    uint32_t* keys, uint32_t* hist0)
{
    __shared__ uint32_t h[kSelectBins];
    for (int b = threadIdx.x; b < kSelectBins; b += 256) h[b] = 0u;
    __syncthreads();
    const int i = blockIdx.x * kT + (threadIdx.x & (kT - 1)), j = blockIdx.y * kT + threadIdx.x / kT;
    if (i < nx && j < ny) {
        Nbhd N;
        load_nbhd(f, nx, ny, i, j, N);
        const size_t xo = (size_t)j * (nx + 1), yo = (size_t)ny * (nx + 1);
        uint32_t k = __float_as_uint(tv_right(N, eps2));
        keys[xo + i + 1] = k;
        atomicAdd(&h[k >> 21], 1u);
        k = __float_as_uint(tv_up(N, eps2));
        keys[yo + (size_t)(j + 1) * nx + i] = k;
        atomicAdd(&h[k >> 21], 1u);
        if (i == 0) {
            k = __float_as_uint(tv_left(N, eps2));
            keys[xo] = k;
            atomicAdd(&h[k >> 21], 1u);
        }
        if (j == 0) {
            k = __float_as_uint(tv_down(N, eps2));
            keys[yo + i] = k;
            atomicAdd(&h[k >> 21], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kSelectBins; b += 256)
        if (h[b]) atomicAdd(&hist0[b], h[b]);
}

hipError_t launch_edges_hist(const Plan& p, const float* f, float eps2, uint32_t* keys, uint32_t* hist0,
                             hipStream_t s)
{
    dim3 grid((p.nx + kT - 1) / kT, (p.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_edges_hist, grid, dim3(256), 0, s, f, p.nx, p.ny, eps2, keys, hist0);
    return hipGetLastError();
}

// ------------------------------------------------------------------ sigma: later digits
// pass 1: digit = bits 20..10 among keys whose bits 31..21 equal the prefix;
// pass 2: digit = bits 9..0 among keys whose bits 31..10 equal the prefix.
__global__ __launch_bounds__(256) void k_select_hist(const uint32_t* __restrict__ keys, size_t n, int pass,
                                                     const DevState* st, uint32_t* hist)
{
    __shared__ uint32_t h[kSelectBins];
    for (int b = threadIdx.x; b < kSelectBins; b += 256) h[b] = 0u;
    __syncthreads();
    const int hshift = pass == 1 ? 21 : 10;
    const int dshift = pass == 1 ? 10 : 0;
    const uint32_t dmask = pass == 1 ? 2047u : 1023u;
    const uint32_t want = st->prefix >> hshift;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        const uint32_t k = keys[e];
        if ((k >> hshift) == want) atomicAdd(&h[(k >> dshift) & dmask], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kSelectBins; b += 256)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

int select_blocks(const Plan& p)
{
    const size_t n = n_edges(p);
    return (int)std::max<size_t>(1, std::min<size_t>((n + 2047) / 2048, 512));
}

hipError_t launch_select_hist(const Plan& p, int pass, const uint32_t* keys, const DevState* st,
                              uint32_t* hist, hipStream_t s)
{
    hipLaunchKernelGGL(k_select_hist, dim3(select_blocks(p)), dim3(256), 0, s, keys, n_edges(p), pass, st,
                       hist);
    return hipGetLastError();
}

// Find the digit whose bucket holds the wanted rank, fold it into the prefix,
// and clear the histogram for the next use.  After the last digit the prefix
// is the bit pattern of the selected magnitude.
__global__ __launch_bounds__(256) void k_select_finalize(DevState* st, int pass, uint32_t* hist, float floor_)
{
    __shared__ uint32_t sums[256];
    __shared__ uint32_t found_digit, found_before;
    const int nb = pass == 2 ? 1024 : 2048;
    const int per = nb / 256;
    const int t = threadIdx.x;
    uint32_t local = 0;
    for (int e = 0; e < per; ++e) local += hist[t * per + e];
    sums[t] = local;
    __syncthreads();
    if (t == 0) {
        const uint32_t rank = st->rank;
        uint32_t before = 0;
        int blk = 0;
        while (blk < 255 && before + sums[blk] <= rank) before += sums[blk++];
        int d = blk * per;
        while (d < blk * per + per - 1 && before + hist[d] <= rank) before += hist[d++];
        found_digit = (uint32_t)d;
        found_before = before;
    }
    __syncthreads();
    for (int e = 0; e < per; ++e) hist[t * per + e] = 0u;
    if (t == 0) {
        const int shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
        st->prefix |= found_digit << shift;
        st->rank -= found_before;
        if (pass == 2) {
            float sg = __uint_as_float(st->prefix);
            sg = fmaxf(sg, floor_);
            st->sigma = sg;
            st->inv_sigma2 = 1.0f / (sg * sg);
        }
    }
}

hipError_t launch_select_finalize(DevState* st, int pass, uint32_t* hist, float sigma_floor, hipStream_t s)
{
    hipLaunchKernelGGL(k_select_finalize, dim3(1), dim3(256), 0, s, st, pass, hist, sigma_floor);
    return hipGetLastError();
}

__global__ void k_sigma_out(const DevState* st, float* out)
{
    if (threadIdx.x == 0) out[0] = st->sigma;
}

hipError_t launch_sigma_out(const DevState* st, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sigma_out, dim3(1), dim3(64), 0, s, st, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ direction g (Eq. 9, A2)
__device__ __forceinline__ float weight(float tv, float inv_s2) { return expf(-(tv * tv) * inv_s2); }

__global__ __launch_bounds__(256) void k_tv_grad(const float* __restrict__ f, const float* __restrict__ v, int nx,
                                                 int ny, float lambda, const DevState* st, float inv_s2_direct,
                                                 float eps2, float* __restrict__ g, float* wx, float* wy,
                                                 double* part)
{
    __shared__ double lds[4];
    const float inv_s2 = st ? st->inv_sigma2 : inv_s2_direct;
    const int i = blockIdx.x * kT + (threadIdx.x & (kT - 1)), j = blockIdx.y * kT + threadIdx.x / kT;
    double q = 0.0, gg = 0.0;
    if (i < nx && j < ny) {
        Nbhd N;
        load_nbhd(f, nx, ny, i, j, N);
        const float c = N.n[1][1];
        const float tR = tv_right(N, eps2), tL = tv_left(N, eps2), tU = tv_up(N, eps2), tD = tv_down(N, eps2);
        const float wR = weight(tR, inv_s2), wL = weight(tL, inv_s2), wU = weight(tU, inv_s2),
                    wD = weight(tD, inv_s2);
        const float FR = wR * (N.n[2][1] - c) / tR;
        const float FL = wL * (c - N.n[0][1]) / tL;
        const float FU = wU * (N.n[1][2] - c) / tU;
        const float FD = wD * (c - N.n[1][0]) / tD;
        const size_t id = (size_t)j * nx + i;
        const float dv = c - v[id];
        const float gv = lambda * dv - (FR - FL) - (FU - FD);
        g[id] = gv;
        const size_t xo = (size_t)j * (nx + 1);
        if (wx) {
            wx[xo + i + 1] = wR;
            if (i == 0) wx[xo] = wL;
        }
        if (wy) {
            wy[(size_t)(j + 1) * nx + i] = wU;
            if (j == 0) wy[i] = wD;
        }
        float e = wR * tR + wU * tU;
        if (i == 0) e += wL * tL;
        if (j == 0) e += wD * tD;
        q = (double)e + 0.5 * (double)lambda * (double)dv * (double)dv;
        gg = (double)gv * (double)gv;
    }
    if (part) {
        const double qs = block_sum<256>(q, lds);
        const double gs = block_sum<256>(gg, lds);
        if (threadIdx.x == 0) {
            const int b = blockIdx.y * gridDim.x + blockIdx.x;
            part[2 * b] = qs;
            part[2 * b + 1] = gs;
        }
    }
}

hipError_t launch_tv_grad(const Plan& p, const float* f, const float* v, float lambda, const DevState* st,
                          float sigma_direct, float eps2, float* g, float* wx, float* wy, double* part,
                          hipStream_t s)
{
    const float inv_s2 = (sigma_direct > 0.0f && std::isfinite(sigma_direct)) ? 1.0f / (sigma_direct * sigma_direct)
                                                                             : 0.0f;
    dim3 grid((p.nx + kT - 1) / kT, (p.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_tv_grad, grid, dim3(256), 0, s, f, v, p.nx, p.ny, lambda, st, inv_s2, eps2, g, wx, wy,
                       part);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_grad_finalize(DevState* st, const double* part, int n)
{
    __shared__ double lds[4];
    const double q = block_sum_array(part, n, 2, lds);
    const double gg = block_sum_array(part + 1, n, 2, lds);
    if (threadIdx.x == 0) {
        st->q0 = q;
        st->gg = gg;
        st->decided = 0;
        st->k = -1;
        st->t = 0.0f;
    }
}

hipError_t launch_grad_finalize(DevState* st, const double* part, int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_finalize, dim3(1), dim3(256), 0, s, st, part, nparts);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Armijo line search
// Candidate k uses t_k = t0 * shrink^k, formed by repeated float multiplication
// in every kernel that needs it, so the evaluated and the applied steps agree.
__device__ __forceinline__ float cand_t(float t0, float shrink, int k)
{
    float t = t0;
    for (int i = 0; i < k; ++i) t *= shrink;
    return t;
}

// Q(f - t_k g) for kArmijoCand candidates k = pass*kArmijoCand + c, with the
// weights frozen at f: partial sums per block, [block][candidate].
__global__ __launch_bounds__(256) void k_armijo(const float* __restrict__ f, const float* __restrict__ g,
                                                const float* __restrict__ v, const float* __restrict__ wx,
                                                const float* __restrict__ wy, int nx, int ny, float lambda,
                                                float eps2, float t0, float shrink, int pass, const DevState* st,
                                                double* part)
{
    __shared__ double lds[4];
    if (st->decided) return;  // uniform: an earlier pass already chose a step
    const int i = blockIdx.x * kT + (threadIdx.x & (kT - 1)), j = blockIdx.y * kT + threadIdx.x / kT;
    const bool in = i < nx && j < ny;
    Nbhd F, G;
    float wR = 0.f, wU = 0.f, wL = 0.f, wD = 0.f, vv = 0.f;
    if (in) {
        load_nbhd(f, nx, ny, i, j, F);
        load_nbhd(g, nx, ny, i, j, G);
        const size_t xo = (size_t)j * (nx + 1);
        wR = wx[xo + i + 1];
        wU = wy[(size_t)(j + 1) * nx + i];
        if (i == 0) wL = wx[xo];
        if (j == 0) wD = wy[i];
        vv = v[(size_t)j * nx + i];
    }
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    float t = cand_t(t0, shrink, pass * kArmijoCand);
    for (int c = 0; c < kArmijoCand; ++c) {
        double e = 0.0;
        if (in) {
            Nbhd H;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) H.n[a][bb] = fmaf(-t, G.n[a][bb], F.n[a][bb]);
            float s = wR * tv_right(H, eps2) + wU * tv_up(H, eps2);
            if (i == 0) s += wL * tv_left(H, eps2);
            if (j == 0) s += wD * tv_down(H, eps2);
            const float d = H.n[1][1] - vv;
            e = (double)s + 0.5 * (double)lambda * (double)d * (double)d;
        }
        const double tot = block_sum<256>(e, lds);
        if (threadIdx.x == 0) part[(size_t)b * kArmijoCand + c] = tot;
        t *= shrink;
    }
}

int armijo_blocks(const Plan& p) { return ((p.nx + kT - 1) / kT) * ((p.ny + kT - 1) / kT); }

hipError_t launch_armijo(const Plan& p, int pass, const float* f, const float* g, const float* v,
                         const float* wx, const float* wy, float lambda, float eps2, float t0, float shrink,
                         const DevState* st, double* part, hipStream_t s)
{
    dim3 grid((p.nx + kT - 1) / kT, (p.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_armijo, grid, dim3(256), 0, s, f, g, v, wx, wy, p.nx, p.ny, lambda, eps2, t0, shrink,
                       pass, st, part);
    return hipGetLastError();
}

// First candidate with Q_k <= Q0 - c t_k ||g||^2; after the last allowed
// candidate without one, the step is skipped (k = -1, t = 0).
__global__ __launch_bounds__(256) void k_armijo_finalize(DevState* st, const double* part, int n, int pass,
                                                         int max_bt, double c, float t0, float shrink)
{
    __shared__ double lds[4];
    if (st->decided) return;
    const double q0 = st->q0, gg = st->gg;
    for (int cc = 0; cc < kArmijoCand; ++cc) {
        const int k = pass * kArmijoCand + cc;
        if (k > max_bt) break;
        const double qk = block_sum_array(part + cc, n, kArmijoCand, lds);
        const float t = cand_t(t0, shrink, k);
        if (qk <= q0 - c * (double)t * gg) {
            if (threadIdx.x == 0) {
                st->decided = 1;
                st->k = k;
                st->t = t;
            }
            return;
        }
    }
    if ((pass + 1) * kArmijoCand > max_bt && threadIdx.x == 0) {
        st->decided = 1;
        st->k = -1;
        st->t = 0.0f;
    }
}

hipError_t launch_armijo_finalize(DevState* st, const double* part, int nparts, int pass, int max_bt, double c,
                                  double t0, double shrink, hipStream_t s)
{
    hipLaunchKernelGGL(k_armijo_finalize, dim3(1), dim3(256), 0, s, st, part, nparts, pass, max_bt, c, (float)t0,
                       (float)shrink);
    return hipGetLastError();
}

// f_out = f - t g (unchanged when no step was accepted), optional truncation at
// zero (step 3 of the algorithm) and optional transposed copy for the projector.
__global__ __launch_bounds__(256) void k_p2_update(const DevState* st, const float* fcur, const float* __restrict__ g,
                                                   float* fout, float* foutT, int clamp, int nx, int ny,
                                                   int32_t* st_k, int step, int T)
{
    __shared__ float tl[32][33];
    const int k = st->k;
    const float t = st->t;
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = bx + tx, j = by + r;
        float val = 0.0f;
        if (i < nx && j < ny) {
            const size_t id = (size_t)j * nx + i;
            val = fcur[id];
            if (k >= 0) val = fmaf(-t, g[id], val);
            if (clamp) val = fmaxf(val, 0.0f);
            fout[id] = val;
        }
        tl[r][tx] = val;
    }
    if (st_k && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) st_k[(size_t)st->iter * T + step] = k;
    if (foutT) {
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = bx + r, j = by + tx;
            if (i < nx && j < ny) foutT[(size_t)i * ny + j] = tl[tx][r];
        }
    }
}

hipError_t launch_p2_update(const Plan& p, const DevState* st, const float* fcur, const float* g, float* fout,
                            float* foutT, int clamp, int32_t* st_k, int step, int T, hipStream_t s)
{
    dim3 grid((p.nx + 31) / 32, (p.ny + 31) / 32);
    hipLaunchKernelGGL(k_p2_update, grid, dim3(256), 0, s, st, fcur, g, fout, foutT, clamp, p.nx, p.ny, st_k, step,
                       T);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy_clamp(const float* src, float* dst, float* dstT, int clamp, int nx,
                                                    int ny)
{
    __shared__ float tl[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = bx + tx, j = by + r;
        float val = 0.0f;
        if (i < nx && j < ny) {
            const size_t id = (size_t)j * nx + i;
            val = src[id];
            if (clamp) val = fmaxf(val, 0.0f);
            dst[id] = val;
        }
        tl[r][tx] = val;
    }
    if (dstT) {
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = bx + r, j = by + tx;
            if (i < nx && j < ny) dstT[(size_t)i * ny + j] = tl[tx][r];
        }
    }
}

hipError_t launch_copy_clamp(const Plan& p, const float* src, float* dst, float* dstT, int clamp, hipStream_t s)
{
    dim3 grid((p.nx + 31) / 32, (p.ny + 31) / 32);
    hipLaunchKernelGGL(k_copy_clamp, grid, dim3(256), 0, s, src, dst, dstT, clamp, p.nx, p.ny);
    return hipGetLastError();
}

}  // namespace eptv
