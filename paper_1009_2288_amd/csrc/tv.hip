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
#include "batch.h"
#include "eptv_internal.h"
#include "tables.h"
#include "reduce.h"

namespace eptv {

constexpr int kT = 16;  // 16 x 16 pixel tiles, one pixel per thread

__device__ __forceinline__ float pix(const float* f, int nx, int ny, int i, int j)
{
    return (i >= 0 && i < nx && j >= 0 && j < ny) ? f[(size_t)j * nx + i] : 0.0f;
}

// Square root of a positive normal float (here >= eps^2) with the hardware
// instruction (within 1 ulp), not the correctly rounded expansion (a dozen
// instructions): the P2 kernels take 36 of them per pixel.  The same for the
// reciprocal of a magnitude and for the weights' exponential below.
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// Reciprocal of a positive normal float with the hardware instruction (within 1 ulp).
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Magnitude of the half-edge between pixel values a and b, whose neighbouring
// pixel pairs on the two sides across the edge direction are (au, bu) and (ad, bd).
__device__ __forceinline__ float tv_edge(float a, float b, float au, float bu, float ad, float bd, float eps2)
{
    const float d = b - a;
    const float m0 = 0.5f * (a + b), mu = 0.5f * (au + bu), md = 0.5f * (ad + bd);
    const float t1 = mu - m0, t2 = m0 - md;
    return hw_sqrt(d * d + 0.5f * (t1 * t1) + 0.5f * (t2 * t2) + eps2);
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


// ------------------------------------------------------------------ sigma (radix select)
// sigma is the order statistic of rank `rank` of all half-edge magnitudes.
// Magnitudes are non-negative floats, so their bit patterns order like the
// values; the selection takes three digits (bits 31..21, 20..10, 9..0), each
// by a histogram of the keys that match the digits found so far, closed by a
// one-block kernel that finds the digit whose bucket holds the rank.

// LDS histogram increment.  Flat image regions give many identical
// magnitudes (sqrt(eps^2)), so the lanes of a wave that share the first
// active lane's bin add their count with one atomic; the others add one each.
__device__ __forceinline__ void hist_add(uint32_t* h, uint32_t bin)
{
    const uint32_t lead = __builtin_amdgcn_readfirstlane(bin);
    const unsigned long long same = __ballot(bin == lead);
    if (bin == lead) {
        if ((int)(threadIdx.x & 63) == __ffsll((long long)same) - 1) atomicAdd(&h[lead], (uint32_t)__popcll(same));
    } else {
        atomicAdd(&h[bin], 1u);
    }
}

// Edge index: x-edge (i+1/2, j) -> j*(nx+1) + i+1; y-edge (i, j+1/2) -> ny*(nx+1) + (j+1)*nx + i.
// One 16x16 tile's half-edge magnitudes into keys and the block's LDS
// histogram of their top 11 bits.
__device__ __forceinline__ void edges_tile(const float* __restrict__ f, int nx, int ny, float eps2, uint32_t* keys,
                                           int bx, int by, uint32_t* h)
{
    const int i = bx * kT + (threadIdx.x & (kT - 1)), j = by * kT + threadIdx.x / kT;
    if (i < nx && j < ny) {
        Nbhd N;
        load_nbhd(f, nx, ny, i, j, N);
        const size_t xo = (size_t)j * (nx + 1), yo = (size_t)ny * (nx + 1);
        uint32_t k = __float_as_uint(tv_right(N, eps2));
        keys[xo + i + 1] = k;
        hist_add(h, k >> 21);
        k = __float_as_uint(tv_up(N, eps2));
        keys[yo + (size_t)(j + 1) * nx + i] = k;
        hist_add(h, k >> 21);
        if (i == 0) {
            k = __float_as_uint(tv_left(N, eps2));
            keys[xo] = k;
            hist_add(h, k >> 21);
        }
        if (j == 0) {
            k = __float_as_uint(tv_down(N, eps2));
            keys[yo + i] = k;
            hist_add(h, k >> 21);
        }
    }
}

__device__ __forceinline__ void hist_clear(uint32_t* h)
{
    for (int b = threadIdx.x; b < kSelectBins; b += 256) h[b] = 0u;
    __syncthreads();
}

__device__ __forceinline__ void hist_flush(const uint32_t* h, uint32_t* hist0)
{
    __syncthreads();
    for (int b = threadIdx.x; b < kSelectBins; b += 256)
        if (h[b]) atomicAdd(&hist0[b], h[b]);
}

// Persistent over tiles: the flat half-edge magnitudes pile into a few
// histogram bins, so the global atomics per bin (one per block) are what
// serialise; a block walks several tiles and flushes once.
__global__ __launch_bounds__(256) void k_edges_hist(const float* __restrict__ f, int nx, int ny, float eps2,
                                                    uint32_t* keys, uint32_t* hist0)
{
    __shared__ uint32_t h[kSelectBins];
    const int tx = (nx + kT - 1) / kT, nt = tx * ((ny + kT - 1) / kT);
    hist_clear(h);
    for (int t = blockIdx.x; t < nt; t += gridDim.x) edges_tile(f, nx, ny, eps2, keys, t % tx, t / tx, h);
    hist_flush(h, hist0);
}

constexpr int kEdgesHistBlocks = 256;

hipError_t launch_edges_hist(const Plan& p, const float* f, float eps2, uint32_t* keys, uint32_t* hist0,
                             hipStream_t s)
{
    const int nt = ((p.nx + kT - 1) / kT) * ((p.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_edges_hist, dim3((unsigned)std::min(nt, kEdgesHistBlocks)), dim3(256), 0, s, f, p.nx, p.ny,
                       eps2, keys, hist0);
    return hipGetLastError();
}

// pass 1: digit = bits 20..10 among keys whose bits 31..21 equal the prefix;
// pass 2: digit = bits 9..0 among keys whose bits 31..10 equal the prefix.
__device__ __forceinline__ void select_hist_block(const uint32_t* __restrict__ keys, size_t n, int pass,
                                                  uint32_t prefix, uint32_t* hist, int blk, int nblk, uint32_t* h)
{
    for (int b = threadIdx.x; b < kSelectBins; b += 256) h[b] = 0u;
    __syncthreads();
    const int hshift = pass == 1 ? 21 : 10;
    const int dshift = pass == 1 ? 10 : 0;
    const uint32_t dmask = pass == 1 ? 2047u : 1023u;
    const uint32_t want = prefix >> hshift;
    for (size_t e = (size_t)blk * 256 + threadIdx.x; e < n; e += (size_t)nblk * 256) {
        const uint32_t k = keys[e];
        if ((k >> hshift) == want) hist_add(h, (k >> dshift) & dmask);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kSelectBins; b += 256)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// The digit of pass `pass` whose bucket holds `rank` (an inclusive scan over
// 256 groups of buckets) and the count of keys in the buckets below it, in
// S.found_digit / S.found_before for every thread.  After the last digit the
// prefix is the bit pattern of the selected magnitude.
struct SelShared {
    uint32_t sums[256];
    uint32_t found_digit, found_before;
};

__device__ __forceinline__ int digit_shift(int pass) { return pass == 0 ? 21 : (pass == 1 ? 10 : 0); }

__device__ __forceinline__ void select_digit(const uint32_t* hist, int pass, uint32_t rank, SelShared& S)
{
    uint32_t* sums = S.sums;
    const int nb = pass == 2 ? 1024 : 2048;
    const int per = nb / 256;
    const int t = threadIdx.x;
    uint32_t local = 0;
    for (int e = 0; e < per; ++e) local += hist[t * per + e];
    sums[t] = local;
    if (t == 0) {  // only kept if the rank exceeded the count, which cannot happen
        S.found_digit = (uint32_t)(nb - 1);
        S.found_before = 0u;
    }
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t add = t >= o ? sums[t - o] : 0u;
        __syncthreads();
        sums[t] += add;
        __syncthreads();
    }
    const uint32_t before_group = t ? sums[t - 1] : 0u;
    if (before_group <= rank && rank < sums[t]) {
        uint32_t before = before_group;
        int d = t * per;
        while (d < t * per + per - 1 && before + hist[d] <= rank) before += hist[d++];
        S.found_digit = (uint32_t)d;
        S.found_before = before;
    }
    __syncthreads();
}

// One digit closed: folded into the prefix, the rank reduced, the histogram
// cleared for its next use; after pass 2, sigma.
__device__ __forceinline__ void select_finalize_block(DevState* st, int pass, uint32_t* hist, float floor_,
                                                      SelShared& S)
{
    const uint32_t rank = st->rank;
    select_digit(hist, pass, rank, S);
    const int per = (pass == 2 ? 1024 : 2048) / 256;
    for (int e = 0; e < per; ++e) hist[threadIdx.x * per + e] = 0u;
    if (threadIdx.x == 0) {
        st->prefix |= S.found_digit << digit_shift(pass);
        st->rank = rank - S.found_before;
        if (pass == 2) {
            const float sg = fmaxf(__uint_as_float(st->prefix), floor_);
            st->sigma = sg;
            st->inv_sigma2 = 1.0f / (sg * sg);
        }
    }
}

// One-slice passes 1 and 2: every block first closes the previous pass's
// digit itself from that pass's histogram (the same computation in every
// block), so the digit needs no kernel of its own; block 0 records the
// prefix and rank after it for the next pass (in entries no block of this
// launch reads).  hist: the three passes' histograms.
__global__ __launch_bounds__(256) void k_select_pass(const uint32_t* __restrict__ keys, size_t n, int pass,
                                                     DevState* st, uint32_t* hist)
{
    __shared__ uint32_t h[kSelectBins];
    __shared__ SelShared S;
    const uint32_t pin = pass == 1 ? st->prefix : st->sel_prefix[0];
    const uint32_t rin = pass == 1 ? st->rank : st->sel_rank[0];
    select_digit(hist + (pass - 1) * kSelectBins, pass - 1, rin, S);
    const uint32_t pout = pin | (S.found_digit << digit_shift(pass - 1));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->sel_prefix[pass - 1] = pout;
        st->sel_rank[pass - 1] = rin - S.found_before;
    }
    select_hist_block(keys, n, pass, pout, hist + pass * kSelectBins, blockIdx.x, gridDim.x, h);
}

int select_blocks(const Plan& p)
{
    const size_t n = n_edges(p);
    return (int)std::max<size_t>(1, std::min<size_t>((n + 2047) / 2048, 512));
}

hipError_t launch_select_pass(const Plan& p, int pass, const uint32_t* keys, DevState* st, uint32_t* hist,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_select_pass, dim3(select_blocks(p)), dim3(256), 0, s, keys, n_edges(p), pass, st, hist);
    return hipGetLastError();
}

// The last digit and sigma = max(selected magnitude, floor), one block.
__global__ __launch_bounds__(256) void k_select_sigma(DevState* st, const uint32_t* hist, float floor_)
{
    __shared__ SelShared S;
    const uint32_t rin = st->sel_rank[1];
    select_digit(hist + 2 * kSelectBins, 2, rin, S);
    if (threadIdx.x == 0) {
        st->prefix = st->sel_prefix[1] | S.found_digit;
        st->rank = rin - S.found_before;
        const float sg = fmaxf(__uint_as_float(st->prefix), floor_);
        st->sigma = sg;
        st->inv_sigma2 = 1.0f / (sg * sg);
    }
}

hipError_t launch_select_sigma(DevState* st, const uint32_t* hist, float sigma_floor, hipStream_t s)
{
    hipLaunchKernelGGL(k_select_sigma, dim3(1), dim3(256), 0, s, st, hist, sigma_floor);
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
__device__ __forceinline__ float weight(float tv, float inv_s2) { return __expf(-(tv * tv) * inv_s2); }

// The step f - t g of the previous descent step (none when it was rejected),
// evaluated with the same float operation as the final update kernel.
__device__ __forceinline__ float stepped(float f, float g, int k, float t) { return k >= 0 ? fmaf(-t, g, f) : f; }

// g = lambda (f - v) + A2 at the current iterate, with the weights at it.
// When g_prev is given the current iterate is first formed from the previous
// one, f - t g_prev (the previous step's decision in st_prev), and stored to
// f_out.  Per-block partials: (Q(f) = sum of w TV over owned edges +
// lambda/2 (f - v)^2, ||g||^2).
__device__ __forceinline__ void tv_grad_block(const float* __restrict__ f, const float* __restrict__ g_prev,
                                              const DevState* st_prev, float* __restrict__ f_out,
                                              const float* __restrict__ v, int nx, int ny, float lambda,
                                              const DevState* st, float inv_s2_direct, float eps2,
                                              float* __restrict__ g, float* wx, float* wy, double* part, int bx,
                                              int by, int b, int nb, double* lds, const float* wx_in = nullptr,
                                              const float* wy_in = nullptr)
{
    const float inv_s2 = st ? st->inv_sigma2 : inv_s2_direct;
    const int i = bx * kT + (threadIdx.x & (kT - 1)), j = by * kT + threadIdx.x / kT;
    double q = 0.0, gg = 0.0;
    if (i < nx && j < ny) {
        Nbhd N;
        load_nbhd(f, nx, ny, i, j, N);
        if (g_prev) {
            Nbhd G;
            load_nbhd(g_prev, nx, ny, i, j, G);
            const int kp = st_prev->k;
            const float tp = st_prev->t;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) N.n[a][b] = stepped(N.n[a][b], G.n[a][b], kp, tp);
            // outside pixels stay zero: f and g are both zero there
            f_out[(size_t)j * nx + i] = N.n[1][1];
        }
        const float c = N.n[1][1];
        const float tR = tv_right(N, eps2), tL = tv_left(N, eps2), tU = tv_up(N, eps2), tD = tv_down(N, eps2);
        // Eq. 5's weights, or the caller's (given half-edge weights in place of Eq. 5)
        const size_t xw = (size_t)j * (nx + 1);
        const float wR = wx_in ? wx_in[xw + i + 1] : weight(tR, inv_s2);
        const float wL = wx_in ? wx_in[xw + i] : weight(tL, inv_s2);
        const float wU = wy_in ? wy_in[(size_t)(j + 1) * nx + i] : weight(tU, inv_s2);
        const float wD = wy_in ? wy_in[(size_t)j * nx + i] : weight(tD, inv_s2);
        const float FR = wR * (N.n[2][1] - c) * hw_rcp(tR);
        const float FL = wL * (c - N.n[0][1]) * hw_rcp(tL);
        const float FU = wU * (N.n[1][2] - c) * hw_rcp(tU);
        const float FD = wD * (c - N.n[1][0]) * hw_rcp(tD);
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
        if (threadIdx.x == 0) {  // slot-major: [Q | ||g||^2][block]
            part[b] = qs;
            part[nb + b] = gs;
        }
    }
}

__global__ __launch_bounds__(256) void k_tv_grad(const float* __restrict__ f, const float* __restrict__ g_prev,
                                                 const DevState* st_prev, float* __restrict__ f_out,
                                                 const float* __restrict__ v, int nx, int ny, float lambda,
                                                 const DevState* st, float inv_s2_direct, float eps2,
                                                 float* __restrict__ g, float* wx, float* wy, double* part,
                                                 const float* wx_in, const float* wy_in)
{
    __shared__ double lds[4];
    tv_grad_block(f, g_prev, st_prev, f_out, v, nx, ny, lambda, st, inv_s2_direct, eps2, g, wx, wy, part,
                  blockIdx.x, blockIdx.y, blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y, lds, wx_in,
                  wy_in);
}

hipError_t launch_tv_grad(const Plan& p, const float* f, const float* g_prev, const DevState* st_prev, float* f_out,
                          const float* v, float lambda, const DevState* st, float sigma_direct, float eps2, float* g,
                          float* wx, float* wy, double* part, hipStream_t s, const float* wx_in,
                          const float* wy_in)
{
    const float inv_s2 = (sigma_direct > 0.0f && std::isfinite(sigma_direct)) ? 1.0f / (sigma_direct * sigma_direct)
                                                                             : 0.0f;
    dim3 grid((p.nx + kT - 1) / kT, (p.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_tv_grad, grid, dim3(256), 0, s, f, g_prev, st_prev, f_out, v, p.nx, p.ny, lambda, st, inv_s2,
                       eps2, g, wx, wy, part, wx_in, wy_in);
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

// Energies Q(f - t_k g) of pixel (i, j)'s share (its own fidelity term and the
// half-edges it owns) for NC consecutive candidates from k0, with the weights
// frozen at f.
template <int NC>
__device__ __forceinline__ void candidate_energies(const float* f, const float* g, const float* v, const float* wx,
                                                   const float* wy, int nx, int ny, int i, int j, float lambda,
                                                   float eps2, float t0, float shrink, int k0, double* e)
{
    Nbhd F, G;
    load_nbhd(f, nx, ny, i, j, F);
    load_nbhd(g, nx, ny, i, j, G);
    const size_t xo = (size_t)j * (nx + 1);
    const float wR = wx[xo + i + 1], wU = wy[(size_t)(j + 1) * nx + i];
    const float wL = i == 0 ? wx[xo] : 0.0f, wD = j == 0 ? wy[i] : 0.0f;
    const float vv = v[(size_t)j * nx + i];
    float t = cand_t(t0, shrink, k0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        Nbhd H;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) H.n[a][bb] = fmaf(-t, G.n[a][bb], F.n[a][bb]);
        float s = wR * tv_right(H, eps2) + wU * tv_up(H, eps2);
        if (i == 0) s += wL * tv_left(H, eps2);
        if (j == 0) s += wD * tv_down(H, eps2);
        const float d = H.n[1][1] - vv;
        e[c] += (double)s + 0.5 * (double)lambda * (double)d * (double)d;
        t *= shrink;
    }
}

// ------------------------------------------------------------------ one descent step's direction and trials, fused
// The direction of tv_grad_block and the first kArmijoFirst Armijo trials
// (candidate_energies) in one pass: the block forms the current iterate on
// its tile plus a 2-pixel halo in LDS, the direction on the tile plus a
// 1-pixel halo (halo values recomputed with the same operations as their
// owning block, so they are bit-identical), and the trial energies of its
// own pixels from those.  Per-block partials: [Q | ||g||^2][block] and
// [trial][block], each summed over the block's pixels in a fixed order.
struct TvArmShared {
    float f[kT + 4][kT + 4];   // current iterate, tile + 2-pixel halo
    float g[kT + 2][kT + 2];   // direction, tile + 1-pixel halo
    float w[4][kT][kT];        // own pixels' weights: right, left, up, down
    float e[kT][kT];           // own pixels' weighted half-edge sum
    float dv[kT][kT];          // own pixels' f - v
    double lds[4];
    double red[4][kArmijoFirst];
    SelShared sel;
};

__device__ __forceinline__ void tv_armijo_block(const float* __restrict__ f, const float* __restrict__ g_prev,
                                                const DevState* st_prev, float* __restrict__ f_out,
                                                const float* __restrict__ v, int nx, int ny, float lambda,
                                                const DevState* st, float eps2, float* __restrict__ g, float* wx,
                                                float* wy, double* part_grad, double* part_arm, float t0,
                                                float shrink, int bx, int by, int b, int nb, TvArmShared& S,
                                                const float* wx_in = nullptr, const float* wy_in = nullptr,
                                                DevState* sel_st = nullptr, const uint32_t* sel_hist = nullptr,
                                                float sel_floor = 0.0f)
{
    const int i0 = bx * kT, j0 = by * kT;
    const int kp = g_prev ? st_prev->k : -1;
    const float tp = g_prev ? st_prev->t : 0.0f;
    // the current iterate on the window (zero outside the image, like pix())
    constexpr int kWin = (kT + 4) * (kT + 4);
    auto win_value = [&](int idx) {
        const int li = idx % (kT + 4), lj = idx / (kT + 4);
        const int gi = i0 - 2 + li, gj = j0 - 2 + lj;
        float val = 0.0f;
        if ((unsigned)gi < (unsigned)nx && (unsigned)gj < (unsigned)ny) {
            const size_t id = (size_t)gj * nx + gi;
            val = f[id];
            if (g_prev) val = stepped(val, g_prev[id], kp, tp);
        }
        return val;
    };
    float inv_s2;
    if (sel_hist) {
        // sigma: the first descent step of an adaptive iteration closes the
        // selection's last digit itself (the same computation in every block,
        // as k_select_sigma would do it; block 0 records it for the later
        // steps), with the window's loads issued first so that they overlap it
        constexpr int kWinPer = (kWin + 255) / 256;
        float fv[kWinPer];
#pragma unroll
        for (int u = 0; u < kWinPer; ++u) {
            const int idx = threadIdx.x + 256 * u;
            fv[u] = idx < kWin ? win_value(idx) : 0.0f;
        }
        const uint32_t rin = sel_st->sel_rank[1];
        select_digit(sel_hist, 2, rin, S.sel);
        const uint32_t prefix = sel_st->sel_prefix[1] | S.sel.found_digit;
        const float sg = fmaxf(__uint_as_float(prefix), sel_floor);
        inv_s2 = 1.0f / (sg * sg);
        if (b == 0 && threadIdx.x == 0) {
            sel_st->prefix = prefix;
            sel_st->rank = rin - S.sel.found_before;
            sel_st->sigma = sg;
            sel_st->inv_sigma2 = inv_s2;
        }
#pragma unroll
        for (int u = 0; u < kWinPer; ++u) {
            const int idx = threadIdx.x + 256 * u;
            if (idx < kWin) S.f[idx / (kT + 4)][idx % (kT + 4)] = fv[u];
        }
    } else {
        inv_s2 = st->inv_sigma2;
        for (int idx = threadIdx.x; idx < kWin; idx += 256) S.f[idx / (kT + 4)][idx % (kT + 4)] = win_value(idx);
    }
    __syncthreads();
    const int ti = threadIdx.x & (kT - 1), tj = threadIdx.x / kT;
    const int i = i0 + ti, j = j0 + tj;
    const bool own = i < nx && j < ny;
    if (g_prev && own) f_out[(size_t)j * nx + i] = S.f[tj + 2][ti + 2];
    // the direction on the tile and its 1-pixel halo
    for (int idx = threadIdx.x; idx < (kT + 2) * (kT + 2); idx += 256) {
        const int li = idx % (kT + 2), lj = idx / (kT + 2);
        const int gi = i0 - 1 + li, gj = j0 - 1 + lj;
        float gv = 0.0f;
        if ((unsigned)gi < (unsigned)nx && (unsigned)gj < (unsigned)ny) {
            Nbhd N;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) N.n[a][bb] = S.f[lj + bb][li + a];
            const float c = N.n[1][1];
            const float tR = tv_right(N, eps2), tL = tv_left(N, eps2), tU = tv_up(N, eps2), tD = tv_down(N, eps2);
            const size_t xw = (size_t)gj * (nx + 1);
            const float wR = wx_in ? wx_in[xw + gi + 1] : weight(tR, inv_s2);
            const float wL = wx_in ? wx_in[xw + gi] : weight(tL, inv_s2);
            const float wU = wy_in ? wy_in[(size_t)(gj + 1) * nx + gi] : weight(tU, inv_s2);
            const float wD = wy_in ? wy_in[(size_t)gj * nx + gi] : weight(tD, inv_s2);
            const float FR = wR * (N.n[2][1] - c) * hw_rcp(tR);
            const float FL = wL * (c - N.n[0][1]) * hw_rcp(tL);
            const float FU = wU * (N.n[1][2] - c) * hw_rcp(tU);
            const float FD = wD * (c - N.n[1][0]) * hw_rcp(tD);
            const size_t id = (size_t)gj * nx + gi;
            const float dv = c - v[id];
            gv = lambda * dv - (FR - FL) - (FU - FD);
            if (li >= 1 && li <= kT && lj >= 1 && lj <= kT) {  // an own pixel
                g[id] = gv;
                if (wx) {
                    wx[xw + gi + 1] = wR;
                    if (gi == 0) wx[xw] = wL;
                }
                if (wy) {
                    wy[(size_t)(gj + 1) * nx + gi] = wU;
                    if (gj == 0) wy[gi] = wD;
                }
                float e = wR * tR + wU * tU;
                if (gi == 0) e += wL * tL;
                if (gj == 0) e += wD * tD;
                S.w[0][lj - 1][li - 1] = wR;
                S.w[1][lj - 1][li - 1] = wL;
                S.w[2][lj - 1][li - 1] = wU;
                S.w[3][lj - 1][li - 1] = wD;
                S.e[lj - 1][li - 1] = e;
                S.dv[lj - 1][li - 1] = dv;
            }
        }
        S.g[lj][li] = gv;
    }
    __syncthreads();
    // the partials of the direction kernel, in its thread order
    double q = 0.0, gg = 0.0;
    double en[kArmijoFirst];
#pragma unroll
    for (int c = 0; c < kArmijoFirst; ++c) en[c] = 0.0;
    if (own) {
        const float dv = S.dv[tj][ti], gv = S.g[tj + 1][ti + 1];
        q = (double)S.e[tj][ti] + 0.5 * (double)lambda * (double)dv * (double)dv;
        gg = (double)gv * (double)gv;
        // the trial energies, as candidate_energies with the weights frozen at f
        Nbhd F, G;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                F.n[a][bb] = S.f[tj + 1 + bb][ti + 1 + a];
                G.n[a][bb] = S.g[tj + bb][ti + a];
            }
        const float wR = S.w[0][tj][ti], wU = S.w[2][tj][ti];
        const float wL = i == 0 ? S.w[1][tj][ti] : 0.0f, wD = j == 0 ? S.w[3][tj][ti] : 0.0f;
        const float vv = v[(size_t)j * nx + i];
        float t = t0;
#pragma unroll
        for (int c = 0; c < kArmijoFirst; ++c) {
            Nbhd H;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) H.n[a][bb] = fmaf(-t, G.n[a][bb], F.n[a][bb]);
            float sm = wR * tv_right(H, eps2) + wU * tv_up(H, eps2);
            if (i == 0) sm += wL * tv_left(H, eps2);
            if (j == 0) sm += wD * tv_down(H, eps2);
            const float d = H.n[1][1] - vv;
            en[c] += (double)sm + 0.5 * (double)lambda * (double)d * (double)d;
            t *= shrink;
        }
    }
    const double qs = block_sum<256>(q, S.lds);
    const double gs = block_sum<256>(gg, S.lds);
    if (threadIdx.x == 0) {  // slot-major: [Q | ||g||^2][block]
        part_grad[b] = qs;
        part_grad[nb + b] = gs;
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < kArmijoFirst; ++c) {
        const double sc = wave_sum(en[c]);
        if (l == 0) S.red[w][c] = sc;
    }
    __syncthreads();
    if (threadIdx.x < kArmijoFirst) {
        const int c = threadIdx.x;
        part_arm[(size_t)c * nb + b] = S.red[0][c] + S.red[1][c] + S.red[2][c] + S.red[3][c];
    }
}

__global__ __launch_bounds__(256) void k_tv_armijo(const float* __restrict__ f, const float* __restrict__ g_prev,
                                                   const DevState* st_prev, float* __restrict__ f_out,
                                                   const float* __restrict__ v, int nx, int ny, float lambda,
                                                   const DevState* st, float eps2, float* __restrict__ g, float* wx,
                                                   float* wy, double* part_grad, double* part_arm, float t0,
                                                   float shrink, const float* wx_in, const float* wy_in,
                                                   DevState* sel_st, const uint32_t* sel_hist, float sel_floor)
{
    __shared__ TvArmShared S;
    tv_armijo_block(f, g_prev, st_prev, f_out, v, nx, ny, lambda, st, eps2, g, wx, wy, part_grad, part_arm, t0,
                    shrink, blockIdx.x, blockIdx.y, blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y, S,
                    wx_in, wy_in, sel_st, sel_hist, sel_floor);
}

hipError_t launch_tv_armijo(const Plan& p, const float* f, const float* g_prev, const DevState* st_prev,
                            float* f_out, const float* v, float lambda, const DevState* st, float eps2, float* g,
                            float* wx, float* wy, double* part_grad, double* part_arm, float t0, float shrink,
                            hipStream_t s, const float* wx_in, const float* wy_in, DevState* sel_st,
                            const uint32_t* sel_hist, float sel_floor)
{
    dim3 grid((p.nx + kT - 1) / kT, (p.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_tv_armijo, grid, dim3(256), 0, s, f, g_prev, st_prev, f_out, v, p.nx, p.ny, lambda, st,
                       eps2, g, wx, wy, part_grad, part_arm, t0, shrink, wx_in, wy_in, sel_st, sel_hist, sel_floor);
    return hipGetLastError();
}

int armijo_blocks(const Plan& p) { return ((p.nx + kT - 1) / kT) * ((p.ny + kT - 1) / kT); }


// The Armijo decision: the first candidate with Q_k <= Q0 - c t_k ||g||^2.
// One block of 256 threads closes Q0, ||g||^2 (gradient kernel's partials)
// and the first kArmijoFirst candidate energies (Armijo kernel's partials):
// thread t sums blocks t, t + 256, ... of every slot in order, the per-thread
// sums go through LDS, and each wave reduces a few slots with a fixed
// butterfly.  Should none of the first candidates pass while more backtracks
// are allowed (which a reasonable first step t0 never needs), this block goes
// on alone through the image, kArmijoMore candidates at a time: slow, but the
// decision is the same.  Without an accepted candidate the step is skipped
// (k = -1, t = 0).  The accepted index is recorded for the iteration.
constexpr int kDecThreads = 256;
constexpr int kDecVals = kArmijoMore + 2;

template <int NV>
__device__ __forceinline__ void decide_reduce(double* v, double (*red)[kDecThreads], double* tot)
{
    // v[0..NV) per thread -> tot[0..NV) block sums, fixed order
#pragma unroll
    for (int c = 0; c < NV; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int c = w; c < NV; c += kDecThreads / 64) {
        double a = 0.0;
        for (int q = l; q < kDecThreads; q += 64) a += red[c][q];
        a = wave_sum(a);
        if (l == 0) tot[c] = a;
    }
    __syncthreads();
}

struct DecShared {
    double red[kDecVals][kDecThreads];
    double tot[kDecVals];
    double q_acc;  // the energy at the accepted point
    int verdict;
};

__device__ __forceinline__ void armijo_decide_block(DevState* st, const double* part_grad, const double* part_arm,
                                                    int nb, int max_bt, double c_arm, float t0, float shrink,
                                                    int32_t* st_k, double* st_q0, double* st_q1, int step, int T,
                                                    const float* f, const float* g, const float* v, const float* wx,
                                                    const float* wy, int nx, int ny, float lambda, float eps2,
                                                    DecShared& S, int replay = 0)
{
    double (*red)[kDecThreads] = S.red;
    double* tot = S.tot;
    int& verdict = S.verdict;
    double a[kArmijoFirst + 2];
#pragma unroll
    for (int c = 0; c < kArmijoFirst + 2; ++c) a[c] = 0.0;
    // four blocks per thread at a time, all their loads issued before the sums
    // (the same order of additions as one block at a time)
    constexpr int kDecRounds = 4;
    for (int b0 = threadIdx.x; b0 < nb; b0 += kDecRounds * kDecThreads) {
        double v[kDecRounds][kArmijoFirst + 2];
#pragma unroll
        for (int r = 0; r < kDecRounds; ++r) {
            const int b = b0 + r * kDecThreads;
#pragma unroll
            for (int c = 0; c < kArmijoFirst; ++c) v[r][c] = b < nb ? part_arm[(size_t)c * nb + b] : 0.0;
            v[r][kArmijoFirst] = b < nb ? part_grad[b] : 0.0;
            v[r][kArmijoFirst + 1] = b < nb ? part_grad[nb + b] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kDecRounds; ++r)
#pragma unroll
            for (int c = 0; c < kArmijoFirst + 2; ++c) a[c] += v[r][c];
    }
    decide_reduce<kArmijoFirst + 2>(a, red, tot);
    const double q0 = tot[kArmijoFirst], g2 = tot[kArmijoFirst + 1];
    if (threadIdx.x == 0) {
        int kk = -1;
        if (replay) {  // the caller's decision, recorded for this step (-1: no step)
            kk = st_k[(size_t)st->iter * T + step];
        } else {
            for (int k = 0; k < kArmijoFirst && k <= max_bt; ++k)
                if (tot[k] <= q0 - c_arm * (double)cand_t(t0, shrink, k) * g2) {
                    kk = k;
                    break;
                }
        }
        verdict = kk;
        // the energy at the accepted point (the start's when none; later
        // candidates are filled in below)
        S.q_acc = kk < 0 ? q0 : (kk < kArmijoFirst ? tot[kk] : 0.0);
    }
    __syncthreads();
    int kk = verdict;
    if (replay && kk >= kArmijoFirst) {
        // a given index beyond the fused trials: evaluate that candidate (the
        // sums in the order the search below would form them)
        double e[kArmijoMore];
#pragma unroll
        for (int c = 0; c < kArmijoMore; ++c) e[c] = 0.0;
        for (int px = threadIdx.x; px < nx * ny; px += kDecThreads)
            candidate_energies<kArmijoMore>(f, g, v, wx, wy, nx, ny, px % nx, px / nx, lambda, eps2, t0, shrink, kk,
                                            e);
        decide_reduce<kArmijoMore>(e, red, tot);
        if (threadIdx.x == 0) S.q_acc = tot[0];
        __syncthreads();
    }
    // rare: continue the backtracking over the whole image in this block
    for (int k0 = kArmijoFirst; !replay && kk < 0 && k0 <= max_bt; k0 += kArmijoMore) {
        double e[kArmijoMore];
#pragma unroll
        for (int c = 0; c < kArmijoMore; ++c) e[c] = 0.0;
        for (int px = threadIdx.x; px < nx * ny; px += kDecThreads)
            candidate_energies<kArmijoMore>(f, g, v, wx, wy, nx, ny, px % nx, px / nx, lambda, eps2, t0, shrink, k0,
                                            e);
        decide_reduce<kArmijoMore>(e, red, tot);
        if (threadIdx.x == 0) {
            int found = -1;
            for (int c = 0; c < kArmijoMore && k0 + c <= max_bt; ++c)
                if (tot[c] <= q0 - c_arm * (double)cand_t(t0, shrink, k0 + c) * g2) {
                    found = k0 + c;
                    S.q_acc = tot[c];
                    break;
                }
            verdict = found;
        }
        __syncthreads();
        kk = verdict;
    }
    if (threadIdx.x == 0) {
        st->q0 = q0;
        st->gg = g2;
        st->k = kk;
        st->t = kk >= 0 ? cand_t(t0, shrink, kk) : 0.0f;
        const size_t rec = (size_t)st->iter * T + step;
        if (st_k) st_k[rec] = kk;
        if (st_q0) st_q0[rec] = q0;
        if (st_q1) st_q1[rec] = S.q_acc;
    }
}

__global__ __launch_bounds__(kDecThreads) void k_armijo_decide(DevState* st, const double* part_grad,
                                                               const double* part_arm, int nb, int max_bt,
                                                               double c_arm, float t0, float shrink, int32_t* st_k,
                                                               double* st_q0, double* st_q1, int step, int T,
                                                               const float* f, const float* g, const float* v,
                                                               const float* wx, const float* wy, int nx, int ny,
                                                               float lambda, float eps2, int replay)
{
    __shared__ DecShared S;
    armijo_decide_block(st, part_grad, part_arm, nb, max_bt, c_arm, t0, shrink, st_k, st_q0, st_q1, step, T, f, g, v,
                        wx, wy, nx, ny, lambda, eps2, S, replay);
}

hipError_t launch_armijo_decide(const Plan& p, DevState* st, const double* part_grad, const double* part_arm,
                                int max_bt, double c_arm, float t0, float shrink, int32_t* st_k, double* st_q0,
                                double* st_q1, int step, int T, const float* f, const float* g, const float* v,
                                const float* wx, const float* wy, float lambda, float eps2, hipStream_t s,
                                int replay)
{
    hipLaunchKernelGGL(k_armijo_decide, dim3(1), dim3(kDecThreads), 0, s, st, part_grad, part_arm, armijo_blocks(p),
                       max_bt, c_arm, t0, shrink, st_k, st_q0, st_q1, step, T, f, g, v, wx, wy, p.nx, p.ny, lambda,
                       eps2, replay && st_k ? 1 : 0);
    return hipGetLastError();
}

// f_out = f - t g (unchanged when no step was accepted), optional truncation at
// zero (step 3 of the algorithm) and optional transposed copy for the projector.
__device__ __forceinline__ void p2_update_block(const DevState* st, const float* fcur, const float* __restrict__ g,
                                                float* fout, float* foutT, int clamp, int nx, int ny, int tbx,
                                                int tby, float (*tl)[33])
{
    const int k = st->k;
    const float t = st->t;
    const int bx = tbx * 32, by = tby * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = bx + tx, j = by + r;
        float val = 0.0f;
        if (i < nx && j < ny) {
            const size_t id = (size_t)j * nx + i;
            val = stepped(fcur[id], g[id], k, t);
            if (clamp) val = fmaxf(val, 0.0f);
            fout[id] = val;
        }
        tl[r][tx] = val;
    }
    if (foutT) {
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = bx + r, j = by + tx;
            if (i < nx && j < ny) foutT[(size_t)i * ny + j] = tl[tx][r];
        }
    }
}

// Squared error to ref over the pixels of 32 x 32 update tile (tbx, tby), in
// the order p2_update_block writes them (thread (tx, ty): rows ty, ty + 8, ...),
// summed over the block (valid in all threads).  Contains __syncthreads().
__device__ __forceinline__ double update_tile_sq_err(const float* fout, const float* ref, int nx, int ny, int tbx,
                                                     int tby, double* lds)
{
    const int i = tbx * 32 + (threadIdx.x & 31);
    double e2 = 0.0;
    for (int r = threadIdx.x >> 5; r < 32; r += 8) {
        const int j = tby * 32 + r;
        if (i < nx && j < ny) {
            const double d = (double)fout[(size_t)j * nx + i] - (double)ref[(size_t)j * nx + i];
            e2 += d * d;
        }
    }
    return block_sum<256>(e2, lds);
}

// With a reference, each block also writes the squared error of its new
// pixels (one partial per 32 x 32 tile) for the iteration's RMSE record, so
// that needs no kernel of its own.
__global__ __launch_bounds__(256) void k_p2_update(const DevState* st, const float* fcur, const float* __restrict__ g,
                                                   float* fout, float* foutT, int clamp, int nx, int ny,
                                                   const float* ref, double* part_rmse)
{
    __shared__ float tl[32][33];
    __shared__ double lds[4];
    p2_update_block(st, fcur, g, fout, foutT, clamp, nx, ny, blockIdx.x, blockIdx.y, tl);
    if (ref) {
        const double e2 = update_tile_sq_err(fout, ref, nx, ny, blockIdx.x, blockIdx.y, lds);
        if (threadIdx.x == 0) part_rmse[blockIdx.y * gridDim.x + blockIdx.x] = e2;
    }
}

int update_tiles(const Plan& p) { return ((p.nx + 31) / 32) * ((p.ny + 31) / 32); }

hipError_t launch_p2_update(const Plan& p, const DevState* st, const float* fcur, const float* g, float* fout,
                            float* foutT, int clamp, hipStream_t s, const float* ref, double* part_rmse)
{
    dim3 grid((p.nx + 31) / 32, (p.ny + 31) / 32);
    hipLaunchKernelGGL(k_p2_update, grid, dim3(256), 0, s, st, fcur, g, fout, foutT, clamp, p.nx, p.ny, ref,
                       part_rmse);
    return hipGetLastError();
}

__device__ __forceinline__ void copy_clamp_block(const float* src, float* dst, float* dstT, int clamp, int nx, int ny,
                                                 int tbx, int tby, float (*tl)[33])
{
    const int bx = tbx * 32, by = tby * 32;
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

__global__ __launch_bounds__(256) void k_copy_clamp(const float* src, float* dst, float* dstT, int clamp, int nx,
                                                    int ny)
{
    __shared__ float tl[32][33];
    copy_clamp_block(src, dst, dstT, clamp, nx, ny, blockIdx.x, blockIdx.y, tl);
}

hipError_t launch_copy_clamp(const Plan& p, const float* src, float* dst, float* dstT, int clamp, hipStream_t s)
{
    dim3 grid((p.nx + 31) / 32, (p.ny + 31) / 32);
    hipLaunchKernelGGL(k_copy_clamp, grid, dim3(256), 0, s, src, dst, dstT, clamp, p.nx, p.ny);
    return hipGetLastError();
}

// ------------------------------------------------------------------ VJP of the direction
// (dg/df)^T u with sigma fixed, for differentiating through descent steps.
// With g = lambda (f - v) + sum_e F_e (e_B - e_A) over half-edges from pixel A
// to pixel B, F_e = w d / TV (d = f_B - f_A, t1 and t2 the pair-mean
// differences of Eq. A3, w = exp(-TV^2/sigma^2)):
//   dF/dd = w/TV - c d, dF/dt1 = -c t1/2, dF/dt2 = -c t2/2,
//   c = w d (1/TV + 2 TV/sigma^2) / TV^2.
// Pass 1 stores per edge, scaled by u_B - u_A: DD = dF/dd and the half
// derivatives H1 = dF/dt1 / 2, H2 = dF/dt2 / 2 (edge order as for the keys).
// Pass 2 gathers per pixel: as A of an edge -DD - H1 + H2, as B +DD - H1 + H2,
// as a member of the pair beyond the edge (A+p, B+p) +H1, of the pair before
// it (A-p, B-p) -H2.
__device__ __forceinline__ void vjp_coef(float a, float b, float au, float bu, float ad, float bd, float ua,
                                         float ub, float inv_s2, float eps2, float* e3, size_t ne, size_t e)
{
    const float d = b - a;
    const float m0 = 0.5f * (a + b), t1 = 0.5f * (au + bu) - m0, t2 = m0 - 0.5f * (ad + bd);
    const float tv = hw_sqrt(d * d + 0.5f * (t1 * t1) + 0.5f * (t2 * t2) + eps2);
    const float itv = hw_rcp(tv);
    const float w = weight(tv, inv_s2);
    const float c = w * d * (itv + 2.0f * tv * inv_s2) * (itv * itv);
    const float ue = ub - ua;
    e3[e] = ue * (w * itv - c * d);
    e3[ne + e] = -0.25f * ue * c * t1;
    e3[2 * ne + e] = -0.25f * ue * c * t2;
}

__global__ __launch_bounds__(256) void k_vjp_edges(const float* __restrict__ f, const float* __restrict__ u, int nx,
                                                   int ny, float inv_s2, float eps2, float* e3)
{
    const int i = blockIdx.x * kT + (threadIdx.x & (kT - 1)), j = blockIdx.y * kT + threadIdx.x / kT;
    if (i >= nx || j >= ny) return;
    Nbhd N;
    load_nbhd(f, nx, ny, i, j, N);
    const size_t ne = (size_t)ny * (nx + 1) + (size_t)(ny + 1) * nx;
    const size_t xo = (size_t)j * (nx + 1), yo = (size_t)ny * (nx + 1);
    const float uc = u[(size_t)j * nx + i];
    const float ur = pix(u, nx, ny, i + 1, j), uu = pix(u, nx, ny, i, j + 1);
    // right edge (i+1/2, j): A = (i, j), B = (i+1, j), p = (0, 1)
    vjp_coef(N.n[1][1], N.n[2][1], N.n[1][2], N.n[2][2], N.n[1][0], N.n[2][0], uc, ur, inv_s2, eps2, e3, ne,
             xo + i + 1);
    // up edge (i, j+1/2): A = (i, j), B = (i, j+1), p = (1, 0)
    vjp_coef(N.n[1][1], N.n[1][2], N.n[2][1], N.n[2][2], N.n[0][1], N.n[0][2], uc, uu, inv_s2, eps2, e3, ne,
             yo + (size_t)(j + 1) * nx + i);
    if (i == 0)  // left border edge: A is outside the image
        vjp_coef(N.n[0][1], N.n[1][1], N.n[0][2], N.n[1][2], N.n[0][0], N.n[1][0], 0.0f, uc, inv_s2, eps2, e3, ne,
                 xo);
    if (j == 0)  // bottom border edge
        vjp_coef(N.n[1][0], N.n[1][1], N.n[2][0], N.n[2][1], N.n[0][0], N.n[0][1], 0.0f, uc, inv_s2, eps2, e3, ne,
                 yo + i);
}

__global__ __launch_bounds__(256) void k_vjp_gather(const float* __restrict__ e3, const float* __restrict__ u,
                                                    int nx, int ny, float lambda, float* out)
{
    const int i = blockIdx.x * kT + (threadIdx.x & (kT - 1)), j = blockIdx.y * kT + threadIdx.x / kT;
    if (i >= nx || j >= ny) return;
    const size_t ne = (size_t)ny * (nx + 1) + (size_t)(ny + 1) * nx, yo = (size_t)ny * (nx + 1);
    const float* DD = e3;
    const float* H1 = e3 + ne;
    const float* H2 = e3 + 2 * ne;
    // x-edge between (a, b) and (a+1, b), a in [-1, nx-1], b in [0, ny-1]
    auto xe = [&](int a, int b) -> long long {
        return (b >= 0 && b < ny) ? (long long)b * (nx + 1) + a + 1 : -1;
    };
    // y-edge between (a, b) and (a, b+1), a in [0, nx-1], b in [-1, ny-1]
    auto ye = [&](int a, int b) -> long long {
        return (a >= 0 && a < nx) ? (long long)(yo + (size_t)(b + 1) * nx + a) : -1;
    };
    auto h1 = [&](long long e) { return e >= 0 ? H1[e] : 0.0f; };
    auto h2 = [&](long long e) { return e >= 0 ? H2[e] : 0.0f; };
    float acc = lambda * u[(size_t)j * nx + i];
    {
        const long long ea = xe(i, j), eb = xe(i - 1, j);  // this pixel is A of ea, B of eb
        acc += -DD[ea] - H1[ea] + H2[ea];
        acc += DD[eb] - H1[eb] + H2[eb];
        acc += h1(xe(i, j - 1)) + h1(xe(i - 1, j - 1));
        acc -= h2(xe(i, j + 1)) + h2(xe(i - 1, j + 1));
    }
    {
        const long long ea = ye(i, j), eb = ye(i, j - 1);
        acc += -DD[ea] - H1[ea] + H2[ea];
        acc += DD[eb] - H1[eb] + H2[eb];
        acc += h1(ye(i - 1, j)) + h1(ye(i - 1, j - 1));
        acc -= h2(ye(i + 1, j)) + h2(ye(i + 1, j - 1));
    }
    out[(size_t)j * nx + i] = acc;
}

hipError_t launch_tv_vjp(const Plan& p, const float* f, const float* u, float lambda, float sigma, float eps2,
                         float* e3, float* out, hipStream_t s)
{
    dim3 grid((p.nx + kT - 1) / kT, (p.ny + kT - 1) / kT);
    const float inv_s2 = std::isinf(sigma) ? 0.0f : 1.0f / (sigma * sigma);
    hipLaunchKernelGGL(k_vjp_edges, grid, dim3(256), 0, s, f, u, p.nx, p.ny, inv_s2, eps2, e3);
    hipLaunchKernelGGL(k_vjp_gather, grid, dim3(256), 0, s, e3, u, p.nx, p.ny, lambda, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ batched kernels (see batch.h)
// A block takes a contiguous run of the (slice, tile) items (slice-major), so
// it accumulates one slice's histogram over several tiles and flushes it
// only when the slice changes (the flushes' global atomics are what
// serialise: flat regions put most half-edges into a few bins).
__global__ __launch_bounds__(256) void kb_edges_hist(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                     int n_items, int imgs, float eps2)
{
    __shared__ uint32_t h[kSelectBins];
    const int per = (n_items + (int)gridDim.x - 1) / (int)gridDim.x;
    const int beg = (int)blockIdx.x * per, end = min(n_items, beg + per);
    if (beg >= end) return;  // whole block
    hist_clear(h);
    int cur = items[beg].x;
    for (int it = beg; it < end; ++it) {
        const int2 w = items[it];
        if (w.x != cur) {  // uniform over the block
            hist_flush(h, sl[cur].hist);
            __syncthreads();
            hist_clear(h);
            cur = w.x;
        }
        const SliceDev& d = sl[w.x];
        edges_tile(d.buf[imgs], d.nx, d.ny, eps2, d.keys, w.y % d.t16x, w.y / d.t16x, h);
    }
    hist_flush(h, sl[cur].hist);
}

hipError_t blaunch_edges_hist(const BatchDev& b, int img, float eps2, hipStream_t s)
{
    const int n = b.n_items[kShT16];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_edges_hist, dim3(b.grid[kShT16]), dim3(256), 0, s, b.slices, b.items[kShT16], n, img, eps2);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_select_hist(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                      int n_items, int pass)
{
    __shared__ uint32_t h[kSelectBins];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        __syncthreads();
        select_hist_block(d.keys, (size_t)d.n_edges, pass, d.st->prefix, d.hist + pass * kSelectBins, w.y,
                          d.sel_blocks, h);
    }
}

hipError_t blaunch_select_hist(const BatchDev& b, int pass, hipStream_t s)
{
    const int n = b.n_items[kShSel];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_select_hist, dim3(b.grid[kShSel]), dim3(256), 0, s, b.slices, b.items[kShSel], n, pass);
    return hipGetLastError();
}

// one block per slice
__global__ __launch_bounds__(256) void kb_select_finalize(const SliceDev* __restrict__ sl, int pass, float floor_)
{
    __shared__ SelShared S;
    const SliceDev& d = sl[blockIdx.x];
    select_finalize_block(d.st, pass, d.hist + pass * kSelectBins, floor_, S);
}

hipError_t blaunch_select_finalize(const BatchDev& b, int pass, float floor_, hipStream_t s)
{
    hipLaunchKernelGGL(kb_select_finalize, dim3(b.n), dim3(256), 0, s, b.slices, pass, floor_);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_tv_armijo(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                    int n_items, int fs, int gps, int fos, int vs, float lambda,
                                                    float eps2, int gs, float t0, float shrink)
{
    __shared__ TvArmShared S;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        __syncthreads();
        tv_armijo_block(d.buf[fs], bsel(d, gps), d.st, bsel(d, fos), d.buf[vs], d.nx, d.ny, lambda, d.st, eps2,
                        d.buf[gs], d.buf[kBufWX], d.buf[kBufWY], d.part[kPartGrad], d.part[kPartArm], t0, shrink,
                        w.y % d.t16x, w.y / d.t16x, w.y, d.t16x * d.t16y, S);
    }
}

hipError_t blaunch_tv_armijo(const BatchDev& b, int f, int g_prev, int f_out, int v, float lambda, float eps2, int g,
                             float t0, float shrink, hipStream_t s)
{
    const int n = b.n_items[kShT16];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_tv_armijo, dim3(b.grid[kShT16]), dim3(256), 0, s, b.slices, b.items[kShT16], n, f, g_prev,
                       f_out, v, lambda, eps2, g, t0, shrink);
    return hipGetLastError();
}


// one block per slice
__global__ __launch_bounds__(kDecThreads) void kb_armijo_decide(const SliceDev* __restrict__ sl, int max_bt,
                                                                double c_arm, float t0, float shrink, int step, int T,
                                                                int fs, int gs, int vs, float lambda, float eps2)
{
    __shared__ DecShared S;
    const SliceDev& d = sl[blockIdx.x];
    armijo_decide_block(d.st, d.part[kPartGrad], d.part[kPartArm], d.t16x * d.t16y, max_bt, c_arm, t0, shrink,
                        d.st_k, d.st_q0, d.st_q1, step, T, d.buf[fs], d.buf[gs], d.buf[vs], d.buf[kBufWX],
                        d.buf[kBufWY], d.nx, d.ny, lambda, eps2, S);
}

hipError_t blaunch_armijo_decide(const BatchDev& b, int max_bt, double c_arm, float t0, float shrink, int step, int T,
                                 int f, int g, int v, float lambda, float eps2, hipStream_t s)
{
    hipLaunchKernelGGL(kb_armijo_decide, dim3(b.n), dim3(kDecThreads), 0, s, b.slices, max_bt, c_arm, t0, shrink,
                       step, T, f, g, v, lambda, eps2);
    return hipGetLastError();
}

// With `rmse`, a slice with a reference also gets its per-tile squared errors
// (as the one-slice update does), for the iteration's RMSE record.
__global__ __launch_bounds__(256) void kb_p2_update(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                    int n_items, int fcs, int gs, int fos, int fTs, int clamp,
                                                    int rmse)
{
    __shared__ float tl[32][33];
    __shared__ double lds[4];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        __syncthreads();
        p2_update_block(d.st, d.buf[fcs], d.buf[gs], d.buf[fos], bsel(d, fTs), clamp, d.nx, d.ny, w.y % d.t32x,
                        w.y / d.t32x, tl);
        if (rmse && d.buf[kBufFRef]) {  // uniform per item
            const double e2 = update_tile_sq_err(d.buf[fos], d.buf[kBufFRef], d.nx, d.ny, w.y % d.t32x,
                                                 w.y / d.t32x, lds);
            if (threadIdx.x == 0) d.part[kPartRmse][w.y] = e2;
        }
    }
}

hipError_t blaunch_p2_update(const BatchDev& b, int fcur, int g, int fout, int foutT, int clamp, int rmse,
                             hipStream_t s)
{
    const int n = b.n_items[kShT32];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_p2_update, dim3(b.grid[kShT32]), dim3(256), 0, s, b.slices, b.items[kShT32], n, fcur, g,
                       fout, foutT, clamp, rmse);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_copy_clamp(const SliceDev* __restrict__ sl, const int2* __restrict__ items,
                                                     int n_items, int srcs, int dsts, int dTs, int clamp)
{
    __shared__ float tl[32][33];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        __syncthreads();
        copy_clamp_block(d.buf[srcs], d.buf[dsts], bsel(d, dTs), clamp, d.nx, d.ny, w.y % d.t32x, w.y / d.t32x, tl);
    }
}

hipError_t blaunch_copy_clamp(const BatchDev& b, int src, int dst, int dstT, int clamp, hipStream_t s)
{
    const int n = b.n_items[kShT32];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_copy_clamp, dim3(b.grid[kShT32]), dim3(256), 0, s, b.slices, b.items[kShT32], n, src, dst,
                       dstT, clamp);
    return hipGetLastError();
}

}  // namespace eptv
