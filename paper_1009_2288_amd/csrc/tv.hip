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
#include "cgls_step.h"
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

// tv_edge's three differences (across the half-edge, and of the pair means on
// either side along it) are linear in the image, so for a trial point
// f - t g they are f's minus t times g's: one FMA each per candidate instead
// of forming the trial neighbourhood.
struct EdgeLin {
    float d, t1, t2;
};

__device__ __forceinline__ EdgeLin edge_lin(float a, float b, float au, float bu, float ad, float bd)
{
    const float m0 = 0.5f * (a + b), mu = 0.5f * (au + bu), md = 0.5f * (ad + bd);
    return {b - a, mu - m0, m0 - md};
}

// The owned half-edges of a pixel: right and up, and left / down on the
// image's first column / row.
struct EdgeSet {
    EdgeLin R, U, L, D;
};

__device__ __forceinline__ EdgeSet edge_set(const Nbhd& N, bool left, bool down)
{
    EdgeSet E;
    E.R = edge_lin(N.n[1][1], N.n[2][1], N.n[1][2], N.n[2][2], N.n[1][0], N.n[2][0]);
    E.U = edge_lin(N.n[1][1], N.n[1][2], N.n[2][1], N.n[2][2], N.n[0][1], N.n[0][2]);
    E.L = left ? edge_lin(N.n[0][1], N.n[1][1], N.n[0][2], N.n[1][2], N.n[0][0], N.n[1][0]) : EdgeLin{0.f, 0.f, 0.f};
    E.D = down ? edge_lin(N.n[1][0], N.n[1][1], N.n[2][0], N.n[2][1], N.n[0][0], N.n[0][1]) : EdgeLin{0.f, 0.f, 0.f};
    return E;
}

// Magnitude of a half-edge at f - t g from its terms in f (F) and g (G).
__device__ __forceinline__ float edge_at(const EdgeLin& F, const EdgeLin& G, float t, float e2)
{
    const float d = fmaf(-t, G.d, F.d), t1 = fmaf(-t, G.t1, F.t1), t2 = fmaf(-t, G.t2, F.t2);
    return hw_sqrt(d * d + 0.5f * (t1 * t1) + 0.5f * (t2 * t2) + e2);
}

// A pixel's share of Q(f - t g) (Eq. 8 with Eq. A3's magnitudes): its owned
// half-edges' weighted magnitudes (weights frozen) plus lambda/2 (f - t g - v)^2
// at the pixel; dv0 = f - v and g11 = g at the pixel.
__device__ __forceinline__ double trial_energy(const EdgeSet& F, const EdgeSet& G, float wR, float wU, float wL,
                                               float wD, bool left, bool down, float dv0, float g11, float t,
                                               float lambda, float e2)
{
    float s = wR * edge_at(F.R, G.R, t, e2) + wU * edge_at(F.U, G.U, t, e2);
    if (left) s += wL * edge_at(F.L, G.L, t, e2);
    if (down) s += wD * edge_at(F.D, G.D, t, e2);
    const float d = fmaf(-t, g11, dv0);
    return (double)s + 0.5 * (double)lambda * (double)d * (double)d;
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

// The image a half-edge pass reads: pixels in memory, or the pixels that the
// same launch's CGLS update is writing, u_in + a s, formed here again with the
// same FMA (so the same bits) from the step's unchanged inputs.  A pixel is
// loaded as it is stored (Raw) and turned into its value afterwards, so that
// loads can be in flight while a is still being formed.
struct StoredImage {
    const float* f;
    typedef float Raw;
    __device__ Raw load(size_t id) const { return f[id]; }
    __device__ float value(Raw r) const { return r; }
};
struct AxpyImage {
    const float* u_in;
    const float* s;
    float a;
    typedef float2 Raw;
    __device__ Raw load(size_t id) const { return make_float2(u_in[id], s[id]); }
    __device__ float value(Raw r) const { return fmaf(a, r.y, r.x); }
};

template <class Img>
using RawNbhd = typename Img::Raw[3][3];

__device__ __forceinline__ bool in_image(int nx, int ny, int i, int j)
{
    return i >= 0 && i < nx && j >= 0 && j < ny;
}

// Every load is made, at a position clamped into the image (nbhd_of zeroes
// what lies outside): conditional loads into zeroed registers make the
// compiler wait for all loads in flight before each one.
template <class Img>
__device__ __forceinline__ void load_raw(const Img& img, int nx, int ny, int i, int j, RawNbhd<Img>& R)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int ii = min(max(i + a - 1, 0), nx - 1), jj = min(max(j + b - 1, 0), ny - 1);
            R[a][b] = img.load((size_t)jj * nx + ii);
        }
}

// Pixels outside the image are zero.
template <class Img>
__device__ __forceinline__ void nbhd_of(const Img& img, int nx, int ny, int i, int j, const RawNbhd<Img>& R, Nbhd& N)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) N.n[a][b] = in_image(nx, ny, i + a - 1, j + b - 1) ? img.value(R[a][b]) : 0.0f;
}

// Edge index: x-edge (i+1/2, j) -> j*(nx+1) + i+1; y-edge (i, j+1/2) -> ny*(nx+1) + (j+1)*nx + i.
// Pixel (i, j)'s owned half-edge magnitudes into keys and the block's LDS
// histogram of their top 11 bits.
__device__ __forceinline__ void edges_pixel(const Nbhd& N, int nx, int ny, int i, int j, float eps2, uint32_t* keys,
                                            uint32_t* h)
{
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

// One 16x16 tile's half-edges, one pixel per thread.
template <class Img>
__device__ __forceinline__ void edges_tile(const Img& img, int nx, int ny, float eps2, uint32_t* keys, int bx, int by,
                                           uint32_t* h)
{
    const int i = bx * kT + (threadIdx.x & (kT - 1)), j = by * kT + threadIdx.x / kT;
    if (i < nx && j < ny) {
        RawNbhd<Img> R;
        load_raw(img, nx, ny, i, j, R);
        Nbhd N;
        nbhd_of(img, nx, ny, i, j, R, N);
        edges_pixel(N, nx, ny, i, j, eps2, keys, h);
    }
}

// A block's tiles first, first + stride, ... of the image, kEdgeGroup at a
// time: the group's neighbourhoods are all loaded before any is used (a
// block per CU would otherwise wait out one load round trip per tile).
// `ready` runs once, after the first group's loads are issued, by every
// thread of the block (it may hold barriers; AxpyImage forms a there).
constexpr int kEdgeGroup = 4;

template <class Img, class Ready>
__device__ __forceinline__ void edges_walk(Img& img, int nx, int ny, float eps2, uint32_t* keys, int first, int stride,
                                           uint32_t* h, Ready&& ready)
{
    const int tx = (nx + kT - 1) / kT, nt = tx * ((ny + kT - 1) / kT);
    const int li = threadIdx.x & (kT - 1), lj = threadIdx.x / kT;
    bool pending = true;
    for (int t0 = first; t0 < nt; t0 += kEdgeGroup * stride) {
        RawNbhd<Img> R[kEdgeGroup];
#pragma unroll
        for (int g = 0; g < kEdgeGroup; ++g) {  // (past the last tile or the image: a clamped position)
            const int t = min(t0 + g * stride, nt - 1);
            const int i = min((t % tx) * kT + li, nx - 1), j = min((t / tx) * kT + lj, ny - 1);
            load_raw(img, nx, ny, i, j, R[g]);
        }
        if (pending) {
            ready();
            pending = false;
        }
#pragma unroll
        for (int g = 0; g < kEdgeGroup; ++g) {
            const int t = t0 + g * stride;
            const int i = (t % tx) * kT + li, j = (t / tx) * kT + lj;
            if (t < nt && i < nx && j < ny) {
                Nbhd N;
                nbhd_of(img, nx, ny, i, j, R[g], N);
                edges_pixel(N, nx, ny, i, j, eps2, keys, h);
            }
        }
    }
    if (pending) ready();
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
    hist_clear(h);
    StoredImage img{f};
    edges_walk(img, nx, ny, eps2, keys, blockIdx.x, gridDim.x, h, [] {});
    hist_flush(h, hist0);
}

constexpr int kEdgesHistBlocks = 256;

static int edges_hist_blocks(const Plan& p)
{
    const int nt = ((p.nx + kT - 1) / kT) * ((p.ny + kT - 1) / kT);
    return std::min(nt, kEdgesHistBlocks);
}

hipError_t launch_edges_hist(const Plan& p, const float* f, float eps2, uint32_t* keys, uint32_t* hist0,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_edges_hist, dim3((unsigned)edges_hist_blocks(p)), dim3(256), 0, s, f, p.nx, p.ny, eps2,
                       keys, hist0);
    return hipGetLastError();
}

// The last CGLS step's update (u = u_in + a s written to u, r -= a q) and the
// half-edge histogram of that u, one launch: the first blocks are the
// histogram's (k_edges_hist's walk over the tiles), forming the pixels they
// read from u_in and s with the update's own FMA, so they never read what
// the update blocks are writing; u must not alias u_in.
__global__ __launch_bounds__(kAxpyBlock) void k_cgls_axpy_edges(
    DevState* st, int m, const double* part_bp, int n_bp, const double* part_proj, int n_proj, size_t n_img,
    size_t n_sino, int img_blocks, const float* __restrict__ u_in, float* __restrict__ u,
    const float* __restrict__ sdir, float* r, const float* q, double* part_res, int edge_blocks, int nx, int ny,
    float eps2, uint32_t* keys, uint32_t* hist0)
{
    __shared__ double lds[4];
    __shared__ uint32_t h[kSelectBins];
    const int blk = (int)blockIdx.x - edge_blocks;
    if (blk >= 0) {
        cgls_axpy_block(st, m, part_bp, n_bp, part_proj, n_proj, n_img, n_sino, img_blocks, u_in, u, sdir, r, q,
                        part_res, blk, lds);
        return;
    }
    AxpyImage img{u_in, sdir, 0.0f};
    hist_clear(h);
    edges_walk(img, nx, ny, eps2, keys, blockIdx.x, edge_blocks, h,
               [&] { img.a = cgls_step_a(st, m, part_bp, n_bp, part_proj, n_proj, false, lds); });
    hist_flush(h, hist0);
}

hipError_t launch_cgls_axpy_edges(const Plan& p, DevState* st, int m, const double* part_bp,
                                  const double* part_proj, const float* u_in, float* u, const float* sdir, float* r,
                                  const float* q, double* part_res, float eps2, uint32_t* keys, uint32_t* hist0,
                                  hipStream_t s)
{
    if (u == u_in) return hipErrorInvalidValue;
    const size_t ni = (size_t)p.nx * p.ny, ns = (size_t)p.V * p.B;
    const int bi = axpy_blocks(ni), bs = axpy_blocks(ns), be = edges_hist_blocks(p);
    hipLaunchKernelGGL(k_cgls_axpy_edges, dim3(be + bi + bs), dim3(kAxpyBlock), 0, s, st, m, part_bp,
                       image_tile_blocks(p), part_proj, project_blocks(p), ni, ns, bi, u_in, u, sdir, r, q, part_res,
                       be, p.nx, p.ny, eps2, keys, hist0);
    return hipGetLastError();
}

// The keys a thread takes in a grid-stride walk are loaded kSelGroup at a
// time, unconditionally (past the end: the last key, not counted), so that
// they are all in flight together.
constexpr int kSelGroup = 8;

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
    const size_t stride = (size_t)nblk * 256;
    for (size_t e0 = (size_t)blk * 256 + threadIdx.x; e0 < n; e0 += kSelGroup * stride) {
        uint32_t k[kSelGroup];
#pragma unroll
        for (int g = 0; g < kSelGroup; ++g) k[g] = keys[min(e0 + g * stride, n - 1)];
#pragma unroll
        for (int g = 0; g < kSelGroup; ++g)
            if (e0 + g * stride < n && (k[g] >> hshift) == want) hist_add(h, (k[g] >> dshift) & dmask);
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
    // threads 0..255 take part; wider blocks only join the barriers
    uint32_t* sums = S.sums;
    const int nb = pass == 2 ? 1024 : 2048;
    const int per = nb / 256;
    const int t = threadIdx.x;
    const bool act = t < 256;
    if (act) {
        uint32_t local = 0;
        for (int e = 0; e < per; ++e) local += hist[t * per + e];
        sums[t] = local;
    }
    if (t == 0) {  // only kept if the rank exceeded the count, which cannot happen
        S.found_digit = (uint32_t)(nb - 1);
        S.found_before = 0u;
    }
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t add = act && t >= o ? sums[t - o] : 0u;
        __syncthreads();
        if (act) sums[t] += add;
        __syncthreads();
    }
    if (act) {
        const uint32_t before_group = t ? sums[t - 1] : 0u;
        if (before_group <= rank && rank < sums[t]) {
            uint32_t before = before_group;
            int d = t * per;
            while (d < t * per + per - 1 && before + hist[d] <= rank) before += hist[d++];
            S.found_digit = (uint32_t)d;
            S.found_before = before;
        }
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
// (the first group of keys is loaded before the block closes the previous digit)

__global__ __launch_bounds__(256) void k_select_pass(const uint32_t* __restrict__ keys, size_t n, int pass,
                                                     DevState* st, uint32_t* hist)
{
    __shared__ uint32_t h[kSelectBins];
    __shared__ SelShared S;
    for (int b = threadIdx.x; b < kSelectBins; b += 256) h[b] = 0u;  // ordered by select_digit's barriers
    const size_t stride = (size_t)gridDim.x * 256;
    uint32_t k[kSelGroup];
    auto load = [&](size_t e0) {
#pragma unroll
        for (int g = 0; g < kSelGroup; ++g) k[g] = keys[min(e0 + g * stride, n - 1)];
    };
    size_t e0 = (size_t)blockIdx.x * 256 + threadIdx.x;
    load(e0);
    const uint32_t pin = pass == 1 ? st->prefix : st->sel_prefix[0];
    const uint32_t rin = pass == 1 ? st->rank : st->sel_rank[0];
    select_digit(hist + (pass - 1) * kSelectBins, pass - 1, rin, S);
    const uint32_t pout = pin | (S.found_digit << digit_shift(pass - 1));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->sel_prefix[pass - 1] = pout;
        st->sel_rank[pass - 1] = rin - S.found_before;
    }
    // pass 1: digit = bits 20..10 among keys whose bits 31..21 equal the
    // prefix; pass 2: digit = bits 9..0 among keys whose bits 31..10 do
    const int hshift = pass == 1 ? 21 : 10;
    const int dshift = pass == 1 ? 10 : 0;
    const uint32_t dmask = pass == 1 ? 2047u : 1023u;
    const uint32_t want = pout >> hshift;
    for (;;) {
#pragma unroll
        for (int g = 0; g < kSelGroup; ++g)
            if (e0 + g * stride < n && (k[g] >> hshift) == want) hist_add(h, (k[g] >> dshift) & dmask);
        e0 += kSelGroup * stride;
        if (e0 >= n) break;
        load(e0);
    }
    __syncthreads();
    uint32_t* hp = hist + pass * kSelectBins;
    for (int b = threadIdx.x; b < kSelectBins; b += 256)
        if (h[b]) atomicAdd(&hp[b], h[b]);
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

// g = lambda (f - v) + A2 at f, with Eq. 5's weights at f (inv_s2 = 1/sigma^2,
// 0 for sigma = inf) or the given ones; the weights are stored when wx / wy
// are given.  Per-block partials (Q(f) = sum of w TV over owned edges +
// lambda/2 (f - v)^2, ||g||^2) when `part` is given.
__device__ __forceinline__ void tv_grad_block(const float* __restrict__ f, const float* __restrict__ v, int nx, int ny,
                                              float lambda, float inv_s2, float eps2, float* __restrict__ g,
                                              float* wx, float* wy, double* part, int bx, int by, int b, int nb,
                                              double* lds, const float* wx_in = nullptr,
                                              const float* wy_in = nullptr)
{
    const int i = bx * kT + (threadIdx.x & (kT - 1)), j = by * kT + threadIdx.x / kT;
    double q = 0.0, gg = 0.0;
    if (i < nx && j < ny) {
        Nbhd N;
        load_nbhd(f, nx, ny, i, j, N);
        const float c = N.n[1][1];
        const float tR = tv_right(N, eps2), tL = tv_left(N, eps2), tU = tv_up(N, eps2), tD = tv_down(N, eps2);
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
        if (wx) {
            wx[xw + i + 1] = wR;
            if (i == 0) wx[xw] = wL;
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

__global__ __launch_bounds__(256) void k_tv_grad(const float* __restrict__ f, const float* __restrict__ v, int nx,
                                                 int ny, float lambda, float inv_s2, float eps2,
                                                 float* __restrict__ g, float* wx, float* wy, double* part,
                                                 const float* wx_in, const float* wy_in)
{
    __shared__ double lds[4];
    tv_grad_block(f, v, nx, ny, lambda, inv_s2, eps2, g, wx, wy, part, blockIdx.x, blockIdx.y,
                  blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y, lds, wx_in, wy_in);
}

hipError_t launch_tv_grad(const Plan& p, const float* f, const float* v, float lambda, float sigma, float eps2,
                          float* g, float* wx, float* wy, double* part, hipStream_t s, const float* wx_in,
                          const float* wy_in)
{
    const float inv_s2 = (sigma > 0.0f && std::isfinite(sigma)) ? 1.0f / (sigma * sigma) : 0.0f;
    dim3 grid((p.nx + kT - 1) / kT, (p.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_tv_grad, grid, dim3(256), 0, s, f, v, p.nx, p.ny, lambda, inv_s2, eps2, g, wx, wy, part,
                       wx_in, wy_in);
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
// frozen at f: Eq. 5's, recomputed from f with the direction kernel's own
// operations (so equal to the ones it used), or the given ones.
template <int NC>
__device__ __forceinline__ void candidate_energies(const float* f, const float* g, const float* v, const float* wx_in,
                                                   const float* wy_in, float inv_s2, int nx, int ny, int i, int j,
                                                   float lambda, float eps2, float t0, float shrink, int k0, double* e)
{
    Nbhd F, G;
    load_nbhd(f, nx, ny, i, j, F);
    load_nbhd(g, nx, ny, i, j, G);
    const size_t xo = (size_t)j * (nx + 1);
    float wR, wU, wL = 0.0f, wD = 0.0f;
    if (wx_in) {
        wR = wx_in[xo + i + 1];
        wU = wy_in[(size_t)(j + 1) * nx + i];
        if (i == 0) wL = wx_in[xo];
        if (j == 0) wD = wy_in[i];
    } else {
        wR = weight(tv_right(F, eps2), inv_s2);
        wU = weight(tv_up(F, eps2), inv_s2);
        if (i == 0) wL = weight(tv_left(F, eps2), inv_s2);
        if (j == 0) wD = weight(tv_down(F, eps2), inv_s2);
    }
    const float dv0 = F.n[1][1] - v[(size_t)j * nx + i];
    const EdgeSet EF = edge_set(F, i == 0, j == 0), EG = edge_set(G, i == 0, j == 0);
    float t = cand_t(t0, shrink, k0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        e[c] += trial_energy(EF, EG, wR, wU, wL, wD, i == 0, j == 0, dv0, G.n[1][1], t, lambda, eps2);
        t *= shrink;
    }
}

// ------------------------------------------------------------------ descent steps of P2 (Sec. 2.2)
// One kernel per descent step, on 32x32 tiles with one thread per own pixel.
// Step s's kernel
//  * takes the Armijo decision of step s-1 itself, from that step's per-block
//    partials: every block sums them in the same fixed order and so reaches
//    the same decision, and no kernel of its own is launched for it (the
//    slice's first block records it);
//  * forms the iterate f_s = f_{s-1} - t g_{s-1} (f_0: the start image) on its
//    tile plus a 2-pixel halo in LDS, and the direction g_s = lambda (f_s - v)
//    + A2 (Eq. 9-10, App. II A2-A3) with Eq. 5's weights at f_s on the tile
//    plus a 1-pixel halo (halo values recomputed with the same operations as
//    in their owning block, so they are bit-identical);
//  * writes step s's partials: Q(f_s), ||g_s||^2 and the energies
//    Q(f_s - t_k g_s) of the first kArmijoFirst candidates with the weights
//    frozen at f_s, each summed over the block in a fixed order.
// A last kernel decides step T-1 and applies it, with the positivity
// truncation (step 3 of the algorithm) and the transposed copy.  The
// partials are double-buffered by step parity: step s reads step s-1's
// while writing its own.
constexpr int kP2Waves = kP2Threads / 64;
constexpr int kP2Win = kP2T + 4;           // iterate window: 2-pixel halo
constexpr int kP2Dir = kP2T + 2;           // direction window: 1-pixel halo
constexpr int kP2Halo = 4 * kP2Dir - 4;    // direction positions on the halo ring
constexpr int kRedVals = kArmijoMore > kP2Slots ? kArmijoMore : kP2Slots;

int p2_blocks(const Plan& p) { return ((p.nx + kP2T - 1) / kP2T) * ((p.ny + kP2T - 1) / kP2T); }
int update_tiles(const Plan& p) { return p2_blocks(p); }

// Block sums of NV values per thread over NT threads in a fixed order (each
// wave's butterfly, then the waves in order), in R.tot for every thread.
// Contains __syncthreads().
struct RedShared {
    double red[kP2Waves][kRedVals];
    double tot[kRedVals];
};

template <int NT, int NV>
__device__ __forceinline__ void block_sums(const double* v, RedShared& R)
{
    static_assert(NT % 64 == 0 && NT <= kP2Threads && NV <= kRedVals, "reduction shape");
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        const double s = wave_sum(v[c]);
        if (l == 0) R.red[w][c] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) a += R.red[q][threadIdx.x];
        R.tot[threadIdx.x] = a;
    }
    __syncthreads();
}

struct DecShared {
    RedShared R;
    double q_acc;  // the energy at the accepted point
    int verdict;
};

// Block sums of kP2Slots values per thread of a kP2Threads block in a fixed
// order: each thread stores its values in v[c][tid] (threads past the first
// 64 nw store nothing and count as zeros), then lane l of wave c sums slot
// c's entries l, l + 64, ... in order and wave c closes slot c by DPP lane
// patterns (wave_sum_dpp).
struct SlotSums {
    double v[kP2Slots][kP2Threads];
    double tot[kP2Slots];
};

template <int CTRL>
__device__ __forceinline__ double dpp_add_d(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return v + __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value_d(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the 64 lanes by DPP lane patterns within each 16-lane row, then
// the four rows in a fixed order (every lane gets the same bits).
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v = dpp_add_d<0xb1>(v);
    v = dpp_add_d<0x4e>(v);
    v = dpp_add_d<0x141>(v);
    v = dpp_add_d<0x140>(v);
    return (lane_value_d(v, 0) + lane_value_d(v, 16)) + (lane_value_d(v, 32) + lane_value_d(v, 48));
}

// The sums of the values stored in L.v by the first 64 nw threads, in L.tot
// for every thread.  Contains __syncthreads() before and after.
__device__ __forceinline__ void slot_sums_stored(SlotSums& L, int nw = kP2Threads / 64)
{
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (w < kP2Slots) {
        double a = 0.0;
        for (int q = 0; q < nw; ++q) a += L.v[w][l + 64 * q];
        a = wave_sum_dpp(a);
        if (l == 0) L.tot[w] = a;
    }
    __syncthreads();
}

struct P2Shared {
    float f[kP2Win][kP2Win];  // the iterate, tile + 2-pixel halo (the final kernel: the transposition tile)
    float g[kP2Dir][kP2Dir];  // the direction, tile + 1-pixel halo
    SlotSums sums;            // the decision's sums, then the step's partials (written as they are formed)
    DecShared dec;
    SelShared sel;
};

// The Armijo decision of descent step D.step (Sec. 2.2): the first candidate
// t_k = t0 shrink^k, k <= max_bt, with Q_k <= Q0 - c t_k ||g||^2, from that
// step's partials (nb blocks).  Should none of the fused candidates pass
// while more backtracks are allowed (a reasonable t0 never needs it), the
// block goes on through the whole image, kArmijoMore candidates at a time
// (slow, the same decision); without an accepted candidate the step is
// skipped (k = -1, t = 0).  With D.replay the index is the recorded one.
// `record`: this block writes the step's records (index, Q0, Q at the
// accepted point; a replayed index past the fused candidates has its energy
// evaluated for the record).  f, g: the step's iterate and direction.  A
// block of kP2Threads threads sums the partials through L (LDS it may share
// with data it has not stored yet), a narrower one through S.R.
template <int NT>
__device__ __forceinline__ void p2_decide(const P2Decide& D, int nb, const DevState* st, bool record,
                                          const float* f, const float* g, const float* v, const float* wx_in,
                                          const float* wy_in, float inv_s2, int nx, int ny, float lambda, float eps2,
                                          DecShared& S, SlotSums* L, int& k_out, float& t_out)
{
    double a[kP2Slots];
#pragma unroll
    for (int c = 0; c < kP2Slots; ++c) a[c] = 0.0;
    for (int b = threadIdx.x; b < nb; b += NT) {
#pragma unroll
        for (int c = 0; c < kP2Slots; ++c) a[c] += D.part[(size_t)c * nb + b];
    }
    const double* tot;
    if constexpr (NT == kP2Threads) {
        // only the first ceil(nb / 64) waves hold partials: the others' zeros
        // are left out of the sums (adding them would not change a bit)
        const int nw = (nb < NT ? nb + 63 : NT) / 64;
        if ((int)threadIdx.x < 64 * nw) {
#pragma unroll
            for (int c = 0; c < kP2Slots; ++c) L->v[c][threadIdx.x] = a[c];
        }
        slot_sums_stored(*L, nw);
        tot = L->tot;
    } else {
        block_sums<NT, kP2Slots>(a, S.R);
        tot = S.R.tot;
    }
    const double q0 = tot[0], g2 = tot[1];
    const size_t rec = (size_t)st->iter * D.T + D.step;
    if (threadIdx.x < 64) {
        // candidate k tested by lane k; the first that passes is accepted
        const int k = threadIdx.x;
        const bool pass = !D.replay && k < kArmijoFirst && k <= D.max_bt &&
                          tot[2 + (k < kArmijoFirst ? k : 0)] <=
                              q0 - D.c_arm * (double)cand_t(D.t0, D.shrink, k < kArmijoFirst ? k : 0) * g2;
        const unsigned long long mask = __ballot(pass);
        if (threadIdx.x == 0) {
            // the caller's decision for this step (-1: no step), or the search's
            const int kk = D.replay ? D.st_k[rec] : (mask ? __ffsll((long long)mask) - 1 : -1);
            S.verdict = kk;
            S.q_acc = kk < 0 ? q0 : (kk < kArmijoFirst ? tot[2 + kk] : 0.0);
        }
    }
    __syncthreads();
    int kk = S.verdict;
    if (D.replay && kk >= kArmijoFirst && record) {
        double e[kArmijoMore];
#pragma unroll
        for (int c = 0; c < kArmijoMore; ++c) e[c] = 0.0;
        for (int px = threadIdx.x; px < nx * ny; px += NT)
            candidate_energies<kArmijoMore>(f, g, v, wx_in, wy_in, inv_s2, nx, ny, px % nx, px / nx, lambda, eps2,
                                            D.t0, D.shrink, kk, e);
        block_sums<NT, kArmijoMore>(e, S.R);
        if (threadIdx.x == 0) S.q_acc = S.R.tot[0];
        __syncthreads();
    }
    for (int k0 = kArmijoFirst; !D.replay && kk < 0 && k0 <= D.max_bt; k0 += kArmijoMore) {
        double e[kArmijoMore];
#pragma unroll
        for (int c = 0; c < kArmijoMore; ++c) e[c] = 0.0;
        for (int px = threadIdx.x; px < nx * ny; px += NT)
            candidate_energies<kArmijoMore>(f, g, v, wx_in, wy_in, inv_s2, nx, ny, px % nx, px / nx, lambda, eps2,
                                            D.t0, D.shrink, k0, e);
        block_sums<NT, kArmijoMore>(e, S.R);
        if (threadIdx.x == 0) {
            int found = -1;
            for (int c = 0; c < kArmijoMore && k0 + c <= D.max_bt; ++c)
                if (S.R.tot[c] <= q0 - D.c_arm * (double)cand_t(D.t0, D.shrink, k0 + c) * g2) {
                    found = k0 + c;
                    S.q_acc = S.R.tot[c];
                    break;
                }
            S.verdict = found;
        }
        __syncthreads();
        kk = S.verdict;
    }
    if (record && threadIdx.x == 0) {
        if (D.st_k) D.st_k[rec] = kk;
        if (D.st_q0) D.st_q0[rec] = q0;
        if (D.st_q1) D.st_q1[rec] = S.q_acc;
    }
    k_out = kk;
    t_out = kk >= 0 ? cand_t(D.t0, D.shrink, kk) : 0.0f;
    __syncthreads();
}

// The direction g at window position (li, lj) of the 1-pixel-halo window
// (pixel (i0 - 1 + li, j0 - 1 + lj)), from the iterate window in LDS: Eq. A3's
// magnitudes of the pixel's four half-edges, Eq. 5's weights (or the given
// ones), the A2 fluxes and lambda (f - v); vpix is v at the pixel.
struct DirOut {
    float g, wR, wL, wU, wD, tR, tL, tU, tD, dv;
};

__device__ __forceinline__ DirOut p2_direction_at(const P2Shared& S, int li, int lj, int gi, int gj, int nx,
                                                  float vpix, float lambda, float eps2, float inv_s2,
                                                  const float* wx_in, const float* wy_in)
{
    Nbhd N;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) N.n[a][bb] = S.f[lj + bb][li + a];
    DirOut o;
    const float c = N.n[1][1];
    o.tR = tv_right(N, eps2);
    o.tL = tv_left(N, eps2);
    o.tU = tv_up(N, eps2);
    o.tD = tv_down(N, eps2);
    const size_t xw = (size_t)gj * (nx + 1);
    o.wR = wx_in ? wx_in[xw + gi + 1] : weight(o.tR, inv_s2);
    o.wL = wx_in ? wx_in[xw + gi] : weight(o.tL, inv_s2);
    o.wU = wy_in ? wy_in[(size_t)(gj + 1) * nx + gi] : weight(o.tU, inv_s2);
    o.wD = wy_in ? wy_in[(size_t)gj * nx + gi] : weight(o.tD, inv_s2);
    const float FR = o.wR * (N.n[2][1] - c) * hw_rcp(o.tR);
    const float FL = o.wL * (c - N.n[0][1]) * hw_rcp(o.tL);
    const float FU = o.wU * (N.n[1][2] - c) * hw_rcp(o.tU);
    const float FD = o.wD * (c - N.n[1][0]) * hw_rcp(o.tD);
    o.dv = c - vpix;
    o.g = lambda * o.dv - (FR - FL) - (FU - FD);
    return o;
}

// Descent step `step` on tile (bx, by) = block b of nb (see above); with D.part
// null the previous step's decision is read from st (a batch decides each
// slice's step in a kernel of its own, one block per slice).  f: the
// previous iterate f_{s-1} (g_prev its direction, null for step 0, when f is
// the start image); f_out receives f_s for s > 0.  sel_hist: the first step of
// an adaptive iteration closes sigma's last digit from that histogram (the
// same computation in every block; block 0 records it), else sigma is st's.
__device__ __forceinline__ void p2_step_block(const float* __restrict__ f, const float* __restrict__ g_prev,
                                              float* __restrict__ f_out, const float* __restrict__ v, int nx, int ny,
                                              float lambda, DevState* st, float eps2, float* __restrict__ g,
                                              double* part, float t0, float shrink, int bx, int by, int b, int nb,
                                              P2Shared& S, const float* wx_in, const float* wy_in,
                                              const uint32_t* sel_hist, float sel_floor, const P2Decide& D)
{
    const int tid = threadIdx.x;
    const int i0 = bx * kP2T, j0 = by * kP2T;
    constexpr int kWin = kP2Win * kP2Win;
    constexpr int kWinPer = (kWin + kP2Threads - 1) / kP2Threads;
    const int ti = tid & (kP2T - 1), tj = tid / kP2T;
    const int i = i0 + ti, j = j0 + tj;
    const bool own = i < nx && j < ny;
    // this thread's position on the direction window's halo ring (tid < kP2Halo)
    int li = 0, lj = 0;
    if (tid < kP2Dir) {
        li = tid;
    } else if (tid < 2 * kP2Dir) {
        li = tid - kP2Dir;
        lj = kP2Dir - 1;
    } else if (tid < 2 * kP2Dir + kP2T) {
        lj = tid - 2 * kP2Dir + 1;
    } else {
        li = kP2Dir - 1;
        lj = tid - 2 * kP2Dir - kP2T + 1;
    }
    const int hi = i0 - 1 + li, hj = j0 - 1 + lj;
    const bool ring = tid < kP2Halo && (unsigned)hi < (unsigned)nx && (unsigned)hj < (unsigned)ny;
    // the window's and v's loads first, so they overlap sigma's digit and the decision
    float fv[kWinPer], gv[kWinPer];
#pragma unroll
    for (int u = 0; u < kWinPer; ++u) {
        const int idx = tid + kP2Threads * u;
        fv[u] = 0.0f;
        gv[u] = 0.0f;
        if (idx < kWin) {
            const int gi = i0 - 2 + idx % kP2Win, gj = j0 - 2 + idx / kP2Win;
            if ((unsigned)gi < (unsigned)nx && (unsigned)gj < (unsigned)ny) {
                const size_t id = (size_t)gj * nx + gi;
                fv[u] = f[id];
                if (g_prev) gv[u] = g_prev[id];
            }
        }
    }
    float inv_s2;
    if (sel_hist) {
        const uint32_t rin = st->sel_rank[1];
        select_digit(sel_hist, 2, rin, S.sel);
        const uint32_t prefix = st->sel_prefix[1] | S.sel.found_digit;
        const float sg = fmaxf(__uint_as_float(prefix), sel_floor);
        inv_s2 = 1.0f / (sg * sg);
        if (b == 0 && tid == 0) {
            st->prefix = prefix;
            st->rank = rin - S.sel.found_before;
            st->sigma = sg;
            st->inv_sigma2 = inv_s2;
        }
    } else {
        inv_s2 = st->inv_sigma2;
    }
    int kp = -1;
    float tp = 0.0f;
    if (g_prev) {
        if (D.part) {
            p2_decide<kP2Threads>(D, nb, st, b == 0, f, g_prev, v, wx_in, wy_in, inv_s2, nx, ny, lambda, eps2, S.dec,
                                  &S.sums, kp, tp);
        } else {  // taken by a kernel of its own
            kp = st->k;
            tp = st->t;
        }
    }
#pragma unroll
    for (int u = 0; u < kWinPer; ++u) {
        const int idx = tid + kP2Threads * u;
        if (idx < kWin) S.f[idx / kP2Win][idx % kP2Win] = g_prev ? stepped(fv[u], gv[u], kp, tp) : fv[u];
    }
    __syncthreads();
    // the own pixel's direction (its weights and terms kept for the trials)
    DirOut o{};
    if (own) {
        o = p2_direction_at(S, ti + 1, tj + 1, i, j, nx, v[(size_t)j * nx + i], lambda, eps2, inv_s2, wx_in, wy_in);
        const size_t id = (size_t)j * nx + i;
        g[id] = o.g;
        if (g_prev) f_out[id] = S.f[tj + 2][ti + 2];
    }
    S.g[tj + 1][ti + 1] = own ? o.g : 0.0f;
    // the halo ring of the direction window
    if (tid < kP2Halo)
        S.g[lj][li] = ring ? p2_direction_at(S, li, lj, hi, hj, nx, v[(size_t)hj * nx + hi], lambda, eps2, inv_s2, wx_in, wy_in).g
                           : 0.0f;
    __syncthreads();
    // this step's partials: Q(f_s), ||g_s||^2 and the trial energies, the
    // trials as candidate_energies with the weights frozen at f_s, each
    // stored to LDS as it is formed
    double (*val)[kP2Threads] = S.sums.v;
    if (!own) {
#pragma unroll
        for (int c = 0; c < kP2Slots; ++c) val[c][tid] = 0.0;
    } else {
        float e = o.wR * o.tR + o.wU * o.tU;
        if (i == 0) e += o.wL * o.tL;
        if (j == 0) e += o.wD * o.tD;
        val[0][tid] = (double)e + 0.5 * (double)lambda * (double)o.dv * (double)o.dv;
        val[1][tid] = (double)o.g * (double)o.g;
        Nbhd F, G;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                F.n[a][bb] = S.f[tj + 1 + bb][ti + 1 + a];
                G.n[a][bb] = S.g[tj + bb][ti + a];
            }
        const EdgeSet EF = edge_set(F, i == 0, j == 0), EG = edge_set(G, i == 0, j == 0);
        const float g11 = G.n[1][1];
        float t = t0;
#pragma unroll
        for (int c = 0; c < kArmijoFirst; ++c) {
            val[2 + c][tid] = trial_energy(EF, EG, o.wR, o.wU, o.wL, o.wD, i == 0, j == 0, o.dv, g11, t, lambda, eps2);
            t *= shrink;
        }
    }
    slot_sums_stored(S.sums);
    if (tid < kP2Slots) part[(size_t)tid * nb + b] = S.sums.tot[tid];
}

// The last descent step's decision and update: f_out = f - t g (f unchanged
// when the step was skipped), truncated at zero with `clamp`, its transposed
// copy (foutT, for the projector) and, with a reference, the squared error of
// the tile's new pixels (part_rmse[b], for the iteration's RMSE record).
__device__ __forceinline__ void p2_final_block(const float* __restrict__ fcur, const float* __restrict__ g,
                                               float* fout, float* foutT, int clamp, const float* ref,
                                               double* part_rmse, const float* __restrict__ v, int nx, int ny,
                                               float lambda, const DevState* st, float eps2, int bx, int by, int b,
                                               int nb, P2Shared& S, const float* wx_in, const float* wy_in,
                                               const P2Decide& D)
{
    const int tid = threadIdx.x;
    const int ti = tid & (kP2T - 1), tj = tid / kP2T;
    const int i0 = bx * kP2T, j0 = by * kP2T;
    const int i = i0 + ti, j = j0 + tj;
    const bool own = i < nx && j < ny;
    const size_t id = (size_t)j * nx + i;
    float fv = 0.0f, gv = 0.0f, rv = 0.0f;
    if (own) {
        fv = fcur[id];
        gv = g[id];
        if (ref) rv = ref[id];
    }
    int k = st->k;
    float t = st->t;
    if (D.part)
        p2_decide<kP2Threads>(D, nb, st, b == 0, fcur, g, v, wx_in, wy_in, st->inv_sigma2, nx, ny, lambda, eps2,
                              S.dec, &S.sums, k, t);
    float val = 0.0f;
    if (own) {
        val = stepped(fv, gv, k, t);
        if (clamp) val = fmaxf(val, 0.0f);
        fout[id] = val;
    }
    if (foutT) {
        S.f[tj][ti] = val;
        __syncthreads();
        const int it = i0 + tj, jt = j0 + ti;
        if (it < nx && jt < ny) foutT[(size_t)it * ny + jt] = S.f[ti][tj];
    }
    if (ref) {
        double e2[1] = {0.0};
        if (own) {
            const double d = (double)val - (double)rv;
            e2[0] = d * d;
        }
        block_sums<kP2Threads, 1>(e2, S.dec.R);
        if (tid == 0) part_rmse[b] = S.dec.R.tot[0];
    }
}

__global__ __launch_bounds__(kP2Threads) void k_p2_step(const float* __restrict__ f, const float* __restrict__ g_prev,
                                                        float* __restrict__ f_out, const float* __restrict__ v,
                                                        int nx, int ny, float lambda, DevState* st, float eps2,
                                                        float* __restrict__ g, double* part, float t0, float shrink,
                                                        const float* wx_in, const float* wy_in,
                                                        const uint32_t* sel_hist, float sel_floor, P2Decide D)
{
    __shared__ P2Shared S;
    p2_step_block(f, g_prev, f_out, v, nx, ny, lambda, st, eps2, g, part, t0, shrink, blockIdx.x, blockIdx.y,
                  blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y, S, wx_in, wy_in, sel_hist, sel_floor,
                  D);
}

hipError_t launch_p2_step(const Plan& p, const float* f, const float* g_prev, float* f_out, const float* v,
                          float lambda, DevState* st, float eps2, float* g, double* part, float t0, float shrink,
                          const float* wx_in, const float* wy_in, const uint32_t* sel_hist, float sel_floor,
                          const P2Decide& D, hipStream_t s)
{
    dim3 grid((p.nx + kP2T - 1) / kP2T, (p.ny + kP2T - 1) / kP2T);
    hipLaunchKernelGGL(k_p2_step, grid, dim3(kP2Threads), 0, s, f, g_prev, f_out, v, p.nx, p.ny, lambda, st, eps2, g,
                       part, t0, shrink, wx_in, wy_in, sel_hist, sel_floor, D);
    return hipGetLastError();
}

__global__ __launch_bounds__(kP2Threads) void k_p2_final(const float* __restrict__ fcur, const float* __restrict__ g,
                                                         float* fout, float* foutT, int clamp, const float* ref,
                                                         double* part_rmse, const float* __restrict__ v, int nx,
                                                         int ny, float lambda, const DevState* st, float eps2,
                                                         const float* wx_in, const float* wy_in, P2Decide D)
{
    __shared__ P2Shared S;
    p2_final_block(fcur, g, fout, foutT, clamp, ref, part_rmse, v, nx, ny, lambda, st, eps2, blockIdx.x, blockIdx.y,
                   blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y, S, wx_in, wy_in, D);
}

hipError_t launch_p2_final(const Plan& p, const float* fcur, const float* g, float* fout, float* foutT, int clamp,
                           const float* ref, double* part_rmse, const float* v, float lambda, const DevState* st,
                           float eps2, const float* wx_in, const float* wy_in, const P2Decide& D, hipStream_t s)
{
    dim3 grid((p.nx + kP2T - 1) / kP2T, (p.ny + kP2T - 1) / kP2T);
    hipLaunchKernelGGL(k_p2_final, grid, dim3(kP2Threads), 0, s, fcur, g, fout, foutT, clamp, ref, part_rmse, v, p.nx,
                       p.ny, lambda, st, eps2, wx_in, wy_in, D);
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
        edges_tile(StoredImage{d.buf[imgs]}, d.nx, d.ny, eps2, d.keys, w.y % d.t16x, w.y / d.t16x, h);
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

// The per-slice decision of a descent step: the batch-wide constants of D
// with this slice's partials (by step parity) and records.
__device__ __forceinline__ P2Decide slice_decision(const P2Decide& D, const SliceDev& d)
{
    P2Decide s = D;
    s.part = d.part[kPartP2] + (size_t)(D.step & 1) * kP2Slots * (d.t32x * d.t32y);
    s.st_k = d.st_k;
    s.st_q0 = d.st_q0;
    s.st_q1 = d.st_q1;
    return s;
}

// One block per slice: descent step D.step's decision, into the slice's
// state for the kernel after it (the one-slice kernels take it themselves in
// every block; here every tile item would repeat it).
__global__ __launch_bounds__(256) void kb_p2_decide(const SliceDev* __restrict__ sl, int fs, int gs, int vs,
                                                    float lambda, float eps2, P2Decide D)
{
    __shared__ DecShared S;
    const SliceDev& d = sl[blockIdx.x];
    int k;
    float t;
    p2_decide<256>(slice_decision(D, d), d.t32x * d.t32y, d.st, true, d.buf[fs], d.buf[gs], d.buf[vs], nullptr,
                   nullptr, d.st->inv_sigma2, d.nx, d.ny, lambda, eps2, S, nullptr, k, t);
    if (threadIdx.x == 0) {
        d.st->k = k;
        d.st->t = t;
    }
}

hipError_t blaunch_p2_decide(const BatchDev& b, int f, int g, int v, float lambda, float eps2, const P2Decide& D,
                             hipStream_t s)
{
    hipLaunchKernelGGL(kb_p2_decide, dim3(b.n), dim3(256), 0, s, b.slices, f, g, v, lambda, eps2, D);
    return hipGetLastError();
}

// step D.step + 1; its predecessor's decision is the slice's state
__global__ __launch_bounds__(kP2Threads) void kb_p2_step(const SliceDev* __restrict__ sl,
                                                         const int2* __restrict__ items, int n_items, int fs, int gps,
                                                         int fos, int vs, float lambda, float eps2, int gs, float t0,
                                                         float shrink, P2Decide D)
{
    __shared__ P2Shared S;
    const int step = D.step + 1;
    D.part = nullptr;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        const int nb = d.t32x * d.t32y;
        __syncthreads();
        p2_step_block(d.buf[fs], bsel(d, gps), bsel(d, fos), d.buf[vs], d.nx, d.ny, lambda, d.st, eps2, d.buf[gs],
                      d.part[kPartP2] + (size_t)(step & 1) * kP2Slots * nb, t0, shrink, w.y % d.t32x, w.y / d.t32x,
                      w.y, nb, S, nullptr, nullptr, nullptr, 0.0f, D);
    }
}

static int p2_grid(const BatchDev& b) { return std::max(1, std::min(b.n_items[kShT32], 2 * 256)); }

hipError_t blaunch_p2_step(const BatchDev& b, int f, int g_prev, int f_out, int v, float lambda, float eps2, int g,
                           float t0, float shrink, const P2Decide& D, hipStream_t s)
{
    const int n = b.n_items[kShT32];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_p2_step, dim3(p2_grid(b)), dim3(kP2Threads), 0, s, b.slices, b.items[kShT32], n, f, g_prev,
                       f_out, v, lambda, eps2, g, t0, shrink, D);
    return hipGetLastError();
}

// The last step's update with the decision in the slice's state.  With
// `rmse`, a slice with a reference also gets its per-tile squared errors (as
// the one-slice update does), for the iteration's RMSE record.
__global__ __launch_bounds__(kP2Threads) void kb_p2_final(const SliceDev* __restrict__ sl,
                                                          const int2* __restrict__ items, int n_items, int fcs,
                                                          int gs, int fos, int fTs, int clamp, int rmse, int vs,
                                                          float lambda, float eps2, P2Decide D)
{
    __shared__ P2Shared S;
    D.part = nullptr;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const SliceDev& d = sl[w.x];
        const float* ref = rmse ? d.buf[kBufFRef] : nullptr;
        __syncthreads();
        p2_final_block(d.buf[fcs], d.buf[gs], d.buf[fos], bsel(d, fTs), clamp, ref, d.part[kPartRmse], d.buf[vs],
                       d.nx, d.ny, lambda, d.st, eps2, w.y % d.t32x, w.y / d.t32x, w.y, d.t32x * d.t32y, S, nullptr,
                       nullptr, D);
    }
}

hipError_t blaunch_p2_final(const BatchDev& b, int fcur, int g, int fout, int foutT, int clamp, int rmse, int v,
                            float lambda, float eps2, const P2Decide& D, hipStream_t s)
{
    const int n = b.n_items[kShT32];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_p2_final, dim3(p2_grid(b)), dim3(kP2Threads), 0, s, b.slices, b.items[kShT32], n, fcur, g,
                       fout, foutT, clamp, rmse, v, lambda, eps2, D);
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
