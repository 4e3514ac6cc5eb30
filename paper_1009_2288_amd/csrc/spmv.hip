// spmv.hip -- the stored system matrix: the paper's look-up-table strategy
// for P and P^T (Sec. 2.3), on MI355X.
//
// The float32 matrix is the one the on-the-fly kernels compute (every entry
// from cell_weights on the host, bit for bit), held twice: CSR by ray for P
// and CSC by pixel for P^T, so both products are gathers.  Each nonzero costs
// 8 bytes (index and length, interleaved) per product, so the kernels are
// HBM-bound: 108 MB per call at 512^2 / 40 x 736 (13.4 M nonzeros), well
// inside HBM3E's 288 GB; both copies together (219 MB) fit the 256 MB
// Infinity Cache.  Rows and columns are padded to a multiple of 4 entries
// (0.3 % more entries for P, 3 % for P^T at that size).
//
// P:   one wave per ray; the ray's entries come in chunks of 128 stored as
//      64 16-byte slots, slot l of a chunk of n holding entries l and n/2 + l,
//      so each lane loads one slot per chunk and each gather instruction
//      reads n/2 consecutive entries of the ray.  A ray swept row by row
//      indexes the transposed image, so consecutive entries of any ray lie
//      mostly along the fast axis: a gather touches a few cache lines, not
//      one per lane.  A fixed grid of (B/64) x V blocks of 16 waves loops
//      over the rays, so the per-block partials of ||q||^2 line up with the
//      on-the-fly projector's.
// P^T: kCscLanes lanes per pixel (~52 entries), each lane 4 consecutive
//      entries (two 16-byte loads) per pass; a pixel's entries are rays of
//      the same views at neighbouring bins, so the gathers are local without
//      any reordering.  A fixed grid of one block per 16x16 image tile loops
//      over the pixels.
// Sums are per lane then a fixed butterfly: deterministic.
#include "eptv_internal.h"
#include "reduce.h"

namespace eptv {

#ifndef EPTV_CSR_PASSES
#define EPTV_CSR_PASSES 1
#endif
#ifndef EPTV_CSC_LANES
#define EPTV_CSC_LANES 4
#endif
#ifndef EPTV_CSC_PASSES
#define EPTV_CSC_PASSES 2
#endif
#ifndef EPTV_CSC_THREADS
#define EPTV_CSC_THREADS 1024
#endif
#ifndef EPTV_SPMV_NT
#define EPTV_SPMV_NT 0
#endif
constexpr int kCsrPasses = EPTV_CSR_PASSES;   // 128-entry chunks whose loads are in flight together
constexpr int kCscLanes = EPTV_CSC_LANES;     // lanes per pixel
constexpr int kCscPasses = EPTV_CSC_PASSES;
constexpr int kCscThreads = EPTV_CSC_THREADS; // threads per block
static_assert(kStoredPad == 4, "P^T: a lane takes 4 entries (two 16-byte loads); P: chunks of even length");
static_assert(kStoredChunk == 128, "P: a wave's 64 lanes take one 16-byte slot of a chunk each");

typedef int i32x4 __attribute__((ext_vector_type(4)));  // two entries (index, length bits)

__device__ __forceinline__ i32x4 ld_ent(const i32x4* p)
{
#if EPTV_SPMV_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

__device__ __forceinline__ float sub_sum(float v, int width)
{
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
    return v;
}

// sum of length * vec[index] over the 4 entries in a and b
__device__ __forceinline__ float dot4(const i32x4& a, const i32x4& b, const float* __restrict__ vec, float acc)
{
    const float x0 = vec[a.x], x1 = vec[a.z], x2 = vec[b.x], x3 = vec[b.z];
    acc = fmaf(__int_as_float(a.y), x0, acc);
    acc = fmaf(__int_as_float(a.w), x1, acc);
    acc = fmaf(__int_as_float(b.y), x2, acc);
    return fmaf(__int_as_float(b.w), x3, acc);
}

// Dot product of one padded row [e0, e1) (in units of two entries; both even)
// with vec, by a group of L lanes (lane = 0..L-1): each lane takes 4 entries
// per pass, the loads of PASSES passes are issued before their gathers, and
// the group's partial sums meet in a fixed butterfly.  Every lane of the
// group returns the sum.
template <int L, int PASSES>
__device__ __forceinline__ float row_dot(const i32x4* __restrict__ ent, int e0, int e1, int lane,
                                         const float* __restrict__ vec)
{
    float acc = 0.0f;
    for (int e = e0 + 2 * lane; e < e1; e += 2 * L * PASSES) {
        i32x4 a[PASSES], b[PASSES];
#pragma unroll
        for (int u = 0; u < PASSES; ++u)
            if (e + 2 * L * u < e1) {
                a[u] = ld_ent(ent + e + 2 * L * u);
                b[u] = ld_ent(ent + e + 2 * L * u + 1);
            }
#pragma unroll
        for (int u = 0; u < PASSES; ++u)
            if (e + 2 * L * u < e1) acc = dot4(a[u], b[u], vec, acc);
    }
    return sub_sum(acc, L);
}

// P: one wave per ray.  The ray's entries are stored in chunks of 128 (the
// last one shorter); within a chunk of n entries, 16-byte slot l holds entries
// l and n/2 + l, so one load per lane brings two entries and each gather
// instruction reads n/2 consecutive entries of the ray (a few cache lines).
__global__ __launch_bounds__(1024) void k_csr_rows(const int* __restrict__ rowptr, const i32x4* __restrict__ ent,
                                                   const RayFx* __restrict__ rays, const float* __restrict__ x,
                                                   const float* __restrict__ xT, int nrows, float alpha, float beta,
                                                   const float* c, float* q, double* partial)
{
    __shared__ double lds[16];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double s2 = 0.0;
    for (int row = blockIdx.x * 16 + w; row < nrows; row += gridDim.x * 16) {
        const float* img = rays[row].wfull < 0.0f ? xT : x;  // the layout the entries index
        // slots (two entries each) of the row; both bounds are even
        const int e0 = rowptr[row] >> 1, e1 = rowptr[row + 1] >> 1;
        float acc = 0.0f;
        for (int s = e0; s < e1; s += 64 * kCsrPasses) {
            i32x4 a[kCsrPasses];
#pragma unroll
            for (int u = 0; u < kCsrPasses; ++u)
                if (s + 64 * u + lane < e1) a[u] = ld_ent(ent + s + 64 * u + lane);
#pragma unroll
            for (int u = 0; u < kCsrPasses; ++u)
                if (s + 64 * u + lane < e1) {
                    const float x0 = img[a[u].x], x1 = img[a[u].z];
                    acc = fmaf(__int_as_float(a[u].y), x0, acc);
                    acc = fmaf(__int_as_float(a[u].w), x1, acc);
                }
        }
        acc = sub_sum(acc, 64);
        float out = alpha * acc;
        if (beta != 0.0f) out = fmaf(beta, c[row], out);
        if (lane == 0) q[row] = out;
        s2 += (double)out * (double)out;
    }
    if (partial) {
        // every lane of a wave holds the same s2: take lane 0's
        if (lane == 0) lds[w] = s2;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < 16; ++i) t += lds[i];
            partial[blockIdx.x] = t;
        }
    }
}

__global__ __launch_bounds__(kCscThreads) void k_csc_cols(const int* __restrict__ colptr,
                                                          const i32x4* __restrict__ ent,
                                                          const float* __restrict__ r, int nx, int ny, float alpha,
                                                          float beta, const float* c, float* z, float* zT,
                                                          double* partial)
{
    constexpr int kGroups = kCscThreads / kCscLanes;
    __shared__ double lds[kGroups];
    const int g = threadIdx.x / kCscLanes, lane = threadIdx.x % kCscLanes;
    const int npix = nx * ny;
    double s2 = 0.0;
    for (int pix = blockIdx.x * kGroups + g; pix < npix; pix += gridDim.x * kGroups) {
        const float acc = row_dot<kCscLanes, kCscPasses>(ent, colptr[pix] >> 1, colptr[pix + 1] >> 1, lane, r);
        float out = alpha * acc;
        if (beta != 0.0f) out = fmaf(beta, c[pix], out);
        if (lane == 0) {
            z[pix] = out;
            if (zT) zT[(size_t)(pix % nx) * ny + pix / nx] = out;
        }
        s2 += (double)out * (double)out;
    }
    if (partial) {
        if (lane == 0) lds[g] = s2;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < kGroups; ++i) t += lds[i];
            partial[blockIdx.x] = t;
        }
    }
}

hipError_t launch_project_stored(const Plan& p, const float* x, const float* xT, float alpha, float beta,
                                 const float* c, float* q, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_csr_rows, dim3(project_blocks(p)), dim3(1024), 0, s, p.mat.d_rowptr,
                       (const i32x4*)p.mat.d_rent, p.rays.d_ray, x, xT, p.V * p.B, alpha, beta, c, q, partial);
    return hipGetLastError();
}

hipError_t launch_backproject_stored(const Plan& p, const float* r, float alpha, float beta, const float* c, float* z,
                                     float* zT, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_csc_cols, dim3(image_tile_blocks(p)), dim3(kCscThreads), 0, s, p.mat.d_colptr,
                       (const i32x4*)p.mat.d_cent, r, p.nx, p.ny, alpha, beta, c, z, zT, partial);
    return hipGetLastError();
}

}  // namespace eptv
