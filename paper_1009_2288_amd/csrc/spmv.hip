// spmv.hip -- the stored system matrix: the paper's look-up-table strategy
// for P and P^T (Sec. 2.3), on MI355X.
//
// The float32 matrix is the one the on-the-fly kernels compute (every entry
// from cell_weights on the host, bit for bit), held twice: CSR by ray for P
// and CSC by pixel for P^T, so both products are gathers.  A nonzero costs 6
// bytes in the compact CSR encoding (float32 length, 16-bit index offset from
// its chunk's base) and 8 in the CSC copy (index and length, interleaved), so
// the kernels are bound by memory traffic: 81 + 109 MB per P / P^T call at
// 512^2 / 40 x 736 (13.4 M nonzeros), well inside HBM3E's 288 GB; both copies
// together (190 MB) fit the 256 MB Infinity Cache.  Rows and columns are
// padded to a multiple of 4 entries (0.3 % more entries for P, 3 % for P^T at
// that size).
//
// P:   one wave per ray; the ray's entries come in chunks of 128, chunk slot l
//      holding entries l and n/2 + l of a chunk of n, so each lane loads one
//      slot per chunk and each gather instruction reads n/2 consecutive
//      entries of the ray.  A ray swept row by row indexes the transposed
//      image, so consecutive entries of any ray lie mostly along the fast
//      axis: a gather touches a few cache lines, not one per lane, and a
//      chunk's indices span less than 64 image rows (hence the 16-bit offsets;
//      a geometry where some chunk spans more keeps 16-byte wide slots).  The
//      wave's ray index is uniform, so the ray's offsets (the top bit of the
//      first one flagging a row sweep) and each chunk's base come through
//      scalar loads.  A fixed grid of
//      (B/64) x V blocks of 16 waves loops over the rays, so the per-block
//      partials of ||q||^2 line up with the on-the-fly projector's.
// P^T: kCscLanes lanes per pixel (~52 entries), each lane 4 consecutive
//      entries (two 16-byte loads) per pass; a pixel's entries are rays of
//      the same views at neighbouring bins, so the gathers are local without
//      any reordering.  A fixed grid of one block per 16x16 image tile loops
//      over the pixels.
// Sums are per lane then a fixed lane pattern: deterministic.
#include "eptv_internal.h"
#include "reduce.h"
#include "state.h"

namespace eptv {

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

// v + v of another lane of the same 16-lane row, by a DPP lane pattern.
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float lane_value(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Sum over each aligned group of 4 lanes (partner 2 away, then 1 away; every
// lane of the group ends with the same bits), by DPP within the quad.
__device__ __forceinline__ float quad_sum(float v)
{
    v = dpp_add<0x4e>(v);  // quad_perm [2, 3, 0, 1]
    return dpp_add<0xb1>(v);  // quad_perm [1, 0, 3, 2]
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
// the group's partial sums meet in a fixed pattern (quad_sum).  Every lane of
// the group returns the sum.
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
    static_assert(L == 4, "the group sum is a quad's");
    return quad_sum(acc);
}

// Sum over the 64 lanes without the LDS crossbar: within each 16-lane row by
// DPP (neighbour in the pair, the other pair of the quad, the other quad of
// the 8 (mirror), the other 8 of the 16 (mirror); a + b and b + a agree, so
// every lane of a row holds the same bits), then the four rows' sums in a
// fixed order.
__device__ __forceinline__ float wave_sum64(float v)
{
    v = dpp_add<0xb1>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141>(v);  // row_half_mirror
    v = dpp_add<0x140>(v);  // row_mirror
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// The ray's scaled sum, the output (alpha P x + beta c) and its square:
// shared by both encodings' kernels.
__device__ __forceinline__ void csr_finish(float acc, int row, int lane, float alpha, float beta, float cv,
                                           float* q, double& s2)
{
    acc = wave_sum64(acc);
    float out = alpha * acc;
    if (beta != 0.0f) out = fmaf(beta, cv, out);
    if (lane == 0) q[row] = out;
    s2 += (double)out * (double)out;
}

__device__ __forceinline__ void csr_partial(double s2, int w, int lane, double* lds, double* partial)
{
    if (!partial) return;
    // every lane of a wave holds the same s2: take lane 0's
    if (lane == 0) lds[w] = s2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 16; ++i) t += lds[i];
        partial[blockIdx.x] = t;
    }
}

struct __attribute__((aligned(4))) Slot3 {
    int len0, len1;  // float bits of entries l and n/2 + l
    unsigned off;    // their index offsets from the chunk base, entry l in the low half
};

// P from the compact encoding: per chunk of n entries, n/2 12-byte slots then
// the base word; a lane takes one slot (entries l and n/2 + l).
// With fold.st set, block nblk (one past the projector's blocks) closes the
// previous outer iteration instead (see IterEnd).
__global__ __launch_bounds__(1024) void k_csr_compact(const int* __restrict__ wordptr, const int* __restrict__ words,
                                                      const float* __restrict__ x, const float* __restrict__ xT,
                                                      int nrows, float alpha, float beta, const float* c, float* q,
                                                      double* partial, IterEnd fold, int nblk)
{
    __shared__ double lds[16];
    if (fold.st && (int)blockIdx.x == nblk) {
        iter_end_run<1024>(fold, lds);
        return;
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    double s2 = 0.0;
    for (int row = blockIdx.x * 16 + w; row < nrows; row += nblk * 16) {
        const int r0 = wordptr[row], r1 = wordptr[row + 1];
        const float cv = beta != 0.0f ? c[row] : 0.0f;  // issued ahead of the entries
        const float* img = r0 < 0 ? xT : x;  // the layout the entries index
        const int w0 = r0 & 0x7fffffff, w1 = r1 & 0x7fffffff;
        float acc = 0.0f;
        for (int c0 = w0; c0 < w1; c0 += kChunkWords) {
            const int h = min(kStoredChunk / 2, (w1 - c0 - 1) / 3);  // slots in this chunk
            const int base = words[c0 + 3 * h];
            if (lane < h) {
                const Slot3 e = *reinterpret_cast<const Slot3*>(words + c0 + 3 * lane);
                const float x0 = img[base + (int)(e.off & 0xffffu)], x1 = img[base + (int)(e.off >> 16)];
                acc = fmaf(__int_as_float(e.len0), x0, acc);
                acc = fmaf(__int_as_float(e.len1), x1, acc);
            }
        }
        csr_finish(acc, row, lane, alpha, beta, cv, q, s2);
    }
    csr_partial(s2, w, lane, lds, partial);
}

// P from the wide encoding: 16-byte slots of two (index, length) pairs.
__global__ __launch_bounds__(1024) void k_csr_rows(const int* __restrict__ rowptr, const i32x4* __restrict__ ent,
                                                   const float* __restrict__ x, const float* __restrict__ xT,
                                                   int nrows, float alpha, float beta, const float* c, float* q,
                                                   double* partial, IterEnd fold, int nblk)
{
    __shared__ double lds[16];
    if (fold.st && (int)blockIdx.x == nblk) {
        iter_end_run<1024>(fold, lds);
        return;
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    double s2 = 0.0;
    for (int row = blockIdx.x * 16 + w; row < nrows; row += nblk * 16) {
        const int r0 = rowptr[row], r1 = rowptr[row + 1];
        const float cv = beta != 0.0f ? c[row] : 0.0f;
        const float* img = r0 < 0 ? xT : x;
        // slots (two entries each) of the row; both bounds are even
        const int e0 = (r0 & 0x7fffffff) >> 1, e1 = (r1 & 0x7fffffff) >> 1;
        float acc = 0.0f;
        for (int s = e0; s < e1; s += 64) {
            if (s + lane < e1) {
                const i32x4 a = ld_ent(ent + s + lane);
                const float x0 = img[a.x], x1 = img[a.z];
                acc = fmaf(__int_as_float(a.y), x0, acc);
                acc = fmaf(__int_as_float(a.w), x1, acc);
            }
        }
        csr_finish(acc, row, lane, alpha, beta, cv, q, s2);
    }
    csr_partial(s2, w, lane, lds, partial);
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
                                 const float* c, float* q, double* partial, hipStream_t s, const IterEnd* fold)
{
    const int nblk = project_blocks(p);
    const IterEnd fe = fold ? *fold : IterEnd();
    const dim3 grid((unsigned)(nblk + (fold ? 1 : 0)));
    if (p.mat.compact)
        hipLaunchKernelGGL(k_csr_compact, grid, dim3(1024), 0, s, p.mat.d_rowptr, p.mat.d_rwords, x, xT, p.V * p.B,
                           alpha, beta, c, q, partial, fe, nblk);
    else
        hipLaunchKernelGGL(k_csr_rows, grid, dim3(1024), 0, s, p.mat.d_rowptr, (const i32x4*)p.mat.d_rent, x, xT,
                           p.V * p.B, alpha, beta, c, q, partial, fe, nblk);
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
