// spmv.hip -- the stored system matrix: the paper's look-up-table strategy
// for P and P^T (Sec. 2.3), on MI355X.
//
// The float32 matrix is the one the on-the-fly kernels compute (every entry
// from cell_weights on the host, bit for bit), held twice: CSR by ray for P
// and CSC by pixel for P^T, so both products are gathers.  Each nonzero costs
// 8 bytes (length + index) per product, so the kernels are HBM-bound:
// 107 MB per call at 512^2 / 40 x 736 (13.4 M nonzeros), well inside HBM3E's
// 288 GB and close to the 256 MB Infinity Cache for both matrices together.
//
// P:   one wave per ray (64 lanes over its ~460 entries), a fixed grid of
//      (B/64) x V blocks of 16 waves looping over the rays, so the per-block
//      partials of ||q||^2 line up with the on-the-fly projector's.
// P^T: 16 lanes per pixel (~50 entries), 16 pixels per 256-thread block per
//      trip, a fixed grid of one block per 16x16 image tile.
// Sums are per lane then a fixed butterfly: deterministic.
#include "eptv_internal.h"
#include "reduce.h"

namespace eptv {

__device__ __forceinline__ float sub_sum(float v, int width)
{
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
    return v;
}

__global__ __launch_bounds__(1024) void k_csr_rows(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                   const float* __restrict__ val, const float* __restrict__ x,
                                                   int nrows, float alpha, float beta, const float* c, float* q,
                                                   double* partial)
{
    __shared__ double lds[16];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double s2 = 0.0;
    for (int row = blockIdx.x * 16 + w; row < nrows; row += gridDim.x * 16) {
        const int e0 = rowptr[row], e1 = rowptr[row + 1];
        float acc = 0.0f;
        for (int e = e0 + lane; e < e1; e += 64) acc = fmaf(val[e], x[col[e]], acc);
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

__global__ __launch_bounds__(256) void k_csc_cols(const int* __restrict__ colptr, const int* __restrict__ rowi,
                                                  const float* __restrict__ val, const float* __restrict__ r, int nx,
                                                  int ny, float alpha, float beta, const float* c, float* z, float* zT,
                                                  double* partial)
{
    __shared__ double lds[16];
    const int g = threadIdx.x >> 4, lane = threadIdx.x & 15;
    const int npix = nx * ny;
    double s2 = 0.0;
    for (int pix = blockIdx.x * 16 + g; pix < npix; pix += gridDim.x * 16) {
        const int e0 = colptr[pix], e1 = colptr[pix + 1];
        float acc = 0.0f;
        for (int e = e0 + lane; e < e1; e += 16) acc = fmaf(val[e], r[rowi[e]], acc);
        acc = sub_sum(acc, 16);
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
            for (int i = 0; i < 16; ++i) t += lds[i];
            partial[blockIdx.x] = t;
        }
    }
}

hipError_t launch_project_stored(const Plan& p, const float* x, float alpha, float beta, const float* c, float* q,
                                 double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_csr_rows, dim3(project_blocks(p)), dim3(1024), 0, s, p.mat.d_rowptr, p.mat.d_col,
                       p.mat.d_val, x, p.V * p.B, alpha, beta, c, q, partial);
    return hipGetLastError();
}

hipError_t launch_backproject_stored(const Plan& p, const float* r, float alpha, float beta, const float* c, float* z,
                                     float* zT, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_csc_cols, dim3(image_tile_blocks(p)), dim3(256), 0, s, p.mat.d_colptr, p.mat.d_row,
                       p.mat.d_cval, r, p.nx, p.ny, alpha, beta, c, z, zT, partial);
    return hipGetLastError();
}

}  // namespace eptv
