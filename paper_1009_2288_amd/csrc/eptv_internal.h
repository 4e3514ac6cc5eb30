// eptv_internal.h -- plan layout, device state and kernel launchers of libeptv.
//
// Internal to the HIP library; the public contract is include/eptv.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/eptv.h"

namespace eptv {

// ---------------------------------------------------------------- rays
// Every ray is stored in "sweep form".  A ray that is closer to the x axis
// (|cos| >= |sin|) is swept column by column: in column k it enters at the
// continuous row coordinate e(k) = e0 + k*slope and leaves at e(k+1) (row
// units: 0 at the image bottom edge, 1 per pixel, |slope| <= 1).  A ray closer
// to the y axis is swept row by row with the roles of rows and columns
// exchanged.  Coordinates are 32.32 fixed point, so stepping along the ray is
// exact integer arithmetic and a crossing of a row boundary is located to
// ~1e-10 pixel however shallow the ray.  For cell k of the sweep,
//     lo(k) = lo0 + k*step  = min(E(k), E(k+1)),   hi(k) = lo(k) + span,
// span = |step|; the ray's length inside cross cell m of that sweep cell is
// given by cell_weights() below.  The projector and the backprojector both
// evaluate exactly that function, so their float32 matrices are transposes of
// each other bit for bit.
struct alignas(16) RayFx {
    long long lo0;   // lo(0)
    long long step;  // E(k+1) - E(k)
    long long span;  // |step| (0: the ray is parallel to the sweep axis)
    float w32;       // 2^-32 d/|sin| (d/|cos| for row sweeps): length per fixed-point unit crossed
    float wfull;     // d/|cos| (d/|sin|): length across a whole cell; < 0 marks a row sweep
};

struct RayTable {
    RayFx* d_ray = nullptr;    // [V*B]
    int2* d_range = nullptr;   // [V*B] sweep range [k_lo, k_hi) that can meet the image
    float2* d_view = nullptr;  // [V] (cos theta, sin theta)
    double2* d_view_d = nullptr; // [V] (cos theta, sin theta) in double
    double* d_tau = nullptr;   // [B+2] tan of the bin angles, bins -1 .. B
    int* d_list_off = nullptr; // [tiles+1] backprojector ray lists: offsets
    int* d_list = nullptr;     // ray ids v*B + b that can meet each 16x16 tile
};

// Lengths of a ray inside the (at most two) cross cells m0 and m0+1 of one
// sweep cell with lower/upper fixed-point bounds lo and lo + span:
//     span == 0:                 c0 = wfull,                         c1 = 0
//     floor(lo) == floor(hi):    c0 = (hi - lo) * w32,               c1 = 0
//     otherwise (floor(hi) = m0+1): c0 = (2^32 - frac(lo)) * w32,    c1 = frac(hi) * w32
// with every fixed-point length converted to float exactly once, so each entry
// carries a relative error of about 1e-7 however shallow the ray.
struct CellW {
    int m0;
    float c0, c1;
};

__host__ __device__ __forceinline__ CellW cell_weights(long long lo, long long span, float w32, float wfull)
{
    const long long hi = lo + span;
    const int m0 = (int)(lo >> 32), m1 = (int)(hi >> 32);
    const unsigned flo = (unsigned)lo, fhi = (unsigned)hi;
    const bool same = m0 == m1;
    CellW w;
    w.m0 = m0;
    // 2^32 - frac(lo) formed in integers (exact) before the one rounding to float
    const float rest = flo ? (float)(0u - flo) : 4294967296.0f;
    w.c0 = span == 0 ? wfull : (same ? (float)(fhi - flo) : rest) * w32;
    w.c1 = same ? 0.0f : (float)fhi * w32;
    return w;
}

// ---------------------------------------------------------------- device state
constexpr int kMaxCgls = 64;
constexpr int kSelectBins = 2048;  // 11-bit radix digits
constexpr int kArmijoFirst = 8;    // Armijo candidates k = 0..7, evaluated by the whole grid
constexpr int kArmijoMore = 16;    // candidates per round of the rare longer search
constexpr int kP2T = 32;            // P2 descent-step tiles: 32 x 32 pixels
constexpr int kP2Threads = kP2T * kP2T;  // one thread per pixel
constexpr int kP2Slots = 2 + kArmijoFirst;  // per-block partials of a step: Q, ||g||^2, trial energies

// Scalars that stay on the device.  Each entry is written by one kernel and
// read only by later kernels on the stream (never by the writer's own grid).
struct DevState {
    // P1 (CGLS): per-step entries, written by the step's vector kernels
    double gamma[kMaxCgls + 1];  // ||P^T r_m||^2
    double delta[kMaxCgls];      // ||P s_m||^2 of each step that formed it (0 after a breakdown)
    double gamma0;
    float a[kMaxCgls], b[kMaxCgls];
    int active[kMaxCgls];        // CGLS still running after step m
    int cg_steps;
    // sigma selection
    uint32_t prefix;
    uint32_t rank;               // rank still to find below the digits chosen so far
    uint32_t rank0;              // the order statistic's rank (set once per run)
    uint32_t sel_prefix[2], sel_rank[2];  // one-slice path: prefix and rank after digits 0 and 1
    float sigma;
    float inv_sigma2;
    // P2: a descent step's decision, when a kernel of its own takes it (batches)
    int k;
    float t;
    // bookkeeping
    int iter;
    int nonfinite;               // the input scan found NaN or inf
};

// What closes an outer iteration (records, counter, reset of the
// per-iteration state); run by k_iter_end, or by one extra block of the next
// iteration's first projector launch (st non-null there).
struct IterEnd {
    DevState* st = nullptr;
    const double* part_res = nullptr;   // ||r||^2 partials (with_resid)
    const double* part_rmse = nullptr;  // squared-error partials (with_rmse)
    int n_res = 0, with_resid = 0, n_rmse = 0, with_rmse = 0;
    double npix = 0.0;
    float* st_sigma = nullptr;
    int32_t* st_steps = nullptr;
    double *st_resid = nullptr, *st_rmse = nullptr, *st_gamma = nullptr, *st_delta = nullptr;
    int M = 0;  // CGLS steps per P1, whose gamma_m / delta_m go to st_gamma / st_delta ([K*M])
    uint32_t* hist = nullptr;
    float sigma_fixed = -1.0f;
};
struct Plan;
IterEnd iter_end_args(const Plan& p, DevState* st, const double* part_res, int with_resid, const double* part_rmse,
                      int n_rmse, int with_rmse, float* st_sigma, int32_t* st_steps, double* st_resid, double* st_rmse,
                      int M, double* st_gamma, double* st_delta, uint32_t* hist, float sigma_fixed);
// The float32 system matrix stored on the device (optional, see spmv.hip).
// Every row and column is padded to a multiple of kStoredPad entries with its
// last index and length 0.  The CSR copy (by ray) is split in chunks of
// kStoredChunk entries per ray (the last one shorter); within a chunk of n
// entries, slot l holds entries l and n/2 + l.  It has two encodings:
//  * compact (whenever every chunk's indices span at most 65535): a chunk is
//    n/2 slots of three 32-bit words (the two lengths' float bits, then the
//    two indices as 16-bit offsets from the chunk's smallest index, entry l in
//    the low half) followed by one word holding that smallest index, so a
//    full chunk is kChunkWords words and an entry costs 6 bytes;
//  * wide: slots of two (index, length bits) pairs, 16 bytes, 8 per entry.
// The CSC copy (by pixel) holds (ray index, length bits) pairs, entry order,
// so a lane's 4 entries are two aligned 16-byte loads.
constexpr int kStoredPad = 4;
constexpr int kStoredChunk = 128;
constexpr int kChunkWords = 3 * (kStoredChunk / 2) + 1;
struct StoredMatrix {
    long long nnz = 0;          // nonzeros, padding excluded
    long long slots = 0;        // entries per copy, padding included
    bool compact = false;       // the CSR copy's encoding
    int* d_rowptr = nullptr;    // [V*B + 1] CSR by ray: word offsets into d_rwords (compact) or
                                //  entry offsets into d_rent (wide); bit 31 set for a ray swept
                                //  row by row
    int* d_rwords = nullptr;    // compact CSR chunks (pixel index into x, or into x transposed
                                //  for rays swept row by row)
    int2* d_rent = nullptr;     // wide CSR slots: (index as above, length bits) pairs
    int* d_colptr = nullptr;    // [nx*ny + 1] CSC by pixel, offsets into d_cent
    int2* d_cent = nullptr;     // [slots of the CSC copy] (ray index, length)
    size_t bytes = 0;           // both copies with their offsets
    size_t csr_bytes = 0;       // the CSR copy with its offsets
};

struct Plan {
    int nx = 0, ny = 0, V = 0, B = 0;
    double pixel = 0, dbeta = 0, bin_offset = 0, sad = 0, sdd = 0;
    std::vector<double> angles;
    long long nnz = 0;
    int device = 0;
    RayTable rays;
    StoredMatrix mat;
    hipStream_t cap_stream = nullptr;
    // cached graph of one outer iteration
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> gkey;
    // and of an iteration with given (frozen) edge weights
    hipGraphExec_t gexec_w = nullptr;
    std::vector<uint64_t> gkey_w;
};

// The Armijo decision of one descent step, taken by the kernel after it.
struct P2Decide {
    const double* part;  // the step's partials [kP2Slots][blocks]; null: the decision is st->k, st->t
    int step, T;         // the step and the steps per P2 (record index iter * T + step)
    int max_bt;
    double c_arm;
    float t0, shrink;
    int replay;          // 1: the index comes from st_k
    int32_t* st_k;       // per-step records [K*T], may be null
    double* st_q0;
    double* st_q1;
};

// ---------------------------------------------------------------- workspace
struct Workspace {
    float* fT;      // transposed image for the projector [nx][ny]
    float* u;       // CGLS iterate / v
    float* s;       // CGLS direction
    float* sT;      // its transposed copy
    float* z;       // backprojection P^T r
    float* g;       // P2 direction (ping)
    float* g2;      // P2 direction (pong)
    float* f1;      // P2 iterate (ping)
    float* f2;      // P2 iterate (pong)
    float* r;       // CGLS residual [V][B]
    float* q;       // P s [V][B]
    uint32_t* keys; // edge magnitude bit patterns [n_edges]
    float* edge3;   // three values per half-edge [3][n_edges] (direction VJP)
    uint32_t* hist; // [3][kSelectBins]
    double* part_proj;  // ||P s||^2 per projector block
    double* part_bp;    // ||P^T r||^2 per backprojector block
    double* part_p2;    // descent-step partials, two by step parity: [2][kP2Slots][p2_blocks]
    double* part_res;   // ||r||^2 per sinogram block of the last CGLS axpy
    double* part_rmse;  // (f - f_ref)^2 per block
    DevState* st;
    float* st_sigma;     // [K]
    int32_t* st_k;       // [K*T]
    int32_t* st_steps;   // [K]
    double* st_resid;    // [K]
    double* st_rmse;     // [K]
    double* st_q0;       // [K*T] Armijo energy at each descent step's start
    double* st_q1;       // [K*T] and at the accepted point
    double* st_gamma;    // [K*M] CGLS gamma_m
    double* st_delta;    // [K*M] CGLS delta_m
    size_t bytes;
};

size_t workspace_layout(const Plan& p, int K, int T, int M, char* base, Workspace* w);

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return hipGetLastError().
int project_blocks(const Plan& p);
int image_tile_blocks(const Plan& p);
int sino_blocks(const Plan& p);
int select_blocks(const Plan& p);
constexpr int kRmseBlocks = 256;

// zero f and fT (zero != 0) or transpose f into fT, and reset the device state
// with the selection rank and the iteration counter (one launch)
hipError_t launch_recon_start(float* f, float* fT, int nx, int ny, int zero, DevState* st, uint32_t* hist,
                              uint32_t rank, float sigma_fixed, hipStream_t s);
hipError_t launch_transpose(const float* src, float* dst, int nx, int ny, hipStream_t s);
hipError_t launch_fill(float* dst, size_t n, float value, hipStream_t s);
hipError_t launch_project(const Plan& p, const float* x, const float* xT, float alpha, float beta,
                          const float* c, float* q, double* partial, hipStream_t s);
hipError_t launch_backproject(const Plan& p, const float* r, float alpha, float beta, const float* c,
                              float* z, float* zT, double* partial, hipStream_t s);
hipError_t launch_backproject_interp(const Plan& p, const float* r, float alpha, float beta, const float* c,
                                     float* z, float* zT, double* partial, hipStream_t s);

// fold: the previous outer iteration's closing, run by one extra block of
// this launch (null: none)
hipError_t launch_project_stored(const Plan& p, const float* x, const float* xT, float alpha, float beta, const float* c, float* q,
                                 double* partial, hipStream_t s, const IterEnd* fold = nullptr);
hipError_t launch_backproject_stored(const Plan& p, const float* r, float alpha, float beta, const float* c, float* z,
                                     float* zT, double* partial, hipStream_t s);

// CGLS (App. I): the vector kernels sum the partials of the operator call
// before them, so no separate scalar kernel is launched.
hipError_t launch_state_init(DevState* st, uint32_t* hist, uint32_t rank, float sigma_fixed,
                             int zero_iter, hipStream_t s);
hipError_t launch_cgls_axpy(const Plan& p, DevState* st, int m, const double* part_bp,
                            const double* part_proj, const float* u_in, float* u, const float* sdir,
                            float* r, const float* q, double* part_res, hipStream_t s);
hipError_t launch_cgls_supdate(const Plan& p, DevState* st, int m, const double* part_bp, const float* z,
                               float* sdir, float* sdirT, hipStream_t s);
hipError_t launch_gd_p1(const Plan& p, const float* f, const float* z, float step, float* u,
                        hipStream_t s);

// sigma: three histogram passes, each closed by a one-block kernel
hipError_t launch_edges_hist(const Plan& p, const float* f, float eps2, uint32_t* keys,
                             uint32_t* hist0, hipStream_t s);
// a CGLS step's update (as launch_cgls_axpy, u distinct from u_in) with the
// histogram of the resulting u's half-edges (as launch_edges_hist), one launch
hipError_t launch_cgls_axpy_edges(const Plan& p, DevState* st, int m, const double* part_bp,
                                  const double* part_proj, const float* u_in, float* u, const float* sdir, float* r,
                                  const float* q, double* part_res, float eps2, uint32_t* keys, uint32_t* hist0,
                                  hipStream_t s);
// pass 1 and 2 (each first closing the previous digit), then the last digit and sigma
hipError_t launch_select_pass(const Plan& p, int pass, const uint32_t* keys, DevState* st, uint32_t* hist,
                              hipStream_t s);
hipError_t launch_select_sigma(DevState* st, const uint32_t* hist, float sigma_floor, hipStream_t s);
hipError_t launch_sigma_out(const DevState* st, float* out, hipStream_t s);

// P2 (Sec. 2.2): the stand-alone direction, its VJP, the descent steps
hipError_t launch_tv_vjp(const Plan& p, const float* f, const float* u, float lambda, float sigma, float eps2,
                         float* e3, float* out, hipStream_t s);
// g = lambda (f - v) + A2 at f; sigma = inf gives w = 1; weights stored when
// wx / wy are given; partials (Q, ||g||^2) per 16x16 block when part is given
hipError_t launch_tv_grad(const Plan& p, const float* f, const float* v, float lambda, float sigma, float eps2,
                          float* g, float* wx, float* wy, double* part, hipStream_t s, const float* wx_in = nullptr,
                          const float* wy_in = nullptr);
// One kernel per descent step (32x32 tiles): the previous step's Armijo
// decision (D; D.part null for the first step), the iterate, the direction and
// this step's partials [kP2Slots][p2_blocks] (Q, ||g||^2, kArmijoFirst trial
// energies); then one kernel deciding and applying the last step, with
// positivity, the transposed copy and (with ref) one squared-error partial
// per tile in part_rmse.
int p2_blocks(const Plan& p);
int update_tiles(const Plan& p);
hipError_t launch_p2_step(const Plan& p, const float* f, const float* g_prev, float* f_out, const float* v,
                          float lambda, DevState* st, float eps2, float* g, double* part, float t0, float shrink,
                          const float* wx_in, const float* wy_in, const uint32_t* sel_hist, float sel_floor,
                          const P2Decide& D, hipStream_t s);
hipError_t launch_p2_final(const Plan& p, const float* fcur, const float* g, float* fout, float* foutT, int clamp,
                           const float* ref, double* part_rmse, const float* v, float lambda, const DevState* st,
                           float eps2, const float* wx_in, const float* wy_in, const P2Decide& D, hipStream_t s);
hipError_t launch_copy_clamp(const Plan& p, const float* src, float* dst, float* dstT, int clamp,
                             hipStream_t s);

// bookkeeping
hipError_t launch_rmse_part(const Plan& p, const float* f, const float* ref, double* part,
                            hipStream_t s);
hipError_t launch_iter_end(const IterEnd& e, hipStream_t s);
// st->nonfinite = whether a[0..n) holds NaN or inf (accumulate: or-ed into the
// flag of an earlier scan); one block, no other state touched
hipError_t launch_scan_finite(const float* a, size_t n, DevState* st, int accumulate, hipStream_t s);

}  // namespace eptv
