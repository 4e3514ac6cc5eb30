// batch.h -- device view of a batch of slices for the batched kernels.
//
// A batch runs the same EPTV iteration on many slices of different sizes,
// view and bin counts.  Every phase of the iteration is one launch for the
// whole batch: a persistent grid walks a work list of (slice, block) items,
// block meaning whatever the one-slice kernel of that phase calls a block (a
// 64-ray group of one view, a 16x16 or 32x32 pixel tile, a vector chunk, the
// single block of a scalar kernel).  Items are listed slice by slice and
// handed out round-robin, block b taking items b, b + G, b + 2G, ...; the
// per-block work is the one-slice kernel's own __device__ function, so a
// slice gets bit-for-bit the result it gets alone.
#pragma once

#include "eptv_internal.h"

namespace eptv {

// Buffers a batched call may name (per slice, bound before each run).
enum BufId : int {
    kBufF,     // the iterate f            [ny][nx]
    kBufFT,    // its transposed copy      [nx][ny]
    kBufU,     // CGLS iterate / v
    kBufS,     // CGLS direction
    kBufST,    // its transposed copy
    kBufZ,     // P^T r
    kBufG,     // P2 direction (ping)
    kBufG2,    // P2 direction (pong)
    kBufF1,    // P2 iterate (ping)
    kBufF2,    // P2 iterate (pong)
    kBufR,     // residual              [V][B]
    kBufQ,     // P s                   [V][B]
    kBufY,     // the sinogram y
    kBufFRef,  // reference image (RMSE), may be null
    kNumBufs
};

enum PartId : int { kPartProj, kPartBp, kPartP2, kPartRes, kPartRmse, kNumParts };

constexpr int kNoBuf = -1;

struct SliceDev {
    int nx, ny, V, B;
    int proj_gx;           // 64-bin ray groups per view
    int t16x, t16y;        // 16x16 tiles
    int t32x, t32y;        // 32x32 tiles
    int axpy_img, axpy_sino;
    int sel_blocks;
    long long n_edges;
    uint32_t rank;         // sigma's order-statistic rank for this slice
    const RayFx* rays;
    const int2* range;
    const int* list_off;
    const int* list;
    float* buf[kNumBufs];
    double* part[kNumParts];
    uint32_t* keys;
    uint32_t* hist;
    DevState* st;
    float* st_sigma;
    int32_t* st_k;
    int32_t* st_steps;
    double* st_resid;
    double* st_rmse;
    double* st_q0;
    double* st_q1;
    double* st_gamma;
    double* st_delta;
    int cgls_iters;        // M, the stride of st_gamma / st_delta
};

// Item lists, one per block shape.
enum Shape : int { kShProj, kShT16, kShT32, kShAxpy, kShSel, kShRmse, kShOne, kNumShapes };

struct BatchDev {
    const SliceDev* slices = nullptr;
    int n = 0;
    const int2* items[kNumShapes] = {};
    int n_items[kNumShapes] = {};
    int grid[kNumShapes] = {};  // persistent grid per shape (chosen by the tuner)
    int proj_seg = 16;          // projector sweep segments per block (chosen by the tuner)
};

__device__ __forceinline__ float* bsel(const SliceDev& d, int id) { return id >= 0 ? d.buf[id] : nullptr; }
__device__ __forceinline__ double* psel(const SliceDev& d, int id) { return id >= 0 ? d.part[id] : nullptr; }

// ---------------------------------------------------------------- batched launchers
hipError_t blaunch_project(const BatchDev& b, int x, int xT, float alpha, float beta, int c, int out, int part,
                           hipStream_t s);
hipError_t blaunch_backproject(const BatchDev& b, int r, float alpha, float beta, int c, int z, int zT, int part,
                               hipStream_t s);
hipError_t blaunch_cgls_axpy(const BatchDev& b, int m, int u_in, bool with_res, hipStream_t s);
hipError_t blaunch_cgls_supdate(const BatchDev& b, int m, hipStream_t s);
hipError_t blaunch_gd_p1(const BatchDev& b, float step, hipStream_t s);
hipError_t blaunch_edges_hist(const BatchDev& b, int img, float eps2, hipStream_t s);
hipError_t blaunch_select_hist(const BatchDev& b, int pass, hipStream_t s);
hipError_t blaunch_select_finalize(const BatchDev& b, int pass, float floor_, hipStream_t s);
// Descent step D.step + 1 (the previous step's decision read from the slice's
// state) and the last step's update; blaunch_p2_decide takes each decision,
// D carrying the constants (its pointers are each slice's own).
hipError_t blaunch_p2_step(const BatchDev& b, int f, int g_prev, int f_out, int v, float lambda, float eps2, int g,
                           float t0, float shrink, const P2Decide& D, hipStream_t s);
hipError_t blaunch_p2_final(const BatchDev& b, int fcur, int g, int fout, int foutT, int clamp, int rmse, int v,
                            float lambda, float eps2, const P2Decide& D, hipStream_t s);
// One block per slice: step D.step's decision into the slice's state.
hipError_t blaunch_p2_decide(const BatchDev& b, int f, int g, int v, float lambda, float eps2, const P2Decide& D,
                             hipStream_t s);
hipError_t blaunch_copy_clamp(const BatchDev& b, int src, int dst, int dstT, int clamp, hipStream_t s);
hipError_t blaunch_rmse_part(const BatchDev& b, int f, hipStream_t s);
hipError_t blaunch_iter_end(const BatchDev& b, bool with_resid, bool with_rmse, bool rmse_tiles, float sigma_fixed,
                            hipStream_t s);
hipError_t blaunch_state_init(const BatchDev& b, float sigma_fixed, int zero_iter, hipStream_t s);
hipError_t blaunch_transpose(const BatchDev& b, int src, int dst, hipStream_t s);
hipError_t blaunch_fill_zero(const BatchDev& b, int dst, hipStream_t s);

}  // namespace eptv
