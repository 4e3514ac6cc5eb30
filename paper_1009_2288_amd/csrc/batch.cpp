// batch.cpp -- host side of the batched EPTV iteration (eptv_batch_* of
// eptv.h): one plan per slice, the (slice, block) work lists of every block
// shape, the per-slice device descriptors, the tuner that picks the launch
// shapes, and the outer loop (each iteration of the whole batch launched
// phase by phase, or replayed from one captured graph with EPTV_GRAPH=1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "batch.h"
#include "eptv_internal.h"
#include "host_internal.h"

namespace eptv {

int axpy_blocks(size_t n);
int select_blocks(const Plan& p);

static constexpr int kCUs = 256;  // MI355X compute units

}  // namespace eptv

struct eptv_batch_s {
    std::vector<eptv_plan> plans;
    eptv::BatchDev bd;
    eptv::SliceDev* d_slices = nullptr;
    eptv::SliceDev* h_stage = nullptr;  // pinned staging for the descriptor upload
    hipEvent_t staged = nullptr;         // the last upload has been consumed
    int2* d_items[eptv::kNumShapes] = {};
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> gkey;
    std::mutex mu;
};

namespace eptv {

static int tiles(int n, int t) { return (n + t - 1) / t; }

// Per-slice block counts and the fixed (workspace-independent) descriptor fields.
static SliceDev slice_shape(const Plan& p)
{
    SliceDev d{};
    d.nx = p.nx;
    d.ny = p.ny;
    d.V = p.V;
    d.B = p.B;
    d.proj_gx = tiles(p.B, 64);
    d.t16x = tiles(p.nx, 16);
    d.t16y = tiles(p.ny, 16);
    d.t32x = tiles(p.nx, 32);
    d.t32y = tiles(p.ny, 32);
    d.axpy_img = axpy_blocks((size_t)p.nx * p.ny);
    d.axpy_sino = axpy_blocks((size_t)p.V * p.B);
    d.sel_blocks = select_blocks(p);
    d.n_edges = (long long)n_edges(p);
    d.rays = p.rays.d_ray;
    d.range = p.rays.d_range;
    d.list_off = p.rays.d_list_off;
    d.list = p.rays.d_list;
    return d;
}

static int items_of(const SliceDev& d, int shape)
{
    switch (shape) {
    case kShProj: return d.proj_gx * d.V;
    case kShT16: return d.t16x * d.t16y;
    case kShT32: return d.t32x * d.t32y;
    case kShAxpy: return d.axpy_img + d.axpy_sino;
    case kShSel: return d.sel_blocks;
    case kShRmse: return kRmseBlocks;
    default: return 1;
    }
}

// Default persistent grids: enough blocks for every CU several times over,
// never more than there are items.
static int default_grid(int shape, int n_items)
{
    const int per_cu = shape == kShProj ? 2 : 8;
    return std::max(1, std::min(n_items, per_cu * kCUs));
}

static size_t batch_ws_layout(const eptv_batch_s& b, int K, int T, int M, char* base, std::vector<Workspace>* Ws)
{
    size_t off = 0;
    if (Ws) Ws->resize(b.plans.size());
    for (size_t i = 0; i < b.plans.size(); ++i) {
        Workspace W;
        const size_t need = workspace_layout(b.plans[i]->p, K, T, M, base ? base + off : nullptr, &W);
        if (Ws) (*Ws)[i] = W;
        off += (need + 255) & ~(size_t)255;
    }
    return off;
}

// Fill the per-slice descriptors for one run and upload them.
static int bind_batch(eptv_batch_s& b, const eptv_params& q, const std::vector<Workspace>& Ws, const float* const* y,
                      float* const* f, const float* const* f_ref, hipStream_t s)
{
    EPTV_HIP(hipEventSynchronize(b.staged));  // the previous upload has left the staging buffer
    for (int i = 0; i < b.bd.n; ++i) {
        const Plan& p = b.plans[i]->p;
        const Workspace& W = Ws[i];
        SliceDev d = slice_shape(p);
        d.rank = select_rank(p, q.edge_quantile);
        float* bufs[kNumBufs] = {f[i], W.fT, W.u,  W.s,  W.sT, W.z, W.g, W.g2, W.f1, W.f2, W.r, W.q,
                                 (float*)y[i], f_ref ? (float*)f_ref[i] : nullptr};
        std::memcpy(d.buf, bufs, sizeof bufs);
        double* parts[kNumParts] = {W.part_proj, W.part_bp, W.part_p2, W.part_res, W.part_rmse};
        std::memcpy(d.part, parts, sizeof parts);
        d.keys = W.keys;
        d.hist = W.hist;
        d.st = W.st;
        d.st_sigma = W.st_sigma;
        d.st_k = W.st_k;
        d.st_steps = W.st_steps;
        d.st_resid = W.st_resid;
        d.st_rmse = W.st_rmse;
        d.st_q0 = W.st_q0;
        d.st_q1 = W.st_q1;
        d.st_gamma = W.st_gamma;
        d.st_delta = W.st_delta;
        d.cgls_iters = q.cgls_iters;
        b.h_stage[i] = d;
    }
    EPTV_HIP(hipMemcpyAsync(b.d_slices, b.h_stage, sizeof(SliceDev) * b.bd.n, hipMemcpyHostToDevice, s));
    EPTV_HIP(hipEventRecord(b.staged, s));
    return EPTV_OK;
}

// One outer iteration of the EPTV algorithm (Sec. 2.2) for every slice of the
// batch, each phase one launch; mirrors the one-slice enqueue.
static hipError_t enqueue_batch_iteration(const BatchDev& b, const eptv_params& q, bool with_ref, hipStream_t s)
{
    const int M = q.cgls_iters, T = q.tv_iters;
    const bool adaptive = q.sigma_fixed < 0;
    hipError_t e;
#define EPTV_TRY(call)                          \
    do {                                        \
        if ((e = (call)) != hipSuccess) return e; \
    } while (0)
    // Step 1: P1.  r = y - P f
    EPTV_TRY(blaunch_project(b, kBufF, kBufFT, -1.0f, 1.0f, kBufY, kBufR, kNoBuf, s));
    if (M > 0) {
        EPTV_TRY(blaunch_backproject(b, kBufR, 1.0f, 0.0f, kNoBuf, kBufS, kBufST, kPartBp, s));
        for (int m = 0; m < M; ++m) {
            const bool last = m == M - 1;
            EPTV_TRY(blaunch_project(b, kBufS, kBufST, 1.0f, 0.0f, kNoBuf, kBufQ, kPartProj, s));
            EPTV_TRY(blaunch_cgls_axpy(b, m, m == 0 ? kBufF : kBufU, last, s));
            if (last) break;
            EPTV_TRY(blaunch_backproject(b, kBufR, 1.0f, 0.0f, kNoBuf, kBufZ, kNoBuf, kPartBp, s));
            EPTV_TRY(blaunch_cgls_supdate(b, m, s));
        }
    } else {
        // gradient form of Eq. 8: v = f - mu/lambda P^T (P f - y) = f + mu/lambda P^T r
        EPTV_TRY(blaunch_backproject(b, kBufR, 1.0f, 0.0f, kNoBuf, kBufZ, kNoBuf, kNoBuf, s));
        EPTV_TRY(blaunch_gd_p1(b, (float)(q.mu / q.lambda), s));
    }
    // Step 2: P2 from v (or f^(k)), sigma from the start image
    const int start = q.p2_start ? kBufF : kBufU;
    const float eps2 = (float)(q.tv_eps * q.tv_eps);
    if (adaptive && T > 0) {
        EPTV_TRY(blaunch_edges_hist(b, start, eps2, s));
        EPTV_TRY(blaunch_select_finalize(b, 0, (float)q.sigma_floor, s));
        for (int pass = 1; pass <= 2; ++pass) {
            EPTV_TRY(blaunch_select_hist(b, pass, s));
            EPTV_TRY(blaunch_select_finalize(b, pass, (float)q.sigma_floor, s));
        }
    }
    const float t0 = t0_of(q), shrink = (float)q.armijo_shrink;
    const int gbuf[2] = {kBufG, kBufG2}, fbuf[2] = {kBufF1, kBufF2};
    // the decision of step `step`: a kernel of its own per step, one block per slice
    auto decision = [&](int step) {
        P2Decide D{};
        D.part = nullptr;
        D.step = step;
        D.T = T;
        D.max_bt = q.armijo_max_backtracks;
        D.c_arm = q.armijo_c;
        D.t0 = t0;
        D.shrink = shrink;
        D.replay = 0;
        return D;
    };
    int fcur = start;
    if (T == 1 && start == kBufF) {
        // the last step's kernel reads its iterate across the whole image in
        // the rare longer Armijo search while it writes f: keep them apart
        EPTV_TRY(blaunch_copy_clamp(b, start, kBufF1, kNoBuf, 0, s));
        fcur = kBufF1;
    }
    for (int t = 0; t < T; ++t) {
        const int gprev = t > 0 ? gbuf[(t - 1) & 1] : kNoBuf;
        const int fnext = t > 0 ? fbuf[t & 1] : kNoBuf;
        if (t > 0) EPTV_TRY(blaunch_p2_decide(b, fcur, gprev, kBufU, (float)q.lambda, eps2, decision(t - 1), s));
        EPTV_TRY(blaunch_p2_step(b, fcur, gprev, fnext, kBufU, (float)q.lambda, eps2, gbuf[t & 1], t0, shrink,
                                 decision(t - 1), s));
        if (t > 0) fcur = fnext;
    }
    // Step 3 (positivity) fused into the last update
    // (the update also forms the squared errors to the references, per tile)
    if (T == 0) {
        EPTV_TRY(blaunch_copy_clamp(b, start, kBufF, kBufFT, q.positivity, s));
        if (with_ref) EPTV_TRY(blaunch_rmse_part(b, kBufF, s));
    } else {
        EPTV_TRY(blaunch_p2_decide(b, fcur, gbuf[(T - 1) & 1], kBufU, (float)q.lambda, eps2, decision(T - 1), s));
        EPTV_TRY(blaunch_p2_final(b, fcur, gbuf[(T - 1) & 1], kBufF, kBufFT, q.positivity, with_ref, kBufU,
                                  (float)q.lambda, eps2, decision(T - 1), s));
    }
    EPTV_TRY(blaunch_iter_end(b, M > 0, with_ref, T > 0, sigma_init(q), s));
#undef EPTV_TRY
    return hipSuccess;
}

// Kernels are launched on the stream one by one unless EPTV_GRAPH is set to a
// value other than 0, which captures one outer iteration as a HIP graph and
// replays it.  On MI355X the direct launches are the faster of the two (a
// replayed kernel node costs a little more than a kernel launched on the
// stream, and an idle host keeps ahead of the GPU either way); the graph is
// for callers whose host thread is busy.
static bool no_graph()
{
    const char* v = std::getenv("EPTV_GRAPH");
    return !(v && *v && std::strcmp(v, "0") != 0);
}

}  // namespace eptv

using namespace eptv;

extern "C" {

int eptv_batch_create(const eptv_geometry* geoms, int n_slices, eptv_batch* out)
{
    if (!out) return EPTV_ERR_ARG;
    *out = nullptr;
    if (!geoms || n_slices <= 0 || n_slices > 65535) return EPTV_ERR_ARG;
    for (int i = 0; i < n_slices; ++i) {
        const int rc = validate_geometry(&geoms[i]);
        if (rc != EPTV_OK) return rc;
    }
    eptv_batch b = new (std::nothrow) eptv_batch_s();
    if (!b) return EPTV_ERR_ARG;
    for (int i = 0; i < n_slices; ++i) {
        eptv_plan p = nullptr;
        const int rc = eptv_plan_create(&geoms[i], &p);
        if (rc != EPTV_OK) {
            eptv_batch_destroy(b);
            return rc;
        }
        b->plans.push_back(p);
    }
    b->bd.n = n_slices;
    // work lists, slice by slice
    std::vector<int2> items[kNumShapes];
    for (int i = 0; i < n_slices; ++i) {
        const SliceDev d = slice_shape(b->plans[i]->p);
        for (int sh = 0; sh < kNumShapes; ++sh)
            for (int k = 0; k < items_of(d, sh); ++k) items[sh].push_back(make_int2(i, k));
    }
    hipError_t e = hipMalloc(&b->d_slices, sizeof(SliceDev) * n_slices);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_stage, sizeof(SliceDev) * n_slices, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b->staged, nullptr);
    for (int sh = 0; sh < kNumShapes && e == hipSuccess; ++sh) {
        e = hipMalloc(&b->d_items[sh], sizeof(int2) * items[sh].size());
        if (e == hipSuccess)
            e = hipMemcpy(b->d_items[sh], items[sh].data(), sizeof(int2) * items[sh].size(), hipMemcpyHostToDevice);
        b->bd.items[sh] = b->d_items[sh];
        b->bd.n_items[sh] = (int)items[sh].size();
        b->bd.grid[sh] = default_grid(sh, (int)items[sh].size());
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "eptv_batch_create");
        eptv_batch_destroy(b);
        return rc;
    }
    b->bd.slices = b->d_slices;
    b->bd.proj_seg = 16;
    *out = b;
    return EPTV_OK;
}

int eptv_batch_destroy(eptv_batch b)
{
    if (!b) return EPTV_ERR_ARG;
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    if (b->cap_stream) hipStreamDestroy(b->cap_stream);
    if (b->staged) hipEventDestroy(b->staged);
    if (b->h_stage) hipHostFree(b->h_stage);
    if (b->d_slices) hipFree(b->d_slices);
    for (int sh = 0; sh < kNumShapes; ++sh)
        if (b->d_items[sh]) hipFree(b->d_items[sh]);
    for (eptv_plan p : b->plans) eptv_plan_destroy(p);
    delete b;
    return EPTV_OK;
}

int eptv_batch_size(eptv_batch b, int* n_slices)
{
    if (!b || !n_slices) return EPTV_ERR_ARG;
    *n_slices = b->bd.n;
    return EPTV_OK;
}

int eptv_batch_plan(eptv_batch b, int slice, eptv_plan* plan)
{
    if (!b || !plan || slice < 0 || slice >= b->bd.n) return EPTV_ERR_ARG;
    *plan = b->plans[slice];
    return EPTV_OK;
}

int eptv_batch_workspace_bytes(eptv_batch b, const eptv_params* q, size_t* bytes)
{
    if (!b || !q || !bytes) return EPTV_ERR_ARG;
    const int rc = check_params(q);
    if (rc != EPTV_OK) return rc;
    *bytes = batch_ws_layout(*b, q->outer_iters, q->tv_iters, q->cgls_iters, nullptr, nullptr);
    return EPTV_OK;
}

int eptv_batch_set_launch(eptv_batch b, int proj_seg, int proj_blocks_per_cu, int tile_blocks_per_cu)
{
    if (!b || (proj_seg != 4 && proj_seg != 8 && proj_seg != 16) || proj_blocks_per_cu < 1 ||
        proj_blocks_per_cu > 64 || tile_blocks_per_cu < 1 || tile_blocks_per_cu > 64)
        return EPTV_ERR_ARG;
    std::lock_guard<std::mutex> lock(b->mu);
    b->bd.proj_seg = proj_seg;
    b->bd.grid[kShProj] = std::max(1, std::min(b->bd.n_items[kShProj], proj_blocks_per_cu * kCUs));
    for (int sh : {kShT16, kShT32, kShAxpy, kShSel, kShRmse})
        b->bd.grid[sh] = std::max(1, std::min(b->bd.n_items[sh], tile_blocks_per_cu * kCUs));
    return EPTV_OK;
}

int eptv_batch_get_launch(eptv_batch b, int* proj_seg, int* proj_grid, int* tile_grid)
{
    if (!b) return EPTV_ERR_ARG;
    if (proj_seg) *proj_seg = b->bd.proj_seg;
    if (proj_grid) *proj_grid = b->bd.grid[kShProj];
    if (tile_grid) *tile_grid = b->bd.grid[kShT16];
    return EPTV_OK;
}

// The launch-shape tuner: times the two operators of the batch (P over all
// slices, P^T over all slices) on scratch data for every candidate shape and
// keeps the fastest.  Candidates: projector sweep segments 4 / 8 / 16 with
// 1, 2 or 4 persistent blocks per CU; tile kernels with 2, 4, 8 or 16 blocks
// per CU (timed on the backprojector, applied to every tile-shaped phase).
int eptv_batch_tune(eptv_batch b, int reps, void* stream, float* proj_ms, float* backproj_ms)
{
    if (!b || reps < 1 || reps > 1000) return EPTV_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    eptv_params q{};
    q.outer_iters = 1;
    q.cgls_iters = 1;
    q.edge_quantile = 0.9;
    q.sigma_floor = 1e-12;
    q.sigma_fixed = -1.0;
    q.lambda = 1.0;
    const size_t bytes = batch_ws_layout(*b, 1, 0, 0, nullptr, nullptr);
    std::vector<float*> img(b->bd.n), sino(b->bd.n);
    char* ws = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = EPTV_OK;
    auto cleanup = [&]() {
        for (float* x : img) hipFree(x);
        for (float* x : sino) hipFree(x);
        if (ws) hipFree(ws);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
    };
    hipError_t e = hipMalloc(&ws, bytes);
    for (int i = 0; i < b->bd.n && e == hipSuccess; ++i) {
        const Plan& p = b->plans[i]->p;
        e = hipMalloc(&img[i], (size_t)p.nx * p.ny * 4);
        if (e == hipSuccess) e = hipMalloc(&sino[i], (size_t)p.V * p.B * 4);
        if (e == hipSuccess) e = launch_fill(img[i], (size_t)p.nx * p.ny, 0.01f, s);
        if (e == hipSuccess) e = launch_fill(sino[i], (size_t)p.V * p.B, 1.0f, s);
    }
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "eptv_batch_tune");
    }
    std::lock_guard<std::mutex> lock(b->mu);
    std::vector<Workspace> Ws;
    batch_ws_layout(*b, 1, 0, 0, ws, &Ws);
    rc = bind_batch(*b, q, Ws, (const float* const*)sino.data(), img.data(), nullptr, s);
    if (rc != EPTV_OK) {
        cleanup();
        return rc;
    }
    BatchDev& bd = b->bd;
    e = blaunch_transpose(bd, kBufF, kBufFT, s);
    auto time = [&](auto&& launch, float* ms) -> hipError_t {
        hipError_t err = launch();  // warm-up
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch();
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
        *ms /= (float)reps;
        return err;
    };
    float best_p = 1e30f, best_b = 1e30f;
    int seg_p = bd.proj_seg, grid_p = bd.grid[kShProj], per_cu_t = 8;
    for (int seg : {4, 8, 16})
        for (int per_cu : {1, 2, 4}) {
            if (e != hipSuccess) break;
            bd.proj_seg = seg;
            bd.grid[kShProj] = std::max(1, std::min(bd.n_items[kShProj], per_cu * kCUs));
            float ms = 0.0f;
            e = time([&]() { return blaunch_project(bd, kBufF, kBufFT, 1.0f, 0.0f, kNoBuf, kBufR, kNoBuf, s); },
                     &ms);
            if (e == hipSuccess && ms < best_p) {
                best_p = ms;
                seg_p = seg;
                grid_p = bd.grid[kShProj];
            }
        }
    for (int per_cu : {2, 4, 8, 16}) {
        if (e != hipSuccess) break;
        bd.grid[kShT16] = std::max(1, std::min(bd.n_items[kShT16], per_cu * kCUs));
        float ms = 0.0f;
        e = time([&]() { return blaunch_backproject(bd, kBufY, 1.0f, 0.0f, kNoBuf, kBufZ, kNoBuf, kNoBuf, s); }, &ms);
        if (e == hipSuccess && ms < best_b) {
            best_b = ms;
            per_cu_t = per_cu;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) return hip_fail(e, "eptv_batch_tune");
    bd.proj_seg = seg_p;
    bd.grid[kShProj] = grid_p;
    for (int sh : {kShT16, kShT32, kShAxpy, kShSel, kShRmse})
        bd.grid[sh] = std::max(1, std::min(bd.n_items[sh], per_cu_t * kCUs));
    if (proj_ms) *proj_ms = best_p;
    if (backproj_ms) *backproj_ms = best_b;
    return EPTV_OK;
}

// The operators of every slice in one launch each (the batch's projector and
// backprojector kernels over all slices), for callers that apply P or P^T to
// a stack of images, such as the differentiable operators.
static int batch_operator(eptv_batch b, bool forward, const float* const* in, float* const* out, float alpha,
                          float beta, void* ws, size_t ws_bytes, void* stream)
{
    if (!b || !in || !out) return EPTV_ERR_ARG;
    for (int i = 0; i < b->bd.n; ++i)
        if (!in[i] || !out[i]) return EPTV_ERR_ARG;
    if (!ws || ((uintptr_t)ws & 255)) return EPTV_ERR_WORKSPACE;
    std::vector<Workspace> Ws;
    if (batch_ws_layout(*b, 1, 0, 0, (char*)ws, &Ws) > ws_bytes) return EPTV_ERR_WORKSPACE;
    eptv_params q{};
    q.edge_quantile = 0.9;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(b->mu);
    const BatchDev& bd = b->bd;
    if (forward) {
        // image -> f (transposed into the workspace for the sweep layout), sinogram -> y
        int rc = bind_batch(*b, q, Ws, (const float* const*)out, (float* const*)in, nullptr, s);
        if (rc != EPTV_OK) return rc;
        EPTV_HIP(blaunch_transpose(bd, kBufF, kBufFT, s));
        EPTV_HIP(blaunch_project(bd, kBufF, kBufFT, alpha, beta, beta != 0.0f ? kBufY : kNoBuf, kBufY, kNoBuf, s));
    } else {
        // sinogram -> y, image -> f
        int rc = bind_batch(*b, q, Ws, in, out, nullptr, s);
        if (rc != EPTV_OK) return rc;
        EPTV_HIP(blaunch_backproject(bd, kBufY, alpha, beta, beta != 0.0f ? kBufF : kNoBuf, kBufF, kNoBuf, kNoBuf, s));
    }
    return EPTV_OK;
}

int eptv_batch_operator_workspace_bytes(eptv_batch b, size_t* bytes)
{
    if (!b || !bytes) return EPTV_ERR_ARG;
    *bytes = batch_ws_layout(*b, 1, 0, 0, nullptr, nullptr);
    return EPTV_OK;
}

int eptv_batch_project(eptv_batch b, const float* const* x, float* const* q, float alpha, float beta, void* ws,
                       size_t ws_bytes, void* stream)
{
    return batch_operator(b, true, x, q, alpha, beta, ws, ws_bytes, stream);
}

int eptv_batch_backproject(eptv_batch b, const float* const* r, float* const* z, float alpha, float beta, void* ws,
                           size_t ws_bytes, void* stream)
{
    return batch_operator(b, false, r, z, alpha, beta, ws, ws_bytes, stream);
}

int eptv_batch_reconstruct(eptv_batch b, const eptv_params* q, const float* const* y, float* const* f,
                           const float* const* f_ref, void* ws, size_t ws_bytes, eptv_stats* stats, void* stream)
{
    if (!b || !y || !f) return EPTV_ERR_ARG;
    int rc = check_params(q);
    if (rc != EPTV_OK) return rc;
    if (q->stored_matrix || q->interp_bp || q->stop_rmse > 0 || q->check_finite)
        return EPTV_ERR_ARG;  // one-slice variants only
    for (int i = 0; i < b->bd.n; ++i)
        if (!y[i] || !f[i] || (f_ref && !f_ref[i])) return EPTV_ERR_ARG;
    if (!ws || ((uintptr_t)ws & 255)) return EPTV_ERR_WORKSPACE;
    const int K = q->outer_iters, T = q->tv_iters;
    std::vector<Workspace> Ws;
    if (batch_ws_layout(*b, K, T, q->cgls_iters, (char*)ws, &Ws) > ws_bytes) return EPTV_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(b->mu);
    rc = bind_batch(*b, *q, Ws, y, f, f_ref, s);
    if (rc != EPTV_OK) return rc;
    const BatchDev& bd = b->bd;
    EPTV_HIP(blaunch_state_init(bd, sigma_init(*q), 1, s));
    if (q->zero_init) EPTV_HIP(blaunch_fill_zero(bd, kBufF, s));
    EPTV_HIP(blaunch_transpose(bd, kBufF, kBufFT, s));
    const bool with_ref = f_ref != nullptr;
    if (K > 0) {
        if (no_graph()) {
            for (int k = 0; k < K; ++k) EPTV_HIP(enqueue_batch_iteration(bd, *q, with_ref, s));
        } else {
            // the graph reads the descriptors at run time, so it depends only on
            // the parameters and the launch shapes
            std::vector<uint64_t> key;
            auto put = [&](const void* ptr, size_t n) {
                const unsigned char* c = (const unsigned char*)ptr;
                for (size_t i = 0; i < n; i += 8) {
                    uint64_t word = 0;
                    std::memcpy(&word, c + i, std::min<size_t>(8, n - i));
                    key.push_back(word);
                }
            };
            eptv_params qk = *q;
            qk.outer_iters = 0;
            qk.zero_init = 0;
            put(&qk, sizeof qk);
            put(bd.grid, sizeof bd.grid);
            const int extra[2] = {bd.proj_seg, (int)with_ref};
            put(extra, sizeof extra);
            if (!b->gexec || key != b->gkey) {
                if (b->gexec) {
                    hipGraphExecDestroy(b->gexec);
                    b->gexec = nullptr;
                }
                hipGraph_t graph = nullptr;
                EPTV_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
                hipError_t e = enqueue_batch_iteration(bd, *q, with_ref, b->cap_stream);
                hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
                if (e != hipSuccess) {
                    if (graph) hipGraphDestroy(graph);
                    return hip_fail(e, "enqueue_batch_iteration (capture)");
                }
                if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
                e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
                hipGraphDestroy(graph);
                if (e != hipSuccess) {
                    b->gexec = nullptr;
                    return hip_fail(e, "hipGraphInstantiate");
                }
                b->gkey = key;
            }
            for (int k = 0; k < K; ++k) EPTV_HIP(hipGraphLaunch(b->gexec, s));
        }
    }
    if (stats) {
        const size_t kk = (size_t)K;
        for (int i = 0; i < bd.n && kk; ++i) {
            const Workspace& W = Ws[i];
            eptv_stats& st = stats[i];
            if (st.sigma) EPTV_HIP(hipMemcpyAsync(st.sigma, W.st_sigma, kk * 4, hipMemcpyDeviceToHost, s));
            if (st.armijo_k && T > 0)
                EPTV_HIP(hipMemcpyAsync(st.armijo_k, W.st_k, kk * T * 4, hipMemcpyDeviceToHost, s));
            if (st.cgls_steps) EPTV_HIP(hipMemcpyAsync(st.cgls_steps, W.st_steps, kk * 4, hipMemcpyDeviceToHost, s));
            if (st.cgls_resid) EPTV_HIP(hipMemcpyAsync(st.cgls_resid, W.st_resid, kk * 8, hipMemcpyDeviceToHost, s));
            if (st.rmse && with_ref) EPTV_HIP(hipMemcpyAsync(st.rmse, W.st_rmse, kk * 8, hipMemcpyDeviceToHost, s));
            if (st.armijo_q0 && T > 0)
                EPTV_HIP(hipMemcpyAsync(st.armijo_q0, W.st_q0, kk * T * 8, hipMemcpyDeviceToHost, s));
            if (st.armijo_q1 && T > 0)
                EPTV_HIP(hipMemcpyAsync(st.armijo_q1, W.st_q1, kk * T * 8, hipMemcpyDeviceToHost, s));
            const size_t M = (size_t)q->cgls_iters;
            if (st.cgls_gamma && M)
                EPTV_HIP(hipMemcpyAsync(st.cgls_gamma, W.st_gamma, kk * M * 8, hipMemcpyDeviceToHost, s));
            if (st.cgls_delta && M)
                EPTV_HIP(hipMemcpyAsync(st.cgls_delta, W.st_delta, kk * M * 8, hipMemcpyDeviceToHost, s));
        }
        EPTV_HIP(hipStreamSynchronize(s));
    }
    return EPTV_OK;
}

}  // extern "C"
