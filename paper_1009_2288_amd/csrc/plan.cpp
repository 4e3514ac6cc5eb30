// plan.cpp -- host side of libeptv: geometry tables, workspace layout, the
// enqueue of one outer iteration, its launch (kernel by kernel, or as a
// captured graph) and the C ABI of eptv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "eptv_internal.h"
#include "geometry.h"
#include "host_internal.h"
#include "tables.h"

#include <vector>

namespace eptv {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return EPTV_ERR_HIP;
}

// ------------------------------------------------------------------ workspace
static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

size_t workspace_layout(const Plan& p, int K, int T, int M, char* base, Workspace* w)
{
    const size_t ni = (size_t)p.nx * p.ny, ns = (size_t)p.V * p.B;
    const size_t kcap = (size_t)std::max(K, 1), ktcap = std::max<size_t>((size_t)std::max(K, 1) * std::max(T, 0), 4096);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* ptr = base ? base + off : nullptr;
        off += align_up(bytes);
        return ptr;
    };
    Workspace tmp;
    Workspace& W = w ? *w : tmp;
    W.fT = (float*)take(ni * 4);
    W.u = (float*)take(ni * 4);
    W.s = (float*)take(ni * 4);
    W.sT = (float*)take(ni * 4);
    W.z = (float*)take(ni * 4);
    W.g = (float*)take(ni * 4);
    W.g2 = (float*)take(ni * 4);
    W.f1 = (float*)take(ni * 4);
    W.f2 = (float*)take(ni * 4);
    W.r = (float*)take(ns * 4);
    W.q = (float*)take(ns * 4);
    W.keys = (uint32_t*)take(n_edges(p) * 4);
    W.edge3 = (float*)take(3 * n_edges(p) * 4);
    W.hist = (uint32_t*)take(3 * kSelectBins * 4);
    W.part_proj = (double*)take((size_t)project_blocks(p) * 8);
    W.part_bp = (double*)take((size_t)image_tile_blocks(p) * 8);
    W.part_p2 = (double*)take((size_t)2 * kP2Slots * p2_blocks(p) * 8);
    W.part_res = (double*)take((size_t)sino_blocks(p) * 8);
    // per-block squared errors: the RMSE kernel's, or the final P2 update's (one per 32 x 32 tile)
    W.part_rmse = (double*)take((size_t)std::max(kRmseBlocks, update_tiles(p)) * 8);
    W.st = (DevState*)take(sizeof(DevState));
    W.st_sigma = (float*)take(kcap * 4);
    W.st_k = (int32_t*)take(ktcap * 4);
    W.st_steps = (int32_t*)take(kcap * 4);
    W.st_resid = (double*)take(kcap * 8);
    W.st_rmse = (double*)take(kcap * 8);
    W.st_q0 = (double*)take(ktcap * 8);
    W.st_q1 = (double*)take(ktcap * 8);
    W.st_gamma = (double*)take(kcap * (size_t)std::max(M, 0) * 8);
    W.st_delta = (double*)take(kcap * (size_t)std::max(M, 0) * 8);
    W.bytes = off;
    return off;
}

struct Ctx {
    const Plan& p;
    Workspace& W;
    const eptv_params& q;
    const float* y;
    float* f;
    const float* f_ref;
    const float* wx_in = nullptr;  // given half-edge weights for P2 (frozen iterations), or null
    const float* wy_in = nullptr;
    int replay = 0;                // 1: the Armijo decisions come from the step records (uploaded by the caller)
};


// sigma from the half-edge magnitudes of `img` (radix select, three digits).
// The selection of sigma (three digit passes); with last_digit false the
// last digit is left to the first P2 kernel (enqueue_p2's close_sigma).
// With edges false the first digit's histogram is already there (formed by
// the launch that produced img).
static hipError_t enqueue_select(const Plan& p, Workspace& W, const float* img, float eps2, float floor_,
                                 hipStream_t s, bool last_digit = true, bool edges = true)
{
    hipError_t e;
    if (edges && (e = launch_edges_hist(p, img, eps2, W.keys, W.hist, s)) != hipSuccess) return e;
    for (int pass = 1; pass <= 2; ++pass)
        if ((e = launch_select_pass(p, pass, W.keys, W.st, W.hist, s)) != hipSuccess) return e;
    return last_digit ? launch_select_sigma(W.st, W.hist, floor_, s) : hipSuccess;
}


// n_steps P2 descent steps (Sec. 2.2; Armijo line search) from `start`
// towards v; the result goes to `fout` (and its transpose to foutT when
// given), truncated at zero when `clamp`.  Step t > 0 applies step t-1 inside
// its gradient kernel, so only the last step has an update kernel of its own.

static hipError_t enqueue_p2(const Plan& p, Workspace& W, const eptv_params& q, const float* start, const float* v,
                             int n_steps, float* fout, float* foutT, int clamp, int32_t* st_k, hipStream_t s,
                             const float* wx_in = nullptr, const float* wy_in = nullptr, int replay = 0,
                             const float* f_ref = nullptr, bool close_sigma = false)
{
    hipError_t e;
    if (n_steps == 0) return launch_copy_clamp(p, start, fout, foutT, clamp, s);
    const float eps2 = (float)(q.tv_eps * q.tv_eps);
    const float t0 = t0_of(q), shrink = (float)q.armijo_shrink;
    const size_t np = (size_t)kP2Slots * p2_blocks(p);
    const float* fcur = start;
    float* gbuf[2] = {W.g, W.g2};
    float* fbuf[2] = {W.f1, W.f2};
    // the decision of step `step`, taken by the kernel after it
    auto decision = [&](int step) {
        P2Decide D{};
        D.part = step >= 0 ? W.part_p2 + (size_t)(step & 1) * np : nullptr;
        D.step = step;
        D.T = n_steps;
        D.max_bt = q.armijo_max_backtracks;
        D.c_arm = q.armijo_c;
        D.t0 = t0;
        D.shrink = shrink;
        D.replay = replay;
        D.st_k = st_k;
        D.st_q0 = W.st_q0;
        D.st_q1 = W.st_q1;
        return D;
    };
    if (n_steps == 1 && start == fout) {
        // the last step's kernel reads its iterate across the whole image in
        // the rare longer Armijo search while it writes fout: keep them apart
        if ((e = launch_copy_clamp(p, start, fbuf[0], nullptr, 0, s)) != hipSuccess) return e;
        fcur = fbuf[0];
    }
    for (int t = 0; t < n_steps; ++t) {
        // step t: the decision of step t-1, the iterate, the direction and
        // the first Armijo trials (the first step closes sigma's last digit
        // when the selection left it open)
        const bool sel = close_sigma && t == 0;
        float* fnext = t > 0 ? fbuf[t & 1] : nullptr;
        if ((e = launch_p2_step(p, fcur, t > 0 ? gbuf[(t - 1) & 1] : nullptr, fnext, v, (float)q.lambda, W.st, eps2,
                                gbuf[t & 1], W.part_p2 + (size_t)(t & 1) * np, t0, shrink, wx_in, wy_in,
                                sel ? W.hist + 2 * kSelectBins : nullptr, (float)q.sigma_floor, decision(t - 1),
                                s)) != hipSuccess)
            return e;
        if (t > 0) fcur = fnext;
    }
    return launch_p2_final(p, fcur, gbuf[(n_steps - 1) & 1], fout, foutT, clamp, f_ref, W.part_rmse, v,
                           (float)q.lambda, W.st, eps2, wx_in, wy_in, decision(n_steps - 1), s);
}

// One outer iteration of the EPTV algorithm (Sec. 2.2), entirely on `s`.
// What closes an outer iteration of c (records, counter, state reset).
static IterEnd iteration_end(const Ctx& c)
{
    const Plan& p = c.p;
    Workspace& W = c.W;
    const int M = c.q.cgls_iters, T = c.q.tv_iters;
    return iter_end_args(p, W.st, W.part_res, M > 0, W.part_rmse, T > 0 ? update_tiles(p) : kRmseBlocks,
                         c.f_ref != nullptr, W.st_sigma, W.st_steps, W.st_resid, W.st_rmse, M, W.st_gamma,
                         W.st_delta, W.hist, sigma_init(c.q));
}

// Whether an iteration can leave its close to the next iteration's first
// kernel: only the stored projector takes it (one extra block of its launch).
static bool can_defer_end(const Ctx& c) { return c.q.stored_matrix == 1; }

// One outer iteration.  fold_prev: the previous iteration's close, still
// pending, run by this iteration's first projector launch (can_defer_end);
// defer_end: leave this iteration's close pending instead of launching it.
static hipError_t enqueue_iteration(const Ctx& c, hipStream_t s, bool fold_prev = false, bool defer_end = false)
{
    const Plan& p = c.p;
    Workspace& W = c.W;
    const eptv_params& q = c.q;
    const int M = q.cgls_iters, T = q.tv_iters;
    const bool adaptive = q.sigma_fixed < 0;
    hipError_t e;
    // (the per-iteration state was reset by the previous iteration's close,
    // by this iteration's first kernel, or by the caller)
    const IterEnd close = iteration_end(c);
    // Step 1: P1.  r = y - P f
    // P and P^T: on the fly, or from the stored matrix (the paper's two strategies,
    // Sec. 2.3), or P on the fly and P^T stored (stored_matrix = 2); both are the
    // same float32 matrix, so the pair stays exactly adjoint
    auto proj = [&](const float* x, const float* xT, float al, float be, const float* cc, float* out, double* part) {
        return q.stored_matrix == 1 ? launch_project_stored(p, x, xT, al, be, cc, out, part, s)
                               : launch_project(p, x, xT, al, be, cc, out, part, s);
    };
    // P^T: the exact transpose (on the fly or stored), or the Eq. 11 operator
    auto bproj = [&](const float* rr, float al, float be, const float* cc, float* zz, float* zzT, double* part) {
        if (q.interp_bp) return launch_backproject_interp(p, rr, al, be, cc, zz, zzT, part, s);
        return q.stored_matrix ? launch_backproject_stored(p, rr, al, be, cc, zz, zzT, part, s)
                               : launch_backproject(p, rr, al, be, cc, zz, zzT, part, s);
    };
    if (fold_prev) {
        if (!can_defer_end(c)) return hipErrorInvalidValue;
        if ((e = launch_project_stored(p, c.f, W.fT, -1.0f, 1.0f, c.y, W.r, nullptr, s, &close)) != hipSuccess)
            return e;
    } else if ((e = proj(c.f, W.fT, -1.0f, 1.0f, c.y, W.r, nullptr)) != hipSuccess) {
        return e;
    }
    // sigma is chosen from P2's start image when it is not given; when that is
    // v, the last CGLS step's launch also forms the first digit's histogram of
    // its half-edges, and writes v to z (free by then) so that the histogram
    // blocks read the step's unchanged inputs
    const bool select = adaptive && T > 0 && !c.wx_in;
    const bool fused_edges = select && M > 0 && !q.p2_start;
    const float eps2 = (float)(q.tv_eps * q.tv_eps);
    float* const v_out = fused_edges ? W.z : W.u;
    if (M > 0) {
        // s = P^T r (gamma_0 partials)
        if ((e = bproj(W.r, 1.0f, 0.0f, nullptr, W.s, W.sT, W.part_bp)) != hipSuccess) return e;
        for (int m = 0; m < M; ++m) {
            const bool last = m == M - 1;
            // q = P s (delta_m partials); u += a_m s, r -= a_m q
            if ((e = proj(W.s, W.sT, 1.0f, 0.0f, nullptr, W.q, W.part_proj)) != hipSuccess) return e;
            const float* u_in = m == 0 ? c.f : W.u;
            if (last && fused_edges)
                e = launch_cgls_axpy_edges(p, W.st, m, W.part_bp, W.part_proj, u_in, v_out, W.s, W.r, W.q,
                                           W.part_res, eps2, W.keys, W.hist, s);
            else
                e = launch_cgls_axpy(p, W.st, m, W.part_bp, W.part_proj, u_in, W.u, W.s, W.r, W.q,
                                     last ? W.part_res : nullptr, s);
            if (e != hipSuccess) return e;
            if (last) break;  // P^T r of the final residual is not needed
            // z = P^T r (gamma_{m+1} partials); s = z + b_m s
            if ((e = bproj(W.r, 1.0f, 0.0f, nullptr, W.z, nullptr, W.part_bp)) != hipSuccess) return e;
            if ((e = launch_cgls_supdate(p, W.st, m, W.part_bp, W.z, W.s, W.sT, s)) != hipSuccess) return e;
        }
    } else {
        // gradient form of Eq. 8: v = f - mu/lambda P^T (P f - y)
        if ((e = bproj(W.r, 1.0f, 0.0f, nullptr, W.z, nullptr, nullptr)) != hipSuccess) return e;
        if ((e = launch_gd_p1(p, c.f, W.z, (float)(q.mu / q.lambda), W.u, s)) != hipSuccess) return e;
    }
    // Step 2: P2 from v (or f^(k)), sigma chosen once from the start image.
    const float* start = q.p2_start ? c.f : v_out;
    if (select) {  // the last digit is closed by the first descent step's kernel
        if ((e = enqueue_select(p, W, start, eps2, (float)q.sigma_floor, s, false, !fused_edges)) != hipSuccess)
            return e;
    }
    // Step 3 (positivity) is fused into the last descent update.
    // With a reference, the last update also forms the squared errors per tile.
    if ((e = enqueue_p2(p, W, q, start, v_out, T, c.f, W.fT, q.positivity, W.st_k, s, c.wx_in, c.wy_in, c.replay,
                        c.f_ref, select)) != hipSuccess)
        return e;
    if (c.f_ref && T == 0) {
        if ((e = launch_rmse_part(p, c.f, c.f_ref, W.part_rmse, s)) != hipSuccess) return e;
    }
    if (defer_end) return can_defer_end(c) ? hipSuccess : hipErrorInvalidValue;
    return launch_iter_end(close, s);
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

// ================================================================== C ABI
extern "C" {

const char* eptv_status_string(int status)
{
    switch (status) {
    case EPTV_OK: return "ok";
    case EPTV_ERR_ARG: return "invalid argument";
    case EPTV_ERR_GEOMETRY: return "invalid geometry";
    case EPTV_ERR_WORKSPACE: return "workspace missing or too small";
    case EPTV_ERR_HIP: return "HIP runtime error";
    case EPTV_ERR_NONFINITE: return "non-finite input";
    default: return "unknown status";
    }
}

const char* eptv_last_error(void) { return g_last_error.c_str(); }

int eptv_plan_create(const eptv_geometry* geom, eptv_plan* out)
{
    if (!out) return EPTV_ERR_ARG;
    *out = nullptr;
    int rc = validate_geometry(geom);
    if (rc != EPTV_OK) return rc;
    eptv_plan h = new (std::nothrow) eptv_plan_s();
    if (!h) return EPTV_ERR_ARG;
    Plan& p = h->p;
    p = host_plan(geom);

    HostTables t;
    build_tables(p, t);
    p.nnz = t.nnz;
    const auto& ray = t.ray;
    const auto& range = t.range;
    const auto& view = t.view;
    const auto& view_d = t.view_d;
    const auto& tau = t.tau;
    const auto& list_off = t.list_off;
    const auto& list = t.list;
    hipError_t e = hipGetDevice(&p.device);
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_ray, ray.size() * sizeof(RayFx));
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_range, range.size() * sizeof(int2));
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_view, view.size() * sizeof(float2));
    if (e == hipSuccess) e = hipMemcpy(p.rays.d_ray, ray.data(), ray.size() * sizeof(RayFx), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p.rays.d_range, range.data(), range.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p.rays.d_view, view.data(), view.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_view_d, view_d.size() * sizeof(double2));
    if (e == hipSuccess)
        e = hipMemcpy(p.rays.d_view_d, view_d.data(), view_d.size() * sizeof(double2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_tau, tau.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(p.rays.d_tau, tau.data(), tau.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_list_off, list_off.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_list, std::max<size_t>(list.size(), 1) * sizeof(int));
    if (e == hipSuccess)
        e = hipMemcpy(p.rays.d_list_off, list_off.data(), list_off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && !list.empty())
        e = hipMemcpy(p.rays.d_list, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        rc = hip_fail(e, "eptv_plan_create");
        eptv_plan_destroy(h);
        return rc;
    }
    *out = h;
    return EPTV_OK;
}

int eptv_plan_destroy(eptv_plan h)
{
    if (!h) return EPTV_ERR_ARG;
    Plan& p = h->p;
    if (h->host_buf) (void)hipHostFree(h->host_buf);
    if (p.gexec) hipGraphExecDestroy(p.gexec);
    if (p.gexec_w) hipGraphExecDestroy(p.gexec_w);
    if (p.cap_stream) hipStreamDestroy(p.cap_stream);
    if (p.rays.d_ray) hipFree(p.rays.d_ray);
    if (p.mat.d_rowptr) hipFree(p.mat.d_rowptr);
    if (p.mat.d_rent) hipFree(p.mat.d_rent);
    if (p.mat.d_rwords) hipFree(p.mat.d_rwords);
    if (p.mat.d_colptr) hipFree(p.mat.d_colptr);
    if (p.mat.d_cent) hipFree(p.mat.d_cent);
    if (p.rays.d_range) hipFree(p.rays.d_range);
    if (p.rays.d_view) hipFree(p.rays.d_view);
    if (p.rays.d_view_d) hipFree(p.rays.d_view_d);
    if (p.rays.d_tau) hipFree(p.rays.d_tau);
    if (p.rays.d_list_off) hipFree(p.rays.d_list_off);
    if (p.rays.d_list) hipFree(p.rays.d_list);
    delete h;
    return EPTV_OK;
}

int eptv_plan_nnz(eptv_plan h, long long* nnz)
{
    if (!h || !nnz) return EPTV_ERR_ARG;
    *nnz = h->p.nnz;
    return EPTV_OK;
}

int eptv_geometry_matrix(const eptv_geometry* geom, long long* nnz, long long* rowptr, int* col, float* val)
{
    if (!nnz) return EPTV_ERR_ARG;
    const int rc = validate_geometry(geom);
    if (rc != EPTV_OK) return rc;
    const Plan p = host_plan(geom);
    HostCsr m;
    build_csr(p, m);
    *nnz = (long long)m.col.size();
    if (rowptr) std::memcpy(rowptr, m.rowptr.data(), m.rowptr.size() * sizeof(long long));
    if (col) std::memcpy(col, m.col.data(), m.col.size() * sizeof(int));
    if (val) std::memcpy(val, m.val.data(), m.val.size() * sizeof(float));
    return EPTV_OK;
}

int eptv_plan_store_matrix(eptv_plan h, size_t* device_bytes)
{
    if (!h) return EPTV_ERR_ARG;
    Plan& p = h->p;
    if (!p.mat.d_rowptr) {
        HostStored hs;
        if (pack_stored(p, hs) != EPTV_OK) return EPTV_ERR_ARG;
        // the CSR copy goes up in one encoding: compact when it applies, else
        // wide; bit 31 of a ray's offset marks a ray swept row by row
        std::vector<int> rowptr = hs.compact ? hs.rwordptr : hs.rowptr;
        for (size_t r = 0; r < hs.rows.size(); ++r)
            if (hs.rows[r]) rowptr[r] = (int)((unsigned)rowptr[r] | 0x80000000u);
        const size_t rbytes = hs.compact ? hs.rwords.size() * 4 : hs.rent.size() * 8;
        const void* rsrc = hs.compact ? (const void*)hs.rwords.data() : (const void*)hs.rent.data();
        const auto& colptr = hs.colptr;
        const auto& cent = hs.cent;
        StoredMatrix& S = p.mat;
        void* rdst = nullptr;
        hipError_t e = hipMalloc(&S.d_rowptr, rowptr.size() * 4);
        if (e == hipSuccess) e = hipMalloc(&rdst, rbytes);
        if (e == hipSuccess) e = hipMalloc(&S.d_colptr, colptr.size() * 4);
        if (e == hipSuccess) e = hipMalloc(&S.d_cent, cent.size() * 8);
        if (e == hipSuccess) e = hipMemcpy(S.d_rowptr, rowptr.data(), rowptr.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(rdst, rsrc, rbytes, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(S.d_colptr, colptr.data(), colptr.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(S.d_cent, cent.data(), cent.size() * 8, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            for (void* ptr : {(void*)S.d_rowptr, rdst, (void*)S.d_colptr, (void*)S.d_cent})
                if (ptr) hipFree(ptr);
            S = StoredMatrix();
            return hip_fail(e, "eptv_plan_store_matrix");
        }
        S.compact = hs.compact;
        if (hs.compact)
            S.d_rwords = (int*)rdst;
        else
            S.d_rent = (int2*)rdst;
        S.slots = (long long)hs.rowptr.back();
        S.nnz = hs.nnz;
        S.csr_bytes = rowptr.size() * 4 + rbytes;
        S.bytes = S.csr_bytes + colptr.size() * 4 + cent.size() * 8;
    }
    if (device_bytes) *device_bytes = p.mat.bytes;
    return EPTV_OK;
}

int eptv_plan_stored_layout(eptv_plan h, int* csr_compact, size_t* csr_bytes, size_t* csc_bytes)
{
    if (!h || !h->p.mat.d_rowptr) return EPTV_ERR_ARG;
    const StoredMatrix& S = h->p.mat;
    if (csr_compact) *csr_compact = S.compact ? 1 : 0;
    if (csr_bytes) *csr_bytes = S.csr_bytes;
    if (csc_bytes) *csc_bytes = S.bytes - S.csr_bytes;
    return EPTV_OK;
}

int eptv_backproject_stored(eptv_plan h, const float* r, float* z, float alpha, float beta, void* stream)
{
    if (!h || !r || !z || !h->p.mat.d_rowptr) return EPTV_ERR_ARG;
    EPTV_HIP(launch_backproject_stored(h->p, r, alpha, beta, z, z, nullptr, nullptr, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_workspace_bytes(eptv_plan h, const eptv_params* q, size_t* bytes)
{
    if (!h || !bytes) return EPTV_ERR_ARG;
    int K = 1, T = 0;
    if (q) {
        int rc = check_params(q);
        if (rc != EPTV_OK) return rc;
        K = q->outer_iters;
        T = q->tv_iters;
    }
    *bytes = workspace_layout(h->p, K, T, q ? q->cgls_iters : 0, nullptr, nullptr);
    return EPTV_OK;
}

static int bind_ws(const Plan& p, int K, int T, int M, void* ws, size_t ws_bytes, Workspace* W)
{
    if (!ws || ((uintptr_t)ws & 255)) return EPTV_ERR_WORKSPACE;
    const size_t need = workspace_layout(p, K, T, M, (char*)ws, W);
    return ws_bytes >= need ? EPTV_OK : EPTV_ERR_WORKSPACE;
}

int eptv_project(eptv_plan h, const float* x, float* q, float alpha, float beta, void* ws, size_t ws_bytes,
                 void* stream)
{
    if (!h || !x || !q) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    EPTV_HIP(launch_transpose(x, W.fT, h->p.nx, h->p.ny, s));
    EPTV_HIP(launch_project(h->p, x, W.fT, alpha, beta, q, q, nullptr, s));
    return EPTV_OK;
}

int eptv_project_dual(eptv_plan h, const float* x, const float* xT, float* q, float alpha, float beta, void* stream)
{
    if (!h || !x || !xT || !q) return EPTV_ERR_ARG;
    EPTV_HIP(launch_project(h->p, x, xT, alpha, beta, q, q, nullptr, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_project_stored(eptv_plan h, const float* x, float* q, float alpha, float beta, void* ws, size_t ws_bytes,
                        void* stream)
{
    if (!h || !x || !q || !h->p.mat.d_rowptr) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    EPTV_HIP(launch_transpose(x, W.fT, h->p.nx, h->p.ny, s));
    EPTV_HIP(launch_project_stored(h->p, x, W.fT, alpha, beta, q, q, nullptr, s));
    return EPTV_OK;
}

int eptv_project_stored_dual(eptv_plan h, const float* x, const float* xT, float* q, float alpha, float beta,
                             void* stream)
{
    if (!h || !x || !xT || !q || !h->p.mat.d_rowptr) return EPTV_ERR_ARG;
    EPTV_HIP(launch_project_stored(h->p, x, xT, alpha, beta, q, q, nullptr, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_backproject(eptv_plan h, const float* r, float* z, float alpha, float beta, void* ws, size_t ws_bytes,
                     void* stream)
{
    if (!h || !r || !z) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    EPTV_HIP(launch_backproject(h->p, r, alpha, beta, z, z, nullptr, nullptr, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_backproject_interp(eptv_plan h, const float* r, float* z, float alpha, float beta, void* stream)
{
    if (!h || !r || !z) return EPTV_ERR_ARG;
    EPTV_HIP(launch_backproject_interp(h->p, r, alpha, beta, z, z, nullptr, nullptr, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_tv_gradient(eptv_plan h, const float* f, const float* v, float lambda, float sigma, float tv_eps, float* g,
                     float* wx, float* wy, void* ws, size_t ws_bytes, void* stream)
{
    if (!h || !f || !v || !g) return EPTV_ERR_ARG;
    if (!(sigma > 0) || !tv_eps_ok(tv_eps) || !std::isfinite(lambda)) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    EPTV_HIP(launch_tv_grad(h->p, f, v, lambda, sigma, tv_eps * tv_eps, g, wx, wy, nullptr, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_tv_gradient_vjp(eptv_plan h, const float* f, const float* u, float lambda, float sigma, float tv_eps,
                         float* out, void* ws, size_t ws_bytes, void* stream)
{
    if (!h || !f || !u || !out) return EPTV_ERR_ARG;
    if (!(sigma > 0) || !tv_eps_ok(tv_eps) || !std::isfinite(lambda)) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    EPTV_HIP(launch_tv_vjp(h->p, f, u, lambda, sigma, tv_eps * tv_eps, W.edge3, out, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_select_sigma(eptv_plan h, const float* f, double q, float tv_eps, float sigma_floor, float* sigma_out,
                      void* ws, size_t ws_bytes, void* stream)
{
    if (!h || !f || !sigma_out) return EPTV_ERR_ARG;
    if (!(q > 0 && q <= 1) || !(tv_eps >= 0) || !(sigma_floor > 0)) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    EPTV_HIP(launch_state_init(W.st, W.hist, select_rank(h->p, q), -1.0f, 1, s));
    EPTV_HIP(enqueue_select(h->p, W, f, tv_eps * tv_eps, sigma_floor, s));
    EPTV_HIP(launch_sigma_out(W.st, sigma_out, s));
    return EPTV_OK;
}

int eptv_tv_step(eptv_plan h, const eptv_params* q, float* f, const float* v, float sigma, int n_steps, void* ws,
                 size_t ws_bytes, eptv_stats* stats, void* stream)
{
    if (!h || !f || !v || n_steps < 0 || n_steps > 4096) return EPTV_ERR_ARG;
    if (!q || !(q->lambda > 0) || !(q->armijo_shrink > 0 && q->armijo_shrink < 1) || q->armijo_max_backtracks < 0 ||
        q->armijo_max_backtracks > 4096 || !tv_eps_ok(q->tv_eps) || !(q->sigma_floor > 0))
        return EPTV_ERR_ARG;
    if (sigma < 0 && !(q->edge_quantile > 0 && q->edge_quantile <= 1)) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Plan& p = h->p;
    EPTV_HIP(launch_state_init(W.st, W.hist, select_rank(p, q->edge_quantile), sigma < 0 ? -1.0f : sigma, 1, s));
    if (sigma < 0) EPTV_HIP(enqueue_select(p, W, f, (float)(q->tv_eps * q->tv_eps), (float)q->sigma_floor, s));
    EPTV_HIP(enqueue_p2(p, W, *q, f, v, n_steps, f, nullptr, 0, W.st_k, s));
    if (stats) {
        if (stats->sigma) EPTV_HIP(hipMemcpyAsync(stats->sigma, &W.st->sigma, 4, hipMemcpyDeviceToHost, s));
        if (stats->armijo_k && n_steps > 0)
            EPTV_HIP(hipMemcpyAsync(stats->armijo_k, W.st_k, (size_t)n_steps * 4, hipMemcpyDeviceToHost, s));
        if (stats->armijo_q0 && n_steps > 0)
            EPTV_HIP(hipMemcpyAsync(stats->armijo_q0, W.st_q0, (size_t)n_steps * 8, hipMemcpyDeviceToHost, s));
        if (stats->armijo_q1 && n_steps > 0)
            EPTV_HIP(hipMemcpyAsync(stats->armijo_q1, W.st_q1, (size_t)n_steps * 8, hipMemcpyDeviceToHost, s));
        EPTV_HIP(hipStreamSynchronize(s));
    }
    return EPTV_OK;
}

// The plan's page-locked staging, at least `bytes`; call with h->host_mu held
// and nothing in flight into the old buffer.
static hipError_t host_staging(eptv_plan h, size_t bytes, void** out)
{
    if (h->host_bytes < bytes) {
        if (h->host_buf) (void)hipHostFree(h->host_buf);
        h->host_buf = nullptr;
        h->host_bytes = 0;
        const size_t n = std::max<size_t>(bytes, 4096);
        const hipError_t e = hipHostMalloc(&h->host_buf, n, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        h->host_bytes = n;
    }
    *out = h->host_buf;
    return hipSuccess;
}

}  // extern "C"

namespace eptv {

// Reads n bytes of device memory back to the host after the stream's work so
// far: through the plan's page-locked staging (grown on demand), or, for a
// caller that must not allocate, straight into the destination.
static int read_back(eptv_plan h, bool noalloc, void* dst, const void* src, size_t n, hipStream_t s)
{
    if (noalloc) {
        EPTV_HIP(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s));
        EPTV_HIP(hipStreamSynchronize(s));
        return EPTV_OK;
    }
    std::lock_guard<std::mutex> hl(h->host_mu);
    void* hb = nullptr;
    EPTV_HIP(host_staging(h, n, &hb));
    EPTV_HIP(hipMemcpyAsync(hb, src, n, hipMemcpyDeviceToHost, s));
    EPTV_HIP(hipStreamSynchronize(s));
    std::memcpy(dst, hb, n);
    return EPTV_OK;
}

// The outer loop behind every eptv_reconstruct* entry point.  With noalloc the
// iteration is launched kernel by kernel whatever EPTV_GRAPH says (a graph's
// instantiation allocates) and host reads go straight to their destination.
int reconstruct_impl(eptv_plan h, const eptv_params* q, const float* y, float* f, const float* f_ref,
                     const float* wx_in, const float* wy_in, int frozen, const int32_t* replay, void* ws,
                     size_t ws_bytes, eptv_stats* stats, void* stream, bool noalloc)
{
    if (!h || !y || !f) return EPTV_ERR_ARG;
    int rc = check_params(q);
    if (rc != EPTV_OK) return rc;
    Plan& p = h->p;
    if (q->stored_matrix && !p.mat.d_rowptr) return EPTV_ERR_ARG;
    Workspace W;
    rc = bind_ws(p, q->outer_iters, q->tv_iters, q->cgls_iters, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int K = q->outer_iters, T = q->tv_iters;
    frozen = std::min(std::max(frozen, 0), K);

    if (replay) {
        for (size_t i = 0; i < (size_t)K * T; ++i)
            if (replay[i] < -1 || replay[i] > q->armijo_max_backtracks) return EPTV_ERR_ARG;
    }
    const bool stop = f_ref && q->stop_rmse > 0;
    const int every = std::max(1, q->check_every);

    if (q->check_finite) {
        // the optional input check, before anything else is enqueued
        EPTV_HIP(launch_scan_finite(y, (size_t)p.V * p.B, W.st, 0, s));
        if (!q->zero_init) EPTV_HIP(launch_scan_finite(f, (size_t)p.nx * p.ny, W.st, 1, s));
        int bad = 0;
        rc = read_back(h, noalloc, &bad, &W.st->nonfinite, sizeof bad, s);
        if (rc != EPTV_OK) return rc;
        if (bad) return EPTV_ERR_NONFINITE;
    }

    EPTV_HIP(launch_recon_start(f, W.fT, p.nx, p.ny, q->zero_init != 0, W.st, W.hist,
                                select_rank(p, q->edge_quantile), sigma_init(*q), s));
    // replay: the decisions are read back from the step records
    if (replay && (size_t)K * T)
        EPTV_HIP(hipMemcpyAsync(W.st_k, replay, (size_t)K * T * 4, hipMemcpyHostToDevice, s));

    Ctx c{p, W, *q, y, f, f_ref};
    c.replay = replay ? 1 : 0;
    Ctx cw{p, W, *q, y, f, f_ref, wx_in, wy_in};
    int done = 0;          // iterations run so far
    bool stopped = false;  // the RMSE reached stop_rmse at a check
    bool pending = false;  // the last iteration's close is left to the next one's first kernel
    // after each iteration: every check_every-th one, read its RMSE record back
    auto check = [&]() -> int {
        ++done;
        if (!stop || done % every) return EPTV_OK;
        double r = 0.0;
        const int rc_ = read_back(h, noalloc, &r, W.st_rmse + (done - 1), sizeof r, s);
        if (rc_ != EPTV_OK) return rc_;
        if (r <= q->stop_rmse) stopped = true;
        return EPTV_OK;
    };
    // the iteration launched kernel by kernel, or (EPTV_GRAPH=1) one captured
    // graph per kind of iteration (adaptive, or with the given weights)
    auto run = [&](const Ctx& cc, int count, hipGraphExec_t& gexec, std::vector<uint64_t>& gkey) -> int {
        if (count <= 0 || stopped) return EPTV_OK;
        if (noalloc || no_graph()) {
            for (int k = 0; k < count && !stopped; ++k) {
                // the close of each iteration goes into the next one's first
                // launch, except where its records are read right after
                const bool defer = can_defer_end(cc) && !(stop && (done + 1) % every == 0);
                EPTV_HIP(enqueue_iteration(cc, s, pending, defer));
                pending = defer;
                const int rc_ = check();
                if (rc_ != EPTV_OK) return rc_;
            }
            return EPTV_OK;
        }
        std::vector<uint64_t> key;
        auto put = [&](const void* ptr, size_t n) {
            const unsigned char* b = (const unsigned char*)ptr;
            for (size_t i = 0; i < n; i += 8) {
                uint64_t word = 0;
                std::memcpy(&word, b + i, std::min<size_t>(8, n - i));
                key.push_back(word);
            }
        };
        eptv_params qk = *q;
        qk.outer_iters = 0;
        qk.zero_init = 0;
        put(&qk, sizeof qk);
        const void* ptrs[8] = {ws, y, f, f_ref, (const void*)(uintptr_t)ws_bytes, cc.wx_in, cc.wy_in,
                               (const void*)(uintptr_t)cc.replay};
        put(ptrs, sizeof ptrs);
        if (!gexec || key != gkey) {
            if (gexec) {
                hipGraphExecDestroy(gexec);
                gexec = nullptr;
            }
            hipGraph_t graph = nullptr;
            EPTV_HIP(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_iteration(cc, p.cap_stream);
            hipError_t e2 = hipStreamEndCapture(p.cap_stream, &graph);
            if (e != hipSuccess) {
                if (graph) hipGraphDestroy(graph);
                return hip_fail(e, "enqueue_iteration (capture)");
            }
            if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
            e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) {
                gexec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
            gkey = key;
        }
        for (int k = 0; k < count && !stopped; ++k) {
            EPTV_HIP(hipGraphLaunch(gexec, s));
            const int rc_ = check();
            if (rc_ != EPTV_OK) return rc_;
        }
        return EPTV_OK;
    };
    {
        std::lock_guard<std::mutex> lock(h->graph_mu);
        rc = run(cw, wx_in ? frozen : 0, p.gexec_w, p.gkey_w);
        if (rc == EPTV_OK) rc = run(c, K - (wx_in ? frozen : 0), p.gexec, p.gkey);
    }
    if (rc != EPTV_OK) return rc;
    if (pending) EPTV_HIP(launch_iter_end(iteration_end(c), s));
    if (stats) {
        const size_t kk = (size_t)done;  // the records of the iterations that ran
        if (stats->iters_run) *stats->iters_run = done;
        // every record into the page-locked staging, one synchronisation, then
        // into the caller's arrays
        struct Part {
            void* dst;
            const void* src;
            size_t n, at;
        } parts[9];
        int np = 0;
        size_t at = 0;
        auto add = [&](void* dst, const void* src, size_t n) {
            if (!dst || !n) return;
            parts[np++] = Part{dst, src, n, at};
            at += (n + 15) & ~(size_t)15;
        };
        add(stats->sigma, W.st_sigma, kk * 4);
        add(T > 0 ? stats->armijo_k : nullptr, W.st_k, kk * T * 4);
        add(stats->cgls_steps, W.st_steps, kk * 4);
        add(stats->cgls_resid, W.st_resid, kk * 8);
        add(f_ref ? stats->rmse : nullptr, W.st_rmse, kk * 8);
        add(T > 0 ? stats->armijo_q0 : nullptr, W.st_q0, kk * T * 8);
        add(T > 0 ? stats->armijo_q1 : nullptr, W.st_q1, kk * T * 8);
        const int M = q->cgls_iters;
        add(M > 0 ? stats->cgls_gamma : nullptr, W.st_gamma, kk * M * 8);
        add(M > 0 ? stats->cgls_delta : nullptr, W.st_delta, kk * M * 8);
        if (noalloc) {
            for (int i = 0; i < np; ++i)
                EPTV_HIP(hipMemcpyAsync(parts[i].dst, parts[i].src, parts[i].n, hipMemcpyDeviceToHost, s));
            EPTV_HIP(hipStreamSynchronize(s));
            return EPTV_OK;
        }
        std::lock_guard<std::mutex> hl(h->host_mu);
        void* hb = nullptr;
        EPTV_HIP(host_staging(h, std::max<size_t>(at, 16), &hb));
        for (int i = 0; i < np; ++i)
            EPTV_HIP(hipMemcpyAsync((char*)hb + parts[i].at, parts[i].src, parts[i].n, hipMemcpyDeviceToHost, s));
        EPTV_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < np; ++i) std::memcpy(parts[i].dst, (const char*)hb + parts[i].at, parts[i].n);
    }
    return EPTV_OK;
}

}  // namespace eptv

extern "C" {

int eptv_reconstruct(eptv_plan h, const eptv_params* q, const float* y, float* f, const float* f_ref, void* ws,
                     size_t ws_bytes, eptv_stats* stats, void* stream)
{
    return reconstruct_impl(h, q, y, f, f_ref, nullptr, nullptr, 0, nullptr, ws, ws_bytes, stats, stream, false);
}

int eptv_reconstruct_replay(eptv_plan h, const eptv_params* q, const float* y, float* f, const float* f_ref,
                            const int32_t* armijo_replay, void* ws, size_t ws_bytes, eptv_stats* stats,
                            void* stream)
{
    if (!armijo_replay) return EPTV_ERR_ARG;
    return reconstruct_impl(h, q, y, f, f_ref, nullptr, nullptr, 0, armijo_replay, ws, ws_bytes, stats, stream, false);
}

int eptv_reconstruct_weighted(eptv_plan h, const eptv_params* q, const float* y, float* f, const float* f_ref,
                              const float* wx, const float* wy, int frozen_iters, void* ws, size_t ws_bytes,
                              eptv_stats* stats, void* stream)
{
    if (!wx || !wy || frozen_iters < 0) return EPTV_ERR_ARG;
    return reconstruct_impl(h, q, y, f, f_ref, wx, wy, frozen_iters, nullptr, ws, ws_bytes, stats, stream, false);
}

}  // extern "C"
