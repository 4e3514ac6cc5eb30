// plan.cpp -- host side of libeptv: geometry tables, workspace layout, the
// enqueue of one outer iteration, graph capture and the C ABI of eptv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "eptv_internal.h"

struct eptv_plan_s {
    eptv::Plan p;
    std::mutex graph_mu;
};

namespace eptv {

static thread_local std::string g_last_error;

static int hip_fail(hipError_t e, const char* what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return EPTV_ERR_HIP;
}

#define EPTV_HIP(call)                                   \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------------------ geometry
// Ray (v, b) leaves the source s_v = -SAD (cos theta_v, sin theta_v) along
// theta_v + beta_b (Sec. 3 scanner; App. III Eq. A6).  Its sweep form is
// computed in double precision and stored in 32.32 fixed point (see RayTable).
struct HostRay {
    long long E0, S;
    float w32, wfull;
    bool rows;
    int k_lo, k_hi;
};

static long long to_fixed(double e) { return std::llround(std::ldexp(e, 32)); }

static HostRay make_ray(const Plan& p, double theta, double beta)
{
    const double d = p.pixel;
    const double c = std::cos(theta + beta), s = std::sin(theta + beta);
    const double sx = -p.sad * std::cos(theta), sy = -p.sad * std::sin(theta);
    const double x0 = -0.5 * p.nx * d, y0 = -0.5 * p.ny * d;
    HostRay R;
    double e0, slope;
    int ncross, nsweep;
    if (std::fabs(c) >= std::fabs(s)) {  // swept column by column
        e0 = (sy + (x0 - sx) * s / c - y0) / d;
        slope = s / c;
        R.w32 = s != 0.0 ? (float)std::ldexp(d / std::fabs(s), -32) : 0.0f;
        R.wfull = (float)(d / std::fabs(c));
        R.rows = false;
        ncross = p.ny;
        nsweep = p.nx;
    } else {  // swept row by row
        e0 = (sx + (y0 - sy) * c / s - x0) / d;
        slope = c / s;
        R.w32 = c != 0.0 ? (float)std::ldexp(d / std::fabs(c), -32) : 0.0f;
        R.wfull = (float)(d / std::fabs(s));
        R.rows = true;
        ncross = p.nx;
        nsweep = p.ny;
    }
    R.E0 = to_fixed(e0);
    R.S = to_fixed(slope);
    // Sweep cells whose entry/exit coordinates can touch [0, ncross), widened
    // far beyond the fixed-point rounding of e.
    const double delta = std::ldexp(1.0, -18) * (p.nx + p.ny + 2);
    if (R.S == 0) {
        const double e = std::ldexp((double)R.E0, -32);
        const bool in = e >= -delta && e < ncross + delta;
        R.k_lo = 0;
        R.k_hi = in ? nsweep : 0;
    } else {
        double ka = (-delta - e0) / slope, kb = (ncross + delta - e0) / slope;
        double lo = std::floor(std::min(ka, kb)) - 1.0, hi = std::ceil(std::max(ka, kb)) + 1.0;
        lo = std::min(std::max(lo, 0.0), (double)nsweep);
        hi = std::min(std::max(hi, 0.0), (double)nsweep);
        R.k_lo = (int)lo;
        R.k_hi = std::max((int)hi, R.k_lo);
    }
    return R;
}

// Nonzeros of the float32 matrix, from the same fixed-point cell bounds the
// kernels use.
static long long count_nnz(const HostRay& R, const Plan& p)
{
    const int ncross = R.rows ? p.nx : p.ny;
    long long n = 0;
    for (int k = R.k_lo; k < R.k_hi; ++k) {
        const long long ea = R.E0 + (long long)k * R.S, eb = ea + R.S;
        const long long lo = std::min(ea, eb), hi = std::max(ea, eb);
        const int m0 = (int)(lo >> 32), m1 = (int)(hi >> 32);
        const bool in0 = m0 >= 0 && m0 < ncross, in1 = m1 >= 0 && m1 < ncross;
        if (R.S == 0 || m0 == m1) {
            n += in0 && (R.S == 0 || hi > lo);
        } else {
            n += in0;
            n += in1 && (unsigned)hi != 0u;
        }
    }
    return n;
}

static int validate_geometry(const eptv_geometry* g)
{
    if (!g) return EPTV_ERR_ARG;
    if (g->nx <= 0 || g->ny <= 0 || g->n_views <= 0 || g->n_bins <= 0) return EPTV_ERR_ARG;
    if (g->nx > 32768 || g->ny > 32768 || (long long)g->n_views * g->n_bins > (1LL << 30)) return EPTV_ERR_ARG;
    if (!(g->pixel_mm > 0) || !std::isfinite(g->pixel_mm)) return EPTV_ERR_GEOMETRY;
    if (!(g->dbeta_rad > 0) || !std::isfinite(g->dbeta_rad) || !std::isfinite(g->bin_offset))
        return EPTV_ERR_GEOMETRY;
    const double half_diag = 0.5 * g->pixel_mm * std::sqrt((double)g->nx * g->nx + (double)g->ny * g->ny);
    if (!(g->sad_mm > half_diag * (1.0 + 1e-6)) || !std::isfinite(g->sad_mm)) return EPTV_ERR_GEOMETRY;
    if (!(g->sdd_mm >= g->sad_mm)) return EPTV_ERR_GEOMETRY;
    const double edge = (0.5 * (g->n_bins - 1) + std::fabs(g->bin_offset)) * g->dbeta_rad;
    if (!(edge < 0.5 * M_PI)) return EPTV_ERR_GEOMETRY;  // every ray must point into the half-plane ahead
    if (g->view_angles_rad)
        for (int v = 0; v < g->n_views; ++v)
            if (!std::isfinite(g->view_angles_rad[v])) return EPTV_ERR_GEOMETRY;
    return EPTV_OK;
}

// ------------------------------------------------------------------ workspace
static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static int partial_count(const Plan& p)
{
    const int img = image_tile_blocks(p);
    int n = project_blocks(p);
    n = std::max(n, img);
    n = std::max(n, 2 * img);
    n = std::max(n, kArmijoCand * armijo_blocks(p));
    n = std::max(n, (int)(((size_t)p.V * p.B + 1023) / 1024));
    n = std::max(n, 256);
    return n;
}

size_t workspace_layout(const Plan& p, int K, int T, char* base, Workspace* w)
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
    W.wx = (float*)take((size_t)p.ny * (p.nx + 1) * 4);
    W.wy = (float*)take((size_t)(p.ny + 1) * p.nx * 4);
    W.r = (float*)take(ns * 4);
    W.q = (float*)take(ns * 4);
    W.keys = (uint32_t*)take(n_edges(p) * 4);
    W.hist = (uint32_t*)take(3 * kSelectBins * 4);
    W.part = (double*)take((size_t)partial_count(p) * 8);
    W.st = (DevState*)take(sizeof(DevState));
    W.st_sigma = (float*)take(kcap * 4);
    W.st_k = (int32_t*)take(ktcap * 4);
    W.st_steps = (int32_t*)take(kcap * 4);
    W.st_resid = (double*)take(kcap * 8);
    W.st_rmse = (double*)take(kcap * 8);
    W.bytes = off;
    return off;
}

static int check_params(const eptv_params* q)
{
    if (!q) return EPTV_ERR_ARG;
    if (q->outer_iters < 0 || q->cgls_iters < 0 || q->cgls_iters > kMaxCgls || q->tv_iters < 0) return EPTV_ERR_ARG;
    if (q->tv_iters > 0 && !(q->lambda > 0)) return EPTV_ERR_ARG;
    if (q->cgls_iters == 0 && !(q->mu >= 0 && q->lambda > 0)) return EPTV_ERR_ARG;
    if (q->sigma_fixed < 0 && !(q->edge_quantile > 0 && q->edge_quantile <= 1)) return EPTV_ERR_ARG;
    if (std::isnan(q->sigma_fixed) || !(q->tv_eps >= 0) || !(q->sigma_floor > 0)) return EPTV_ERR_ARG;
    if (q->tv_iters > 0 && (!(q->armijo_shrink > 0 && q->armijo_shrink < 1) || q->armijo_max_backtracks < 0 ||
                            q->armijo_max_backtracks > 4096 || !(q->armijo_c >= 0)))
        return EPTV_ERR_ARG;
    if ((long long)q->outer_iters * q->tv_iters > (1LL << 28)) return EPTV_ERR_ARG;
    return EPTV_OK;
}

static uint32_t select_rank(const Plan& p, double q)
{
    const double n = (double)n_edges(p);
    long long k = (long long)std::ceil(q * n) - 1;
    k = std::max(0LL, std::min(k, (long long)n - 1));
    return (uint32_t)k;
}

struct Ctx {
    const Plan& p;
    Workspace& W;
    const eptv_params& q;
    const float* y;
    float* f;
    const float* f_ref;
};

static float t0_of(const eptv_params& q)
{
    return (float)(q.armijo_t0 > 0 ? q.armijo_t0 : 1.0 / q.lambda);
}

// sigma from the half-edge magnitudes of `img` (radix select, three digits).
static hipError_t enqueue_select(const Plan& p, Workspace& W, const float* img, float eps2, float floor_,
                                 hipStream_t s)
{
    hipError_t e;
    if ((e = launch_edges_hist(p, img, eps2, W.keys, W.hist, s)) != hipSuccess) return e;
    if ((e = launch_select_finalize(W.st, 0, W.hist, floor_, s)) != hipSuccess) return e;
    for (int pass = 1; pass <= 2; ++pass) {
        if ((e = launch_select_hist(p, pass, W.keys, W.st, W.hist + pass * kSelectBins, s)) != hipSuccess) return e;
        if ((e = launch_select_finalize(W.st, pass, W.hist + pass * kSelectBins, floor_, s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// One P2 descent step from fcur into fout (Sec. 2.2; Armijo line search).
static hipError_t enqueue_gd_step(const Plan& p, Workspace& W, const eptv_params& q, const float* fcur,
                                  const float* v, float* fout, float* foutT, int clamp, int step, int T,
                                  int32_t* st_k, hipStream_t s)
{
    hipError_t e;
    const float eps2 = (float)(q.tv_eps * q.tv_eps);
    const int nb = armijo_blocks(p);
    if ((e = launch_tv_grad(p, fcur, v, (float)q.lambda, W.st, 0.0f, eps2, W.g, W.wx, W.wy, W.part, s)) !=
        hipSuccess)
        return e;
    if ((e = launch_grad_finalize(W.st, W.part, nb, s)) != hipSuccess) return e;
    const int npass = (q.armijo_max_backtracks + kArmijoCand) / kArmijoCand;
    const float t0 = t0_of(q);
    for (int pass = 0; pass < npass; ++pass) {
        if ((e = launch_armijo(p, pass, fcur, W.g, v, W.wx, W.wy, (float)q.lambda, eps2, t0, (float)q.armijo_shrink,
                               W.st, W.part, s)) != hipSuccess)
            return e;
        if ((e = launch_armijo_finalize(W.st, W.part, nb, pass, q.armijo_max_backtracks, q.armijo_c, t0,
                                        q.armijo_shrink, s)) != hipSuccess)
            return e;
    }
    return launch_p2_update(p, W.st, fcur, W.g, fout, foutT, clamp, st_k, step, T, s);
}

// One outer iteration of the EPTV algorithm (Sec. 2.2), entirely on `s`.
static hipError_t enqueue_iteration(const Ctx& c, hipStream_t s)
{
    const Plan& p = c.p;
    Workspace& W = c.W;
    const eptv_params& q = c.q;
    const int M = q.cgls_iters, T = q.tv_iters;
    const bool adaptive = q.sigma_fixed < 0;
    hipError_t e;
    if ((e = launch_state_init(W.st, W.hist, select_rank(p, q.edge_quantile), adaptive ? -1.0f : (float)q.sigma_fixed,
                               0, s)) != hipSuccess)
        return e;
    // Step 1: P1.  r = y - P f
    if ((e = launch_project(p, c.f, W.fT, -1.0f, 1.0f, c.y, W.r, nullptr, s)) != hipSuccess) return e;
    if (M > 0) {
        const int nbp = image_tile_blocks(p), npj = project_blocks(p);
        // s = P^T r, gamma_0
        if ((e = launch_backproject(p, W.r, 1.0f, 0.0f, nullptr, W.s, W.sT, W.part, s)) != hipSuccess) return e;
        if ((e = launch_cgls_gamma(W.st, W.part, nbp, 0, s)) != hipSuccess) return e;
        for (int m = 0; m < M; ++m) {
            const bool last = m == M - 1;
            if ((e = launch_project(p, W.s, W.sT, 1.0f, 0.0f, nullptr, W.q, W.part, s)) != hipSuccess) return e;
            if ((e = launch_cgls_delta(W.st, W.part, npj, m, s)) != hipSuccess) return e;
            if ((e = launch_cgls_axpy(p, W.st, m, m == 0 ? c.f : W.u, W.u, W.s, W.r, W.q, last ? W.part : nullptr,
                                      s)) != hipSuccess)
                return e;
            if (last) {
                const int nsb = (int)(((size_t)p.V * p.B + 1023) / 1024);
                if ((e = launch_cgls_resid(W.st, W.part, nsb, s)) != hipSuccess) return e;
                break;  // P^T r of the final residual is not needed
            }
            if ((e = launch_backproject(p, W.r, 1.0f, 0.0f, nullptr, W.z, nullptr, W.part, s)) != hipSuccess)
                return e;
            if ((e = launch_cgls_gamma(W.st, W.part, nbp, m + 1, s)) != hipSuccess) return e;
            if ((e = launch_cgls_supdate(p, W.st, m, W.z, W.s, W.sT, s)) != hipSuccess) return e;
        }
    } else {
        // gradient form of Eq. 8: v = f - mu/lambda P^T (P f - y)
        if ((e = launch_backproject(p, W.r, 1.0f, 0.0f, nullptr, W.z, nullptr, nullptr, s)) != hipSuccess) return e;
        if ((e = launch_gd_p1(p, c.f, W.z, (float)(q.mu / q.lambda), W.u, s)) != hipSuccess) return e;
    }
    // Step 2: P2 from v (or f^(k)), sigma chosen once from the start image.
    const float* start = q.p2_start ? c.f : W.u;
    if (adaptive && T > 0) {
        if ((e = enqueue_select(p, W, start, (float)(q.tv_eps * q.tv_eps), (float)q.sigma_floor, s)) != hipSuccess)
            return e;
    }
    if (T == 0) {
        if ((e = launch_copy_clamp(p, start, c.f, W.fT, q.positivity, s)) != hipSuccess) return e;
    }
    for (int t = 0; t < T; ++t) {
        const bool last = t == T - 1;
        // Step 3 (positivity) is fused into the last descent update.
        if ((e = enqueue_gd_step(p, W, q, t == 0 ? start : c.f, W.u, c.f, last ? W.fT : nullptr,
                                 last && q.positivity, t, T, W.st_k, s)) != hipSuccess)
            return e;
    }
    if (c.f_ref) {
        if ((e = launch_rmse_part(p, c.f, c.f_ref, W.part, s)) != hipSuccess) return e;
    }
    return launch_iter_end(W.st, W.part, (double)p.nx * p.ny, c.f_ref != nullptr, W.st_sigma, W.st_steps,
                           W.st_resid, W.st_rmse, s);
}

static bool no_graph()
{
    const char* v = std::getenv("EPTV_NO_GRAPH");
    return v && *v && std::strcmp(v, "0") != 0;
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
    p.nx = geom->nx;
    p.ny = geom->ny;
    p.V = geom->n_views;
    p.B = geom->n_bins;
    p.pixel = geom->pixel_mm;
    p.dbeta = geom->dbeta_rad;
    p.bin_offset = geom->bin_offset;
    p.sad = geom->sad_mm;
    p.sdd = geom->sdd_mm;
    p.angles.resize(p.V);
    for (int v = 0; v < p.V; ++v)
        p.angles[v] = geom->view_angles_rad ? geom->view_angles_rad[v] : 2.0 * M_PI * v / p.V;

    std::vector<longlong2> fx((size_t)p.V * p.B);
    std::vector<float2> wt((size_t)p.V * p.B);
    std::vector<int2> range((size_t)p.V * p.B);
    std::vector<float2> view(p.V);
    long long nnz = 0;
    for (int v = 0; v < p.V; ++v) {
        view[v] = make_float2((float)std::cos(p.angles[v]), (float)std::sin(p.angles[v]));
        for (int b = 0; b < p.B; ++b) {
            const double beta = ((double)b - 0.5 * (p.B - 1) + p.bin_offset) * p.dbeta;
            const HostRay R = make_ray(p, p.angles[v], beta);
            const size_t id = (size_t)v * p.B + b;
            fx[id].x = R.E0;
            fx[id].y = R.S;
            wt[id] = make_float2(R.w32, R.rows ? -R.wfull : R.wfull);
            range[id] = make_int2(R.k_lo, R.k_hi);
            nnz += count_nnz(R, p);
        }
    }
    p.nnz = nnz;
    hipError_t e = hipGetDevice(&p.device);
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_fx, fx.size() * sizeof(longlong2));
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_w, wt.size() * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_range, range.size() * sizeof(int2));
    if (e == hipSuccess) e = hipMalloc(&p.rays.d_view, view.size() * sizeof(float2));
    if (e == hipSuccess) e = hipMemcpy(p.rays.d_fx, fx.data(), fx.size() * sizeof(longlong2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p.rays.d_w, wt.data(), wt.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p.rays.d_range, range.data(), range.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p.rays.d_view, view.data(), view.size() * sizeof(float2), hipMemcpyHostToDevice);
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
    if (p.gexec) hipGraphExecDestroy(p.gexec);
    if (p.cap_stream) hipStreamDestroy(p.cap_stream);
    if (p.rays.d_fx) hipFree(p.rays.d_fx);
    if (p.rays.d_w) hipFree(p.rays.d_w);
    if (p.rays.d_range) hipFree(p.rays.d_range);
    if (p.rays.d_view) hipFree(p.rays.d_view);
    delete h;
    return EPTV_OK;
}

int eptv_plan_nnz(eptv_plan h, long long* nnz)
{
    if (!h || !nnz) return EPTV_ERR_ARG;
    *nnz = h->p.nnz;
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
    *bytes = workspace_layout(h->p, K, T, nullptr, nullptr);
    return EPTV_OK;
}

static int bind_ws(const Plan& p, int K, int T, void* ws, size_t ws_bytes, Workspace* W)
{
    if (!ws || ((uintptr_t)ws & 255)) return EPTV_ERR_WORKSPACE;
    const size_t need = workspace_layout(p, K, T, (char*)ws, W);
    return ws_bytes >= need ? EPTV_OK : EPTV_ERR_WORKSPACE;
}

int eptv_project(eptv_plan h, const float* x, float* q, float alpha, float beta, void* ws, size_t ws_bytes,
                 void* stream)
{
    if (!h || !x || !q) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, ws, ws_bytes, &W);
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

int eptv_backproject(eptv_plan h, const float* r, float* z, float alpha, float beta, void* ws, size_t ws_bytes,
                     void* stream)
{
    if (!h || !r || !z) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    EPTV_HIP(launch_backproject(h->p, r, alpha, beta, z, z, nullptr, nullptr, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_tv_gradient(eptv_plan h, const float* f, const float* v, float lambda, float sigma, float tv_eps, float* g,
                     float* wx, float* wy, void* ws, size_t ws_bytes, void* stream)
{
    if (!h || !f || !v || !g) return EPTV_ERR_ARG;
    if (!(sigma > 0) || !(tv_eps >= 0) || !std::isfinite(lambda)) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    EPTV_HIP(launch_tv_grad(h->p, f, v, lambda, nullptr, sigma, tv_eps * tv_eps, g, wx, wy, nullptr,
                            (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_select_sigma(eptv_plan h, const float* f, double q, float tv_eps, float sigma_floor, float* sigma_out,
                      void* ws, size_t ws_bytes, void* stream)
{
    if (!h || !f || !sigma_out) return EPTV_ERR_ARG;
    if (!(q > 0 && q <= 1) || !(tv_eps >= 0) || !(sigma_floor > 0)) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, ws, ws_bytes, &W);
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
        q->armijo_max_backtracks > 4096 || !(q->tv_eps >= 0) || !(q->sigma_floor > 0))
        return EPTV_ERR_ARG;
    if (sigma < 0 && !(q->edge_quantile > 0 && q->edge_quantile <= 1)) return EPTV_ERR_ARG;
    Workspace W;
    int rc = bind_ws(h->p, 1, 0, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Plan& p = h->p;
    EPTV_HIP(launch_state_init(W.st, W.hist, select_rank(p, q->edge_quantile), sigma < 0 ? -1.0f : sigma, 1, s));
    if (sigma < 0) EPTV_HIP(enqueue_select(p, W, f, (float)(q->tv_eps * q->tv_eps), (float)q->sigma_floor, s));
    for (int t = 0; t < n_steps; ++t)
        EPTV_HIP(enqueue_gd_step(p, W, *q, f, v, f, nullptr, 0, t, n_steps, W.st_k, s));
    if (stats) {
        if (stats->sigma) EPTV_HIP(hipMemcpyAsync(stats->sigma, &W.st->sigma, 4, hipMemcpyDeviceToHost, s));
        if (stats->armijo_k && n_steps > 0)
            EPTV_HIP(hipMemcpyAsync(stats->armijo_k, W.st_k, (size_t)n_steps * 4, hipMemcpyDeviceToHost, s));
        EPTV_HIP(hipStreamSynchronize(s));
    }
    return EPTV_OK;
}

int eptv_reconstruct(eptv_plan h, const eptv_params* q, const float* y, float* f, const float* f_ref, void* ws,
                     size_t ws_bytes, eptv_stats* stats, void* stream)
{
    if (!h || !y || !f) return EPTV_ERR_ARG;
    int rc = check_params(q);
    if (rc != EPTV_OK) return rc;
    Plan& p = h->p;
    Workspace W;
    rc = bind_ws(p, q->outer_iters, q->tv_iters, ws, ws_bytes, &W);
    if (rc != EPTV_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int K = q->outer_iters, T = q->tv_iters;

    EPTV_HIP(launch_state_init(W.st, W.hist, select_rank(p, q->edge_quantile), -1.0f, 1, s));
    if (q->zero_init) EPTV_HIP(launch_fill(f, (size_t)p.nx * p.ny, 0.0f, s));
    EPTV_HIP(launch_transpose(f, W.fT, p.nx, p.ny, s));

    Ctx c{p, W, *q, y, f, f_ref};
    if (K > 0) {
        if (no_graph()) {
            for (int k = 0; k < K; ++k) EPTV_HIP(enqueue_iteration(c, s));
        } else {
            std::lock_guard<std::mutex> lock(h->graph_mu);
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
            const void* ptrs[5] = {ws, y, f, f_ref, (const void*)(uintptr_t)ws_bytes};
            put(ptrs, sizeof ptrs);
            if (!p.gexec || key != p.gkey) {
                if (p.gexec) {
                    hipGraphExecDestroy(p.gexec);
                    p.gexec = nullptr;
                }
                hipGraph_t graph = nullptr;
                EPTV_HIP(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
                hipError_t e = enqueue_iteration(c, p.cap_stream);
                hipError_t e2 = hipStreamEndCapture(p.cap_stream, &graph);
                if (e != hipSuccess) {
                    if (graph) hipGraphDestroy(graph);
                    return hip_fail(e, "enqueue_iteration (capture)");
                }
                if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
                e = hipGraphInstantiate(&p.gexec, graph, nullptr, nullptr, 0);
                hipGraphDestroy(graph);
                if (e != hipSuccess) {
                    p.gexec = nullptr;
                    return hip_fail(e, "hipGraphInstantiate");
                }
                p.gkey = key;
            }
            for (int k = 0; k < K; ++k) EPTV_HIP(hipGraphLaunch(p.gexec, s));
        }
    }
    if (stats) {
        const size_t kk = (size_t)K;
        if (kk) {
            if (stats->sigma) EPTV_HIP(hipMemcpyAsync(stats->sigma, W.st_sigma, kk * 4, hipMemcpyDeviceToHost, s));
            if (stats->armijo_k && T > 0)
                EPTV_HIP(hipMemcpyAsync(stats->armijo_k, W.st_k, kk * T * 4, hipMemcpyDeviceToHost, s));
            if (stats->cgls_steps)
                EPTV_HIP(hipMemcpyAsync(stats->cgls_steps, W.st_steps, kk * 4, hipMemcpyDeviceToHost, s));
            if (stats->cgls_resid)
                EPTV_HIP(hipMemcpyAsync(stats->cgls_resid, W.st_resid, kk * 8, hipMemcpyDeviceToHost, s));
            if (stats->rmse && f_ref) EPTV_HIP(hipMemcpyAsync(stats->rmse, W.st_rmse, kk * 8, hipMemcpyDeviceToHost, s));
        }
        EPTV_HIP(hipStreamSynchronize(s));
    }
    return EPTV_OK;
}

}  // extern "C"
