/*
 * The FP64 oracle built with the address and undefined-behaviour sanitizers
 * (tests/test_host_sanitizers.py) and run through every entry point of
 * eptv_oracle.h on small cases: ragged shapes, an odd bin count, a detector
 * offset, every reconstruct variant (CGLS and gradient-form P1, Eq. 11 in P1,
 * P2 from f^(k), fixed and infinite sigma, replay, given weights) with every
 * stats array requested.  Besides the sanitizers' own checks it asserts that
 * every output is finite and that the adjoint identity <Px, r> = <x, P^T r>
 * holds.  Exit status 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "eptv_oracle.h"

static int g_fail = 0;
#define CHECK(cond, msg)                                                  \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, msg); \
            ++g_fail;                                                     \
        }                                                                 \
    } while (0)

static unsigned long long g_state = 88172645463325252ULL;
static double urand(void) /* xorshift64, uniform in [0, 1) */
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

static int all_finite(const double* a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static orc_params defaults(int K)
{
    orc_params p;
    memset(&p, 0, sizeof p);
    p.outer_iters = K;
    p.cgls_iters = 3;
    p.tv_iters = 5;
    p.zero_init = 1;
    p.mu = 1.0;
    p.lambda = 1000.0;
    p.edge_quantile = 0.9;
    p.sigma_fixed = -1.0;
    p.sigma_floor = 1e-12;
    p.tv_eps = 1e-4;
    p.armijo_c = 1e-4;
    p.armijo_shrink = 0.5;
    p.armijo_t0 = 0.0;
    p.armijo_max_backtracks = 20;
    p.positivity = 1;
    return p;
}

typedef struct {
    double *sigma, *margin, *energy, *resid, *rmse, *q0, *q1, *gamma, *delta;
    int *k, *steps;
    orc_stats s;
} stats_buf;

static void stats_alloc(stats_buf* b, int K, int T, int M)
{
    const int KT = K * (T > 0 ? T : 1), KM = K * (M > 0 ? M : 1);
    b->sigma = calloc(K, sizeof(double));
    b->margin = calloc(KT, sizeof(double));
    b->energy = calloc(K, sizeof(double));
    b->resid = calloc(K, sizeof(double));
    b->rmse = calloc(K, sizeof(double));
    b->q0 = calloc(KT, sizeof(double));
    b->q1 = calloc(KT, sizeof(double));
    b->gamma = calloc(KM, sizeof(double));
    b->delta = calloc(KM, sizeof(double));
    b->k = calloc(KT, sizeof(int));
    b->steps = calloc(K, sizeof(int));
    orc_stats s = {b->sigma, b->k, b->margin, b->energy, b->steps, b->resid, b->rmse, b->q0, b->q1, b->gamma, b->delta};
    b->s = s;
}

static void stats_free(stats_buf* b)
{
    free(b->sigma);
    free(b->margin);
    free(b->energy);
    free(b->resid);
    free(b->rmse);
    free(b->q0);
    free(b->q1);
    free(b->gamma);
    free(b->delta);
    free(b->k);
    free(b->steps);
}

static void run_case(int nx, int ny, double pix, int V, int B, double sad, double offset, const char* name)
{
    orc_geometry g;
    g.nx = nx;
    g.ny = ny;
    g.pixel_mm = pix;
    g.n_views = V;
    g.view_angles_rad = NULL;
    g.n_bins = B;
    g.dbeta_rad = 2.0 * asin(0.5 * pix * sqrt((double)nx * nx + (double)ny * ny) / sad) / B;
    g.bin_offset = offset;
    g.sad_mm = sad;
    g.sdd_mm = 2.0 * sad;
    const size_t ni = (size_t)nx * ny, ns = (size_t)V * B;
    const size_t nex = (size_t)ny * (nx + 1), ney = (size_t)(ny + 1) * nx;

    orc_matrix* m = NULL;
    CHECK(orc_matrix_build(&g, &m) == 0 && m, "matrix build");
    const long long nnz = orc_matrix_nnz(m);
    long long* rowptr = malloc((ns + 1) * sizeof(long long));
    int* col = malloc((size_t)nnz * sizeof(int));
    double* val = malloc((size_t)nnz * sizeof(double));
    CHECK(orc_matrix_csr(m, rowptr, col, val) == 0, "csr export");
    CHECK(rowptr[ns] == nnz, "csr row pointer");
    int pixs[4096];
    double lens[4096];
    const int cnt = orc_trace_ray(&g, V / 2, B / 2, 4096, pixs, lens);
    CHECK(cnt == rowptr[(size_t)(V / 2) * B + B / 2 + 1] - rowptr[(size_t)(V / 2) * B + B / 2], "traced ray");

    double *x = malloc(ni * sizeof(double)), *r = malloc(ns * sizeof(double));
    double *q = malloc(ns * sizeof(double)), *z = malloc(ni * sizeof(double)), *zi = malloc(ni * sizeof(double));
    for (size_t i = 0; i < ni; ++i) x[i] = urand();
    for (size_t i = 0; i < ns; ++i) r[i] = urand() - 0.5;
    orc_project(m, x, q);
    orc_backproject(m, r, z);
    orc_backproject_interp(&g, r, zi);
    double lhs = 0, rhs = 0;
    for (size_t i = 0; i < ns; ++i) lhs += q[i] * r[i];
    for (size_t i = 0; i < ni; ++i) rhs += x[i] * z[i];
    CHECK(fabs(lhs - rhs) <= 1e-10 * (fabs(lhs) + 1.0), "adjoint identity");
    CHECK(all_finite(q, ns) && all_finite(z, ni) && all_finite(zi, ni), "operator outputs finite");

    /* P2 pieces */
    double *f = malloc(ni * sizeof(double)), *v = malloc(ni * sizeof(double)), *gr = malloc(ni * sizeof(double));
    double *wx = malloc(nex * sizeof(double)), *wy = malloc(ney * sizeof(double));
    double *tvx = malloc(nex * sizeof(double)), *tvy = malloc(ney * sizeof(double)), *vj = malloc(ni * sizeof(double));
    for (size_t i = 0; i < ni; ++i) {
        f[i] = 0.02 * urand();
        v[i] = f[i] + 1e-3 * (urand() - 0.5);
    }
    orc_tv_edges(nx, ny, f, 1e-4, tvx, tvy);
    const double J = orc_tv_energy(nx, ny, f, 0.01, 1e-4);
    orc_tv_gradient(nx, ny, f, v, 1000.0, 0.01, 1e-4, gr, wx, wy);
    orc_tv_gradient_vjp(nx, ny, f, 1000.0, 0.01, 1e-4, x, vj);
    orc_tv_gradient_vjp(nx, ny, f, 1000.0, INFINITY, 1e-4, x, vj);
    const double Q = orc_surrogate(nx, ny, f, v, 1000.0, wx, wy, 1e-4);
    const double sg = orc_select_sigma(nx, ny, f, 1e-4, 0.9, 1e-12);
    const double sg1 = orc_select_sigma(nx, ny, f, 1e-4, 1.0, 1e-12);
    CHECK(isfinite(J) && isfinite(Q) && sg > 0 && sg <= sg1, "tv scalars");
    CHECK(all_finite(tvx, nex) && all_finite(tvy, ney) && all_finite(gr, ni) && all_finite(wx, nex) &&
              all_finite(wy, ney) && all_finite(vj, ni),
          "tv arrays finite");
    orc_params pp = defaults(1);
    int kk[4];
    double mg[4], so;
    orc_tv_step(nx, ny, &pp, f, v, -1.0, 4, kk, mg, &so);
    orc_tv_step(nx, ny, &pp, f, v, INFINITY, 2, kk, mg, &so);
    CHECK(all_finite(f, ni), "tv step finite");

    /* CGLS, both backprojectors */
    double* u = calloc(ni, sizeof(double));
    double res = 0;
    const int st1 = orc_cgls(m, q, u, 5, &res);
    memset(u, 0, ni * sizeof(double));
    const int st2 = orc_cgls_with(m, 1, q, u, 3, &res);
    CHECK(st1 >= 1 && st2 >= 1 && all_finite(u, ni) && isfinite(res), "cgls");

    /* reconstructions */
    const int K = 3, T = 5, M = 3;
    double* y = malloc(ns * sizeof(double));
    orc_project(m, x, y);
    for (size_t i = 0; i < ns; ++i) y[i] *= 0.01;
    stats_buf sb;
    stats_alloc(&sb, K, T, M);
    for (int variant = 0; variant < 6; ++variant) {
        orc_params rp = defaults(K);
        rp.track_energy = 1;
        if (variant == 1) rp.cgls_iters = 0, rp.mu = 1.0;        /* gradient-form P1 */
        if (variant == 2) rp.interp_bp = 1;                      /* Eq. 11 in P1 */
        if (variant == 3) rp.p2_start = 1, rp.positivity = 0;    /* P2 from f^(k) */
        if (variant == 4) rp.sigma_fixed = INFINITY;             /* plain TV */
        if (variant == 5) rp.armijo_t0 = 0.512, rp.armijo_max_backtracks = 12; /* long searches */
        double* fr = calloc(ni, sizeof(double));
        CHECK(orc_reconstruct(m, &rp, y, fr, x, &sb.s) == 0, "reconstruct");
        CHECK(all_finite(fr, ni) && all_finite(sb.energy, K) && all_finite(sb.rmse, K), "reconstruct finite");
        if (variant == 0) {
            /* replay its own decisions, then given weights */
            int* rep = malloc((size_t)K * T * sizeof(int));
            memcpy(rep, sb.k, (size_t)K * T * sizeof(int));
            double* f2 = calloc(ni, sizeof(double));
            CHECK(orc_reconstruct_replay(m, &rp, y, f2, x, &sb.s, rep) == 0, "replay");
            int same = 1;
            for (size_t i = 0; i < ni; ++i) same &= f2[i] == fr[i];
            CHECK(same, "replay of its own decisions reproduces the run");
            double *wxi = malloc(nex * sizeof(double)), *wyi = malloc(ney * sizeof(double));
            for (size_t i = 0; i < nex; ++i) wxi[i] = urand();
            for (size_t i = 0; i < ney; ++i) wyi[i] = urand();
            memset(f2, 0, ni * sizeof(double));
            CHECK(orc_reconstruct_weighted(m, &rp, y, f2, x, &sb.s, wxi, wyi, 2) == 0, "weighted");
            CHECK(all_finite(f2, ni), "weighted finite");
            free(wxi);
            free(wyi);
            free(f2);
            free(rep);
        }
        free(fr);
    }
    stats_free(&sb);
    printf("%s: %d x %d, %d x %d, nnz %lld, threads %d\n", name, nx, ny, V, B, nnz, orc_num_threads());

    orc_matrix_free(m);
    free(rowptr);
    free(col);
    free(val);
    free(x);
    free(r);
    free(q);
    free(z);
    free(zi);
    free(f);
    free(v);
    free(gr);
    free(wx);
    free(wy);
    free(tvx);
    free(tvy);
    free(vj);
    free(u);
    free(y);
}

int main(void)
{
    run_case(8, 8, 1.0, 6, 24, 40.0, 0.0, "8x8");
    run_case(5, 7, 1.0, 7, 13, 30.0, 0.0, "5x7 odd bins");
    run_case(23, 17, 1.1, 9, 41, 120.0, 0.3, "23x17 offset");
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("oracle: all checks passed\n");
    return 0;
}
