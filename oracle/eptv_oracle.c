/*
 * eptv_oracle.c -- FP64 CPU oracle of the EPTV reconstruction path.
 *
 * TEST INFRASTRUCTURE (see eptv_oracle.h): a plain, slow, step-by-step
 * implementation of the paper's method used only to check the HIP library.
 * Every function names the passage of the paper it follows.  OpenMP is used
 * only on loops whose iterations write disjoint outputs; every sum runs in a
 * fixed sequential order, so results do not depend on the thread count.
 */
#include "eptv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
/* below this many independent outputs a loop runs on one thread */
#define ORC_PAR_MIN 16384

struct orc_matrix {
    orc_geometry g;    /* a copy, view angles included, for the Eq. 11 operator */
    double* angles;
    int nx, ny;
    int n_rows, n_cols;
    long long nnz;
    long long* rowptr; /* CSR over rays */
    int* col;
    double* val;
    long long* colptr; /* the same entries grouped by pixel (for P^T) */
    int* row;
    double* cval;
};

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the oracle's parallel loops from now on (n >= 1). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ geometry
 * Sec. 3 / App. III Eq. A6: view theta_v (equally spaced over a full turn
 * unless given), source at -SAD (cos theta, sin theta), ray b leaves the
 * source along theta + beta_b on an equiangular arc detector. */
static double view_angle(const orc_geometry* g, int v)
{
    return g->view_angles_rad ? g->view_angles_rad[v] : 2.0 * ORC_PI * v / g->n_views;
}

static double bin_angle(const orc_geometry* g, int b)
{
    return ((double)b - 0.5 * (g->n_bins - 1) + g->bin_offset) * g->dbeta_rad;
}

static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* Sec. 2.1, Eq. 1: p_ij = length of ray i inside pixel j, by Siddon's method:
 * clip the line to the image box, collect the parameters where it crosses the
 * vertical and horizontal grid lines, sort them, and give each piece between
 * consecutive parameters to the pixel that contains its midpoint.  Pixels are
 * half-open, [x_k, x_k + d) x [y_l, y_l + d), so a line lying exactly on a grid
 * line belongs to the pixels above / to the right of it. */
int orc_trace_ray(const orc_geometry* g, int v, int b, int cap, int* pix, double* len)
{
    const double d = g->pixel_mm;
    const double th = view_angle(g, v), be = bin_angle(g, b);
    const double sx = -g->sad_mm * cos(th), sy = -g->sad_mm * sin(th);
    const double dx = cos(th + be), dy = sin(th + be);
    const double x0 = -0.5 * g->nx * d, y0 = -0.5 * g->ny * d;
    const double x1 = x0 + g->nx * d, y1 = y0 + g->ny * d;
    double amin = -HUGE_VAL, amax = HUGE_VAL;

    if (dx != 0.0) {
        double a = (x0 - sx) / dx, c = (x1 - sx) / dx;
        amin = fmax(amin, fmin(a, c));
        amax = fmin(amax, fmax(a, c));
    } else if (!(sx >= x0 && sx < x1)) {
        return 0;
    }
    if (dy != 0.0) {
        double a = (y0 - sy) / dy, c = (y1 - sy) / dy;
        amin = fmax(amin, fmin(a, c));
        amax = fmin(amax, fmax(a, c));
    } else if (!(sy >= y0 && sy < y1)) {
        return 0;
    }
    if (!(amax > amin)) return 0;

    int na = 0;
    double* al = (double*)malloc(sizeof(double) * (size_t)(g->nx + g->ny + 4));
    al[na++] = amin;
    al[na++] = amax;
    if (dx != 0.0)
        for (int k = 0; k <= g->nx; ++k) {
            double a = (x0 + k * d - sx) / dx;
            if (a > amin && a < amax) al[na++] = a;
        }
    if (dy != 0.0)
        for (int k = 0; k <= g->ny; ++k) {
            double a = (y0 + k * d - sy) / dy;
            if (a > amin && a < amax) al[na++] = a;
        }
    qsort(al, (size_t)na, sizeof(double), cmp_double);

    int n = 0;
    for (int k = 0; k + 1 < na; ++k) {
        double l = al[k + 1] - al[k];
        if (!(l > 0.0)) continue;
        double mid = 0.5 * (al[k] + al[k + 1]);
        int i = (int)floor((sx + mid * dx - x0) / d);
        int j = (int)floor((sy + mid * dy - y0) / d);
        if (i < 0 || i >= g->nx || j < 0 || j >= g->ny) continue;
        int p = j * g->nx + i;
        if (n > 0 && pix[n - 1] == p) {
            len[n - 1] += l;
        } else if (n < cap) {
            pix[n] = p;
            len[n] = l;
            ++n;
        }
    }
    free(al);
    return n;
}

int orc_matrix_build(const orc_geometry* g, orc_matrix** out)
{
    if (!g || !out || g->nx <= 0 || g->ny <= 0 || g->n_views <= 0 || g->n_bins <= 0 ||
        !(g->pixel_mm > 0) || !(g->dbeta_rad > 0))
        return 1;
    const int nrow = g->n_views * g->n_bins, cap = g->nx + g->ny + 4;
    orc_matrix* m = (orc_matrix*)calloc(1, sizeof(orc_matrix));
    m->g = *g;
    m->angles = (double*)malloc(sizeof(double) * (size_t)g->n_views);
    for (int v = 0; v < g->n_views; ++v) m->angles[v] = view_angle(g, v);
    m->g.view_angles_rad = m->angles;
    m->nx = g->nx;
    m->ny = g->ny;
    m->n_rows = nrow;
    m->n_cols = g->nx * g->ny;
    int* cnt = (int*)calloc((size_t)nrow, sizeof(int));

#pragma omp parallel if (nrow > ORC_PAR_MIN)
    {
        int* pix = (int*)malloc(sizeof(int) * (size_t)cap);
        double* len = (double*)malloc(sizeof(double) * (size_t)cap);
#pragma omp for schedule(dynamic, 16)
        for (int r = 0; r < nrow; ++r)
            cnt[r] = orc_trace_ray(g, r / g->n_bins, r % g->n_bins, cap, pix, len);
        free(pix);
        free(len);
    }
    m->rowptr = (long long*)malloc(sizeof(long long) * (size_t)(nrow + 1));
    m->rowptr[0] = 0;
    for (int r = 0; r < nrow; ++r) m->rowptr[r + 1] = m->rowptr[r] + cnt[r];
    m->nnz = m->rowptr[nrow];
    m->col = (int*)malloc(sizeof(int) * (size_t)(m->nnz ? m->nnz : 1));
    m->val = (double*)malloc(sizeof(double) * (size_t)(m->nnz ? m->nnz : 1));
#pragma omp parallel for schedule(dynamic, 16) if (nrow > ORC_PAR_MIN)
    for (int r = 0; r < nrow; ++r)
        orc_trace_ray(g, r / g->n_bins, r % g->n_bins, cap, m->col + m->rowptr[r], m->val + m->rowptr[r]);

    /* Group the same entries by pixel, rows ascending, for P^T. */
    m->colptr = (long long*)calloc((size_t)m->n_cols + 1, sizeof(long long));
    for (long long e = 0; e < m->nnz; ++e) m->colptr[m->col[e] + 1]++;
    for (int c = 0; c < m->n_cols; ++c) m->colptr[c + 1] += m->colptr[c];
    long long* fill = (long long*)malloc(sizeof(long long) * (size_t)m->n_cols);
    memcpy(fill, m->colptr, sizeof(long long) * (size_t)m->n_cols);
    m->row = (int*)malloc(sizeof(int) * (size_t)(m->nnz ? m->nnz : 1));
    m->cval = (double*)malloc(sizeof(double) * (size_t)(m->nnz ? m->nnz : 1));
    for (int r = 0; r < nrow; ++r)
        for (long long e = m->rowptr[r]; e < m->rowptr[r + 1]; ++e) {
            long long at = fill[m->col[e]]++;
            m->row[at] = r;
            m->cval[at] = m->val[e];
        }
    free(fill);
    free(cnt);
    *out = m;
    return 0;
}

void orc_matrix_free(orc_matrix* m)
{
    if (!m) return;
    free(m->angles);
    free(m->rowptr);
    free(m->col);
    free(m->val);
    free(m->colptr);
    free(m->row);
    free(m->cval);
    free(m);
}

long long orc_matrix_nnz(const orc_matrix* m) { return m ? m->nnz : -1; }

int orc_matrix_csr(const orc_matrix* m, long long* rowptr, int* col, double* val)
{
    if (!m) return 1;
    memcpy(rowptr, m->rowptr, sizeof(long long) * (size_t)(m->n_rows + 1));
    memcpy(col, m->col, sizeof(int) * (size_t)m->nnz);
    memcpy(val, m->val, sizeof(double) * (size_t)m->nnz);
    return 0;
}

/* (P x)_i = sum_j p_ij x_j (Eq. 1). */
void orc_project(const orc_matrix* m, const double* x, double* q)
{
#pragma omp parallel for schedule(static) if (m->n_rows > ORC_PAR_MIN)
    for (int r = 0; r < m->n_rows; ++r) {
        double s = 0.0;
        for (long long e = m->rowptr[r]; e < m->rowptr[r + 1]; ++e) s += m->val[e] * x[m->col[e]];
        q[r] = s;
    }
}

/* (P^T r)_j = sum_i p_ij r_i: the transpose of the same matrix (below Eq. 6). */
void orc_backproject(const orc_matrix* m, const double* r, double* z)
{
#pragma omp parallel for schedule(static) if (m->n_cols > ORC_PAR_MIN)
    for (int c = 0; c < m->n_cols; ++c) {
        double s = 0.0;
        for (long long e = m->colptr[c]; e < m->colptr[c + 1]; ++e) s += m->cval[e] * r[m->row[e]];
        z[c] = s;
    }
}

/* Eq. 11 (derived in App. III): the pixel-driven backprojector of the paper's
 * on-the-fly strategy.  For pixel centre p and view theta, with the source at
 * S = -SAD (cos theta, sin theta):
 *   l     = |p - S|, the source-to-pixel distance;
 *   beta* = the angle of p - S measured from the central ray (counter-clockwise
 *           positive, the sense in which the bin angles grow);
 *   y(beta*) = linear interpolation between the two bins whose centre angles
 *           bracket beta*, a bin beyond the detector reading zero;
 * and [P^T y](p) = (d^2 / dbeta) * sum over views of y(beta*) / l.  It is a
 * smooth approximation of the transpose above, not its exact transpose. */
void orc_backproject_interp(const orc_geometry* g, const double* y, double* z)
{
    const double d = g->pixel_mm, scale = d * d / g->dbeta_rad;
    const int nx = g->nx, ny = g->ny, B = g->n_bins;
#pragma omp parallel for schedule(static) if (nx * ny > ORC_PAR_MIN)
    for (int c = 0; c < nx * ny; ++c) {
        const double px = (c % nx + 0.5 - 0.5 * nx) * d, py = (c / nx + 0.5 - 0.5 * ny) * d;
        double acc = 0.0;
        for (int v = 0; v < g->n_views; ++v) {
            const double th = view_angle(g, v);
            const double ex = cos(th), ey = sin(th);
            const double rx = px + g->sad_mm * ex, ry = py + g->sad_mm * ey; /* p - S */
            const double l = sqrt(rx * rx + ry * ry);
            const double bstar = atan2(ex * ry - ey * rx, ex * rx + ey * ry);
            /* fractional bin index: bin b is centred on beta_b of bin_angle() */
            const double t = bstar / g->dbeta_rad + 0.5 * (B - 1) - g->bin_offset;
            const double b0 = floor(t), a = t - b0;
            const int k = (int)b0;
            const double y0 = (k >= 0 && k < B) ? y[(size_t)v * B + k] : 0.0;
            const double y1 = (k + 1 >= 0 && k + 1 < B) ? y[(size_t)v * B + k + 1] : 0.0;
            acc += ((1.0 - a) * y0 + a * y1) / l;
        }
        z[c] = scale * acc;
    }
}

/* ------------------------------------------------------------------ TV terms
 * App. II, Eq. A3.  f is extended by zeros outside the image (the zero
 * boundary condition assumed below Eq. A1).  x-edge (i+1/2, j):
 *   TV = sqrt( (f[i+1,j]-f[i,j])^2 + 1/2 (m[j+1]-m[j])^2 + 1/2 (m[j]-m[j-1])^2 + eps^2 ),
 *   m[k] = (f[i+1,k] + f[i,k]) / 2 ;
 * y-edges are the same with the roles of i and j exchanged. */
static double px(const double* f, int nx, int ny, int i, int j)
{
    return (i < 0 || i >= nx || j < 0 || j >= ny) ? 0.0 : f[(size_t)j * nx + i];
}

static double tv_x(const double* f, int nx, int ny, int i, int j, double eps)
{
    double d = px(f, nx, ny, i + 1, j) - px(f, nx, ny, i, j);
    double m0 = 0.5 * (px(f, nx, ny, i + 1, j) + px(f, nx, ny, i, j));
    double mu = 0.5 * (px(f, nx, ny, i + 1, j + 1) + px(f, nx, ny, i, j + 1));
    double md = 0.5 * (px(f, nx, ny, i + 1, j - 1) + px(f, nx, ny, i, j - 1));
    return sqrt(d * d + 0.5 * (mu - m0) * (mu - m0) + 0.5 * (m0 - md) * (m0 - md) + eps * eps);
}

static double tv_y(const double* f, int nx, int ny, int i, int j, double eps)
{
    double d = px(f, nx, ny, i, j + 1) - px(f, nx, ny, i, j);
    double m0 = 0.5 * (px(f, nx, ny, i, j + 1) + px(f, nx, ny, i, j));
    double mr = 0.5 * (px(f, nx, ny, i + 1, j + 1) + px(f, nx, ny, i + 1, j));
    double ml = 0.5 * (px(f, nx, ny, i - 1, j + 1) + px(f, nx, ny, i - 1, j));
    return sqrt(d * d + 0.5 * (mr - m0) * (mr - m0) + 0.5 * (m0 - ml) * (m0 - ml) + eps * eps);
}

void orc_tv_edges(int nx, int ny, const double* f, double eps, double* tvx, double* tvy)
{
#pragma omp parallel for schedule(static) if ((long)nx * ny > ORC_PAR_MIN)
    for (int j = 0; j < ny; ++j)
        for (int i = -1; i < nx; ++i) tvx[(size_t)j * (nx + 1) + (i + 1)] = tv_x(f, nx, ny, i, j, eps);
#pragma omp parallel for schedule(static) if ((long)nx * ny > ORC_PAR_MIN)
    for (int j = -1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) tvy[(size_t)(j + 1) * nx + i] = tv_y(f, nx, ny, i, j, eps);
}

/* Eq. 5 on a half-edge: w = exp(-(TV/sigma)^2); sigma = +inf gives w = 1 (plain TV). */
static void weights(size_t n, const double* tv, double sigma, double* w)
{
    for (size_t e = 0; e < n; ++e) {
        double t = tv[e] / sigma;
        w[e] = exp(-t * t);
    }
}

static size_t n_xedges(int nx, int ny) { return (size_t)ny * (nx + 1); }
static size_t n_yedges(int nx, int ny) { return (size_t)(ny + 1) * nx; }

/* Eq. 4 discretised on the half-edges of Eq. A3: J_h = sum_e w_e TV_e. */
double orc_tv_energy(int nx, int ny, const double* f, double sigma, double eps)
{
    size_t ex = n_xedges(nx, ny), ey = n_yedges(nx, ny);
    double* tv = (double*)malloc(sizeof(double) * (ex + ey));
    double* w = (double*)malloc(sizeof(double) * (ex + ey));
    orc_tv_edges(nx, ny, f, eps, tv, tv + ex);
    weights(ex + ey, tv, sigma, w);
    double s = 0.0;
    for (size_t e = 0; e < ex + ey; ++e) s += w[e] * tv[e];
    free(tv);
    free(w);
    return s;
}

double orc_surrogate(int nx, int ny, const double* h, const double* v, double lambda,
                     const double* wx, const double* wy, double eps)
{
    size_t ex = n_xedges(nx, ny), ey = n_yedges(nx, ny);
    double* tvx = (double*)malloc(sizeof(double) * ex);
    double* tvy = (double*)malloc(sizeof(double) * ey);
    orc_tv_edges(nx, ny, h, eps, tvx, tvy);
    double fid = 0.0, tv = 0.0;
    for (size_t p = 0; p < (size_t)nx * ny; ++p) fid += (h[p] - v[p]) * (h[p] - v[p]);
    for (size_t e = 0; e < ex; ++e) tv += wx[e] * tvx[e];
    for (size_t e = 0; e < ey; ++e) tv += wy[e] * tvy[e];
    free(tvx);
    free(tvy);
    return 0.5 * lambda * fid + tv;
}

/* Eq. 9 with the variation of Eq. 10 approximated by Eq. A2:
 *   g_ij = lambda (f_ij - v_ij)
 *          - [ w_{i+1/2,j} (f_{i+1,j}-f_ij)/TV_{i+1/2,j} - w_{i-1/2,j} (f_ij-f_{i-1,j})/TV_{i-1/2,j} ]
 *          - [ w_{i,j+1/2} (f_{i,j+1}-f_ij)/TV_{i,j+1/2} - w_{i,j-1/2} (f_ij-f_{i,j-1})/TV_{i,j-1/2} ]
 * with the weights and magnitudes of Eq. A3 taken at f. */
static void gradient_with(int nx, int ny, const double* f, const double* v, double lambda,
                          const double* tvx, const double* tvy, const double* wx, const double* wy,
                          double* g)
{
#pragma omp parallel for schedule(static) if ((long)nx * ny > ORC_PAR_MIN)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double c = px(f, nx, ny, i, j);
            size_t xr = (size_t)j * (nx + 1) + (i + 1), xl = xr - 1;
            size_t yu = (size_t)(j + 1) * nx + i, yd = (size_t)j * nx + i;
            double fxr = wx[xr] * (px(f, nx, ny, i + 1, j) - c) / tvx[xr];
            double fxl = wx[xl] * (c - px(f, nx, ny, i - 1, j)) / tvx[xl];
            double fyu = wy[yu] * (px(f, nx, ny, i, j + 1) - c) / tvy[yu];
            double fyd = wy[yd] * (c - px(f, nx, ny, i, j - 1)) / tvy[yd];
            size_t p = (size_t)j * nx + i;
            g[p] = lambda * (c - v[p]) - (fxr - fxl) - (fyu - fyd);
        }
}

void orc_tv_gradient(int nx, int ny, const double* f, const double* v, double lambda,
                     double sigma, double eps, double* g, double* wx_out, double* wy_out)
{
    size_t ex = n_xedges(nx, ny), ey = n_yedges(nx, ny);
    double* tvx = (double*)malloc(sizeof(double) * ex);
    double* tvy = (double*)malloc(sizeof(double) * ey);
    double* wx = (double*)malloc(sizeof(double) * ex);
    double* wy = (double*)malloc(sizeof(double) * ey);
    orc_tv_edges(nx, ny, f, eps, tvx, tvy);
    weights(ex, tvx, sigma, wx);
    weights(ey, tvy, sigma, wy);
    gradient_with(nx, ny, f, v, lambda, tvx, tvy, wx, wy, g);
    if (wx_out) memcpy(wx_out, wx, sizeof(double) * ex);
    if (wy_out) memcpy(wy_out, wy, sizeof(double) * ey);
    free(tvx);
    free(tvy);
    free(wx);
    free(wy);
}

/* Vector-Jacobian product of the descent direction g(f) of Eq. 9 / Eq. A2
 * with respect to f, out = (dg/df)^T u, for differentiating through P2 steps
 * (sigma and the step sizes held constant).  Write g = lambda (f - v) +
 * sum_e F_e (e_B - e_A) over half-edges e from pixel A to pixel B, with
 * F_e = w(TV) d / TV, d = f_B - f_A, TV = sqrt(d^2 + t1^2/2 + t2^2/2 + eps^2),
 * t1, t2 the differences of the pair means of Eq. A3 and w = exp(-TV^2/s^2).
 * Then dF/dd = w/TV - c d, dF/dt1 = -c t1/2, dF/dt2 = -c t2/2 with
 * c = w d (1/TV + 2 TV/s^2) / TV^2, and each edge adds (u_B - u_A) times the
 * derivative of F_e to every pixel F_e depends on.  Ghost pixels (outside
 * the image) carry no entry. */
static void vjp_add(double* out, int nx, int ny, int i, int j, double c)
{
    if (i >= 0 && i < nx && j >= 0 && j < ny) out[(size_t)j * nx + i] += c;
}

static void vjp_edge(int nx, int ny, const double* f, const double* u, double sigma, double eps, int ax, int ay,
                     int bx, int by, int px_, int py_, double* out)
{
    /* A = (ax, ay), B = (bx, by); (px_, py_) is the unit step across the edge
     * direction (the "up" pair of an x-edge, the "right" pair of a y-edge). */
    const double fa = px(f, nx, ny, ax, ay), fb = px(f, nx, ny, bx, by);
    const double d = fb - fa, m0 = 0.5 * (fa + fb);
    const double mu = 0.5 * (px(f, nx, ny, ax + px_, ay + py_) + px(f, nx, ny, bx + px_, by + py_));
    const double md = 0.5 * (px(f, nx, ny, ax - px_, ay - py_) + px(f, nx, ny, bx - px_, by - py_));
    const double t1 = mu - m0, t2 = m0 - md;
    const double tv = sqrt(d * d + 0.5 * t1 * t1 + 0.5 * t2 * t2 + eps * eps);
    const double r = tv / sigma, w = exp(-r * r);
    const double c = w * d * (1.0 / tv + 2.0 * tv / (sigma * sigma)) / (tv * tv);
    const double ub = px(u, nx, ny, bx, by), ua = px(u, nx, ny, ax, ay), ue = ub - ua;
    const double dd = ue * (w / tv - c * d), d1 = ue * (-0.5 * c * t1), d2 = ue * (-0.5 * c * t2);
    /* d = fB - fA */
    vjp_add(out, nx, ny, bx, by, dd);
    vjp_add(out, nx, ny, ax, ay, -dd);
    /* t1 = (f(A+p) + f(B+p))/2 - (fA + fB)/2 */
    vjp_add(out, nx, ny, ax + px_, ay + py_, 0.5 * d1);
    vjp_add(out, nx, ny, bx + px_, by + py_, 0.5 * d1);
    vjp_add(out, nx, ny, ax, ay, -0.5 * d1);
    vjp_add(out, nx, ny, bx, by, -0.5 * d1);
    /* t2 = (fA + fB)/2 - (f(A-p) + f(B-p))/2 */
    vjp_add(out, nx, ny, ax, ay, 0.5 * d2);
    vjp_add(out, nx, ny, bx, by, 0.5 * d2);
    vjp_add(out, nx, ny, ax - px_, ay - py_, -0.5 * d2);
    vjp_add(out, nx, ny, bx - px_, by - py_, -0.5 * d2);
}

void orc_tv_gradient_vjp(int nx, int ny, const double* f, double lambda, double sigma, double eps,
                         const double* u, double* out)
{
    for (size_t p = 0; p < (size_t)nx * ny; ++p) out[p] = lambda * u[p];
    for (int j = 0; j < ny; ++j)
        for (int i = -1; i < nx; ++i) vjp_edge(nx, ny, f, u, sigma, eps, i, j, i + 1, j, 0, 1, out);
    for (int j = -1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) vjp_edge(nx, ny, f, u, sigma, eps, i, j, i, j + 1, 1, 0, out);
}

/* Sec. 2.1: sigma from the distribution of gradient magnitudes, a fixed share
 * of them lying above it.  Order statistic of rank ceil(q n) - 1 (0-based,
 * ascending) over all n half-edge magnitudes, by a full sort. */
double orc_select_sigma(int nx, int ny, const double* f, double eps, double q, double sigma_floor)
{
    size_t ex = n_xedges(nx, ny), ey = n_yedges(nx, ny), n = ex + ey;
    double* tv = (double*)malloc(sizeof(double) * n);
    orc_tv_edges(nx, ny, f, eps, tv, tv + ex);
    qsort(tv, n, sizeof(double), cmp_double);
    long long k = (long long)ceil(q * (double)n) - 1;
    if (k < 0) k = 0;
    if (k > (long long)n - 1) k = (long long)n - 1;
    double s = tv[k];
    free(tv);
    return s > sigma_floor ? s : sigma_floor;
}

/* ------------------------------------------------------------------ P2
 * Sec. 2.2: gradient descent on Q(f) = lambda/2 ||f - v||^2 + J(f), direction
 * g of Eq. 9, step by Armijo backtracking t = t0 shrink^k until
 * Q(f - t g) <= Q(f) - c t ||g||^2, the weights recomputed at every step
 * (EPTV algorithm, step 2) and held fixed inside the line search. */
/* The same descent with given half-edge weights in place of Eq. 5's
 * w = exp(-TV^2 / sigma^2) (NULL: the adaptive weights). */
/* With replay (NULL: search), step s takes the given backtrack index
 * instead of searching (-1: no step), and margin_out[s] certifies it against
 * this function's own inequality: the smaller of (thr - Q_k)/|Q0| for the
 * replayed index and (Q_j - thr_j)/|Q0| for every earlier index j (all of
 * them when the index is -1) -- non-negative when the search would have made
 * the same decision, negative by how much it would not. */
static int tv_step_with(int nx, int ny, const orc_params* p, double* f, const double* v, double sigma, int n_steps,
                        int* k_out, double* margin_out, double* sigma_out, const double* wx_in, const double* wy_in,
                        const int* replay, double* q0_out, double* q1_out);

int orc_tv_step(int nx, int ny, const orc_params* p, double* f, const double* v,
                double sigma, int n_steps, int* k_out, double* margin_out, double* sigma_out)
{
    return tv_step_with(nx, ny, p, f, v, sigma, n_steps, k_out, margin_out, sigma_out, NULL, NULL, NULL, NULL, NULL);
}

/* q0_out / q1_out (may be NULL): Q at each step's start and at the accepted
 * point (Q at the start again when no step is taken). */
static int tv_step_with(int nx, int ny, const orc_params* p, double* f, const double* v, double sigma, int n_steps,
                        int* k_out, double* margin_out, double* sigma_out, const double* wx_in, const double* wy_in,
                        const int* replay, double* q0_out, double* q1_out)
{
    size_t np = (size_t)nx * ny, ex = n_xedges(nx, ny), ey = n_yedges(nx, ny);
    if (sigma < 0 && !wx_in) sigma = orc_select_sigma(nx, ny, f, p->tv_eps, p->edge_quantile, p->sigma_floor);
    if (sigma_out) *sigma_out = sigma;
    double* tvx = (double*)malloc(sizeof(double) * ex);
    double* tvy = (double*)malloc(sizeof(double) * ey);
    double* wx = (double*)malloc(sizeof(double) * ex);
    double* wy = (double*)malloc(sizeof(double) * ey);
    double* g = (double*)malloc(sizeof(double) * np);
    double* h = (double*)malloc(sizeof(double) * np);
    const double t0 = p->armijo_t0 > 0 ? p->armijo_t0 : 1.0 / p->lambda;

    for (int s = 0; s < n_steps; ++s) {
        orc_tv_edges(nx, ny, f, p->tv_eps, tvx, tvy);
        if (wx_in) {
            memcpy(wx, wx_in, sizeof(double) * ex);
            memcpy(wy, wy_in, sizeof(double) * ey);
        } else {
            weights(ex, tvx, sigma, wx);
            weights(ey, tvy, sigma, wy);
        }
        gradient_with(nx, ny, f, v, p->lambda, tvx, tvy, wx, wy, g);
        double q0 = orc_surrogate(nx, ny, f, v, p->lambda, wx, wy, p->tv_eps);
        double gg = 0.0;
        for (size_t i = 0; i < np; ++i) gg += g[i] * g[i];

        int acc = -1;
        double margin = HUGE_VAL, t = t0, q_acc = q0;
        const double scale = fabs(q0) > 0 ? fabs(q0) : 1.0;
        if (replay) {
            /* the given decision, certified against every trial the search would make */
            const int kr = replay[s];
            const int last = kr >= 0 ? kr : p->armijo_max_backtracks;
            for (int k = 0; k <= last; ++k) {
                for (size_t i = 0; i < np; ++i) h[i] = f[i] - t * g[i];
                double qk = orc_surrogate(nx, ny, h, v, p->lambda, wx, wy, p->tv_eps);
                double thr = q0 - p->armijo_c * t * gg;
                double cert = (k == kr ? thr - qk : qk - thr) / scale;
                if (cert < margin) margin = cert;
                if (k == kr) {
                    q_acc = qk;
                    break;
                }
                t *= p->armijo_shrink;
            }
            acc = kr;
        } else {
            for (int k = 0; k <= p->armijo_max_backtracks; ++k) {
                for (size_t i = 0; i < np; ++i) h[i] = f[i] - t * g[i];
                double qk = orc_surrogate(nx, ny, h, v, p->lambda, wx, wy, p->tv_eps);
                double thr = q0 - p->armijo_c * t * gg;
                double rel = fabs(qk - thr) / scale;
                if (rel < margin) margin = rel;
                if (qk <= thr) {
                    acc = k;
                    q_acc = qk;
                    break;
                }
                t *= p->armijo_shrink;
            }
        }
        if (acc >= 0) memcpy(f, h, sizeof(double) * np);
        if (k_out) k_out[s] = acc;
        if (margin_out) margin_out[s] = margin;
        if (q0_out) q0_out[s] = q0;
        if (q1_out) q1_out[s] = q_acc;
    }
    free(tvx);
    free(tvy);
    free(wx);
    free(wy);
    free(g);
    free(h);
    return 0;
}

/* ------------------------------------------------------------------ P1
 * App. I: CGLS on min ||P u - y||^2 started from the given u:
 *   r = y - P u, s = P^T r; repeat: a = ||P^T r||^2 / ||P s||^2, u += a s,
 *   r -= a P s, b = ||P^T r_new||^2 / ||P^T r||^2, s = P^T r_new + b s.
 * Stops early when ||P s|| = 0 or ||P^T r||^2 <= 1e-30 of its initial value. */
static double dot(size_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void backproject_with(const orc_matrix* m, int interp, const double* r, double* z)
{
    if (interp)
        orc_backproject_interp(&m->g, r, z);
    else
        orc_backproject(m, r, z);
}

static int cgls_rec(const orc_matrix* m, int interp_bp, const double* y, double* u, int iters, double* resid,
                    double* gamma_out, double* delta_out);

int orc_cgls_with(const orc_matrix* m, int interp_bp, const double* y, double* u, int iters, double* resid)
{
    return cgls_rec(m, interp_bp, y, u, iters, resid, NULL, NULL);
}

/* gamma_out / delta_out (may be NULL, iters entries): ||P^T r||^2 at the top
 * of every step reached and ||P s||^2 of every step that formed it; 0 for
 * the entries after a breakdown. */
static int cgls_rec(const orc_matrix* m, int interp_bp, const double* y, double* u, int iters, double* resid,
                    double* gamma_out, double* delta_out)
{
    size_t nr = (size_t)m->n_rows, nc = (size_t)m->n_cols;
    double* r = (double*)malloc(sizeof(double) * nr);
    double* q = (double*)malloc(sizeof(double) * nr);
    double* s = (double*)malloc(sizeof(double) * nc);
    double* z = (double*)malloc(sizeof(double) * nc);
    orc_project(m, u, q);
    for (size_t i = 0; i < nr; ++i) r[i] = y[i] - q[i];
    backproject_with(m, interp_bp, r, z);
    memcpy(s, z, sizeof(double) * nc);
    double gam = dot(nc, z, z), gam0 = gam;
    int steps = 0;
    for (int it = 0; it < iters; ++it) {
        if (gamma_out) gamma_out[it] = 0.0;
        if (delta_out) delta_out[it] = 0.0;
    }
    for (int it = 0; it < iters; ++it) {
        if (gamma_out) gamma_out[it] = gam;
        if (!(gam > 1e-30 * gam0)) break;
        orc_project(m, s, q);
        double del = dot(nr, q, q);
        if (delta_out) delta_out[it] = del;
        if (!(del > 0.0)) break;
        double a = gam / del;
        for (size_t i = 0; i < nc; ++i) u[i] += a * s[i];
        for (size_t i = 0; i < nr; ++i) r[i] -= a * q[i];
        backproject_with(m, interp_bp, r, z);
        double gnew = dot(nc, z, z);
        double b = gnew / gam;
        for (size_t i = 0; i < nc; ++i) s[i] = z[i] + b * s[i];
        gam = gnew;
        ++steps;
    }
    if (resid) *resid = dot(nr, r, r);
    free(r);
    free(q);
    free(s);
    free(z);
    return steps;
}

int orc_cgls(const orc_matrix* m, const double* y, double* u, int iters, double* resid)
{
    return orc_cgls_with(m, 0, y, u, iters, resid);
}

/* ------------------------------------------------------------------ outer loop
 * The EPTV algorithm of Sec. 2.2: from f^(0) = 0, repeat
 *   1. v = argmin ||P f - y||^2 by CGLS started at f^(k)   (or, with zero CGLS
 *      steps, the gradient form of Eq. 8: v = f - mu/lambda P^T (P f - y));
 *      P^T is the transpose, or with interp_bp the Eq. 11 operator in its
 *      place, as the paper's on-the-fly code does (Sec. 2.3);
 *   2. P2 by gradient descent from v (or f^(k)), sigma chosen once from the
 *      P2 start image, weights updated at every descent step;
 *   3. negative pixels set to zero.
 * With given half-edge weights, the first frozen_iters iterations use them in
 * P2 in place of Eq. 5 (no sigma is chosen there). */
int orc_reconstruct(const orc_matrix* m, const orc_params* p, const double* y, double* f,
                    const double* f_ref, orc_stats* st)
{
    return orc_reconstruct_weighted(m, p, y, f, f_ref, st, NULL, NULL, 0);
}

static int reconstruct_impl(const orc_matrix* m, const orc_params* p, const double* y, double* f,
                            const double* f_ref, orc_stats* st, const double* wx_in, const double* wy_in,
                            int frozen_iters, const int* replay);

int orc_reconstruct_weighted(const orc_matrix* m, const orc_params* p, const double* y, double* f,
                             const double* f_ref, orc_stats* st, const double* wx_in, const double* wy_in,
                             int frozen_iters)
{
    return reconstruct_impl(m, p, y, f, f_ref, st, wx_in, wy_in, frozen_iters, NULL);
}

int orc_reconstruct_replay(const orc_matrix* m, const orc_params* p, const double* y, double* f,
                           const double* f_ref, orc_stats* st, const int* armijo_replay)
{
    if (!armijo_replay) return 1;
    return reconstruct_impl(m, p, y, f, f_ref, st, NULL, NULL, 0, armijo_replay);
}

static int reconstruct_impl(const orc_matrix* m, const orc_params* p, const double* y, double* f,
                            const double* f_ref, orc_stats* st, const double* wx_in, const double* wy_in,
                            int frozen_iters, const int* replay)
{
    if (!m || !p || !y || !f || p->outer_iters < 0 || p->tv_iters < 0 || p->cgls_iters < 0) return 1;
    const int nx = m->nx, ny = m->ny, T = p->tv_iters;
    size_t nc = (size_t)m->n_cols, nr = (size_t)m->n_rows;
    double* v = (double*)malloc(sizeof(double) * nc);
    double* w = (double*)malloc(sizeof(double) * nc);
    double* q = (double*)malloc(sizeof(double) * nr);
    if (p->zero_init) memset(f, 0, sizeof(double) * nc);

    for (int k = 0; k < p->outer_iters; ++k) {
        /* step 1 */
        memcpy(v, f, sizeof(double) * nc);
        double resid = 0.0;
        int steps = 0;
        if (p->cgls_iters > 0) {
            const size_t at = (size_t)k * p->cgls_iters;
            steps = cgls_rec(m, p->interp_bp, y, v, p->cgls_iters, &resid,
                             st && st->cgls_gamma ? st->cgls_gamma + at : NULL,
                             st && st->cgls_delta ? st->cgls_delta + at : NULL);
        } else {
            orc_project(m, f, q);
            for (size_t i = 0; i < nr; ++i) q[i] -= y[i];
            backproject_with(m, p->interp_bp, q, w);
            for (size_t i = 0; i < nc; ++i) v[i] = f[i] - (p->mu / p->lambda) * w[i];
            orc_project(m, v, q);
            for (size_t i = 0; i < nr; ++i) resid += (y[i] - q[i]) * (y[i] - q[i]);
        }
        /* step 2 */
        memcpy(w, p->p2_start ? f : v, sizeof(double) * nc);
        const int frozen = wx_in && wy_in && k < frozen_iters;
        double sigma = p->sigma_fixed;
        if (frozen)
            sigma = -1.0; /* recorded as -1: no sigma, the given weights replace Eq. 5 */
        else if (sigma < 0)
            sigma = orc_select_sigma(nx, ny, w, p->tv_eps, p->edge_quantile, p->sigma_floor);
        tv_step_with(nx, ny, p, w, v, sigma, T, st && st->armijo_k ? st->armijo_k + (size_t)k * T : NULL,
                     st && st->armijo_margin ? st->armijo_margin + (size_t)k * T : NULL, NULL,
                     frozen ? wx_in : NULL, frozen ? wy_in : NULL, replay ? replay + (size_t)k * T : NULL,
                     st && st->armijo_q0 ? st->armijo_q0 + (size_t)k * T : NULL,
                     st && st->armijo_q1 ? st->armijo_q1 + (size_t)k * T : NULL);
        /* step 3 */
        if (p->positivity)
            for (size_t i = 0; i < nc; ++i)
                if (w[i] < 0.0) w[i] = 0.0;
        memcpy(f, w, sizeof(double) * nc);

        if (st) {
            if (st->sigma) st->sigma[k] = sigma;
            if (st->cgls_steps) st->cgls_steps[k] = steps;
            if (st->cgls_resid) st->cgls_resid[k] = resid;
            if (st->energy && p->track_energy) {
                orc_project(m, f, q);
                double dd = 0.0;
                for (size_t i = 0; i < nr; ++i) dd += (q[i] - y[i]) * (q[i] - y[i]);
                st->energy[k] = 0.5 * p->mu * dd + orc_tv_energy(nx, ny, f, sigma, p->tv_eps);
            }
            if (st->rmse && f_ref) {
                double e = 0.0;
                for (size_t i = 0; i < nc; ++i) e += (f[i] - f_ref[i]) * (f[i] - f_ref[i]);
                st->rmse[k] = sqrt(e / (double)nc);
            }
        }
    }
    free(v);
    free(w);
    free(q);
    return 0;
}
