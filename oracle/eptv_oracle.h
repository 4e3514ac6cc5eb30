/*
 * eptv_oracle.h -- FP64 CPU oracle of the EPTV fan-beam reconstruction path.
 *
 * TEST INFRASTRUCTURE.  This library is the plain, slow, obviously-correct
 * reference the HIP path is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does.  It shares no code, header, table or helper with the HIP
 * library.
 *
 * What it computes (paper: "GPU-based Low Dose CT Reconstruction via
 * Edge-preserving Total Variation Regularization", Tian et al.):
 *   - P: the fan-beam system matrix whose entry p_ij is the length of ray i
 *     inside pixel j (Sec. 2.1, Eq. 1), traced with Siddon's parametric method
 *     and stored explicitly (the paper's look-up-table strategy, Sec. 2.3);
 *   - P^T: the transpose of that matrix (Sec. 2.2, below Eq. 6), and the
 *     paper's pixel-driven interpolating backprojector (Eq. 11, App. III);
 *   - the half-edge TV magnitudes and edge weights (Eq. 5; App. II Eq. A3),
 *     the EPTV variation by the symmetric difference scheme (App. II Eq. A2)
 *     and the P2 descent direction (Eq. 9);
 *   - sigma as an order statistic of the edge magnitudes (Sec. 2.1);
 *   - CGLS for P1 (App. I), gradient descent with Armijo backtracking for P2
 *     (Sec. 2.2), the positivity truncation and the outer loop (the EPTV
 *     algorithm of Sec. 2.2).
 *
 * Arrays: image [ny][nx] (x fastest), sinogram [n_views][n_bins] (bin fastest),
 * x-edge magnitudes [ny][nx+1] (edge (i+1/2, j) at column i+1, i = -1..nx-1),
 * y-edge magnitudes [ny+1][nx] (edge (i, j+1/2) at row j+1, j = -1..ny-1).
 * All host memory, double precision, owned by the caller.
 */
#ifndef EPTV_ORACLE_H
#define EPTV_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny;
    double pixel_mm;
    int n_views;
    const double* view_angles_rad; /* NULL: 2*pi*v/n_views */
    int n_bins;
    double dbeta_rad;
    double bin_offset;             /* in bins */
    double sad_mm, sdd_mm;
} orc_geometry;

typedef struct orc_matrix orc_matrix;

/* Build P for a geometry (Siddon traversal of every ray). 0 on success. */
int orc_matrix_build(const orc_geometry* g, orc_matrix** out);
void orc_matrix_free(orc_matrix* m);
long long orc_matrix_nnz(const orc_matrix* m);
/* Copy the CSR form (rows = rays v*n_bins+b, cols = pixels j*nx+i) out. */
int orc_matrix_csr(const orc_matrix* m, long long* rowptr, int* col, double* val);

/* One ray's (pixel, length) list in traversal order; returns the count (<= cap). */
int orc_trace_ray(const orc_geometry* g, int v, int b, int cap, int* pix, double* len);

void orc_project(const orc_matrix* m, const double* x, double* q);     /* q = P x   */
void orc_backproject(const orc_matrix* m, const double* r, double* z); /* z = P^T r */

/* z = the Eq. 11 pixel-driven interpolating backprojection of y (App. III). */
void orc_backproject_interp(const orc_geometry* g, const double* y, double* z);

/* Half-edge TV magnitudes of App. II Eq. A3 (+eps^2 under the root). */
void orc_tv_edges(int nx, int ny, const double* f, double eps, double* tvx, double* tvy);
/* J_h(f) = sum over all half-edges of w_e * TV_e, w_e = exp(-TV_e^2/sigma^2) (Eq. 4-5). */
double orc_tv_energy(int nx, int ny, const double* f, double sigma, double eps);
/* g = lambda (f - v) + A2 variation (Eq. 9, App. II Eq. A2), weights from f. */
void orc_tv_gradient(int nx, int ny, const double* f, const double* v, double lambda,
                     double sigma, double eps, double* g, double* wx, double* wy);
/* out = (dg/df)^T u for the g above, sigma held fixed (may be +inf). */
void orc_tv_gradient_vjp(int nx, int ny, const double* f, double lambda, double sigma, double eps,
                         const double* u, double* out);
/* Q(h) = lambda/2 ||h - v||^2 + sum_e w_e TV_e(h) with caller-frozen weights. */
double orc_surrogate(int nx, int ny, const double* h, const double* v, double lambda,
                     const double* wx, const double* wy, double eps);
/* sigma = max(order statistic of rank ceil(q n) - 1 of all edge magnitudes, floor). */
double orc_select_sigma(int nx, int ny, const double* f, double eps, double q, double sigma_floor);

typedef struct {
    int outer_iters;          /* K */
    int cgls_iters;           /* M; 0 selects the gradient-form P1 of Eq. 8 */
    int tv_iters;             /* GD steps per P2 */
    int zero_init;            /* 1: f^(0) = 0 */
    double mu, lambda;
    double edge_quantile;     /* q of the sigma order statistic */
    double sigma_fixed;       /* < 0: adaptive; otherwise used as is (may be +inf) */
    double sigma_floor;
    double tv_eps;
    double armijo_c, armijo_shrink, armijo_t0; /* t0 <= 0: 1/lambda */
    int armijo_max_backtracks;
    int p2_start;             /* 0: P2 starts at v, 1: at f^(k) */
    int positivity;
    int track_energy;         /* fill energy[] with E(f^(k+1)) */
    int interp_bp;            /* 1: P1 uses the Eq. 11 backprojector for P^T */
} orc_params;

typedef struct {              /* every pointer may be NULL */
    double* sigma;            /* [K] */
    int* armijo_k;            /* [K*T] accepted backtrack index, -1 = none */
    double* armijo_margin;    /* [K*T] min relative decision margin */
    double* energy;           /* [K] E = mu/2||Pf-y||^2 + J_h(f) */
    int* cgls_steps;          /* [K] */
    double* cgls_resid;       /* [K] ||y - P v||^2 at the end of P1 */
    double* rmse;             /* [K] vs f_ref when given */
    double* armijo_q0;        /* [K*T] Q at each descent step's start */
    double* armijo_q1;        /* [K*T] Q at the accepted point (= armijo_q0 when skipped) */
    double* cgls_gamma;       /* [K*M] ||P^T r_m||^2 of each CGLS step reached, else 0 */
    double* cgls_delta;       /* [K*M] ||P s_m||^2 of each step that computed it, else 0 */
} orc_stats;

/* CGLS on min ||P u - y||^2 from the given u (App. I). Returns steps run. */
int orc_cgls(const orc_matrix* m, const double* y, double* u, int iters, double* resid);
/* The same with the Eq. 11 backprojector in place of P^T when interp_bp. */
int orc_cgls_with(const orc_matrix* m, int interp_bp, const double* y, double* u, int iters, double* resid);

/* n GD steps of P2 from f (in/out) towards v; sigma < 0 selects it from f. */
int orc_tv_step(int nx, int ny, const orc_params* p, double* f, const double* v,
                double sigma, int n_steps, int* k_out, double* margin_out, double* sigma_out);

/* The outer EPTV loop. f is the warm start unless zero_init. */
int orc_reconstruct(const orc_matrix* m, const orc_params* p, const double* y, double* f,
                    const double* f_ref, orc_stats* st);
/* The same, with the half-edge weights wx_in [ny][nx+1], wy_in [ny+1][nx]
 * used in place of Eq. 5's weights during the first frozen_iters iterations. */
int orc_reconstruct_weighted(const orc_matrix* m, const orc_params* p, const double* y, double* f,
                             const double* f_ref, orc_stats* st, const double* wx_in, const double* wy_in,
                             int frozen_iters);

/* Replay mode: the outer loop with the Armijo decisions taken from
 * armijo_replay [K*T] (backtrack index per descent step, -1 = no step)
 * instead of searching; st->armijo_margin then certifies each decision
 * against this implementation's own inequality (>= 0: the search agrees;
 * negative: by how much, relative to |Q0|, it would not). */
int orc_reconstruct_replay(const orc_matrix* m, const orc_params* p, const double* y, double* f,
                           const double* f_ref, orc_stats* st, const int* armijo_replay);

int orc_num_threads(void);
/* Threads of the parallel loops from now on (OpenMP builds; n >= 1). */
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
