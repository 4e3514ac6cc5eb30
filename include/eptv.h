/*
 * eptv.h -- C ABI of the MI355X (gfx950) EPTV fan-beam reconstruction library
 * (libeptv.so).
 *
 * The method is the edge-preserving total-variation (EPTV) reconstruction of
 * Tian, Jia, Yuan, Pan, Jiang, "GPU-based Low Dose CT Reconstruction via
 * Edge-preserving Total Variation Regularization":
 *
 *   minimise  mu/2 ||P f - y||^2 + sum_e w_e TV_e(f)   subject to f >= 0
 *
 * (Sec. 2.1, Eq. 2 and Eq. 4-5), solved by alternating a CGLS data step (P1,
 * App. I) and a gradient-descent EPTV step with Armijo line search (P2,
 * Sec. 2.2 Eq. 8-10 and App. II Eq. A2-A3), followed by positivity.
 *
 * Conventions shared by every call
 *   image     float32 [ny][nx], x fastest.  Pixel (i, j) is the square of side
 *             pixel_mm centred at ((i + 1/2 - nx/2) d, (j + 1/2 - ny/2) d);
 *             pixels are half-open, so a ray lying exactly on a grid line
 *             belongs to the pixel above / to the right of it.
 *   sinogram  float32 [n_views][n_bins], bin fastest.  View v has angle
 *             theta_v (default 2 pi v / n_views); its source sits at
 *             -sad_mm (cos theta_v, sin theta_v); bin b is the ray leaving the
 *             source along theta_v + beta_b, beta_b = (b - (n_bins-1)/2 +
 *             bin_offset) dbeta_rad (equiangular arc detector, Sec. 3).
 *   edges     x-edge magnitudes/weights [ny][nx+1]: entry [j][i+1] is the
 *             half-edge (i+1/2, j), i = -1..nx-1; y-edges [ny+1][nx]: entry
 *             [j+1][i] is (i, j+1/2), j = -1..ny-1.  Values outside the image
 *             are zero (the zero boundary condition of App. II).
 *   memory    every array argument is a device pointer on the current HIP
 *             device, owned by the caller, contiguous, 4-byte aligned (ws:
 *             256-byte aligned).  Structs and stats arrays are host memory.
 *   streams   `stream` is a hipStream_t (NULL = the default stream).  Every
 *             call only enqueues work on it and returns, except where a call
 *             says it synchronises.
 *   errors    every call returns an eptv_status; no call throws or aborts.
 *             Argument checks happen before anything is enqueued.
 */
#ifndef EPTV_H
#define EPTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EPTV_OK = 0,
    EPTV_ERR_ARG = 1,       /* null pointer, non-positive size, bad parameter */
    EPTV_ERR_GEOMETRY = 2,  /* source inside the image circle, dbeta <= 0 ... */
    EPTV_ERR_WORKSPACE = 3, /* workspace missing or smaller than required */
    EPTV_ERR_HIP = 4,       /* a HIP runtime call failed */
    EPTV_ERR_NONFINITE = 5  /* an input holds NaN or +-inf (only with eptv_params.check_finite) */
} eptv_status;

/* Scanner geometry (Sec. 3; App. III Eq. A6).  view_angles_rad is a host array
 * of n_views angles, or NULL for equally spaced views over a full turn.  The
 * image has at least 2 x 2 pixels (else EPTV_ERR_ARG).  The
 * source must lie outside the circle through the image corners, and the fan
 * (bin angles (b - (n_bins-1)/2 + bin_offset) dbeta_rad, one bin beyond each
 * end included) must stay within +-pi/2 of the central ray; otherwise
 * EPTV_ERR_GEOMETRY.  Pixel (i, j) is centred at
 * ((i + 1/2 - nx/2) pixel_mm, (j + 1/2 - ny/2) pixel_mm), the source of view
 * theta at -sad_mm (cos theta, sin theta), ray b along theta + beta_b. */
typedef struct {
    int nx, ny;
    double pixel_mm;
    int n_views;
    const double* view_angles_rad;
    int n_bins;
    double dbeta_rad;
    double bin_offset;
    double sad_mm, sdd_mm;
} eptv_geometry;

/* Solver parameters.  The paper fixes none of the counts or step constants;
 * each field names the passage it parameterises. */
typedef struct {
    int outer_iters;     /* K, outer iterations of the EPTV algorithm (Sec. 2.2) */
    int cgls_iters;      /* M, CGLS steps per P1 (App. I); 0 = gradient form of Eq. 8 */
    int tv_iters;        /* gradient-descent steps per P2 (Sec. 2.2) */
    int zero_init;       /* 1: f^(0) = 0 as in the algorithm; 0: f is a warm start */
    double mu;           /* data weight of Eq. 2 (used by the gradient form of P1) */
    double lambda;       /* splitting weight of Eq. 7-9 */
    double edge_quantile;/* sigma = this quantile of the half-edge magnitudes (Sec. 2.1) */
    double sigma_fixed;  /* < 0: adaptive sigma; otherwise used as is (+inf = plain TV) */
    double sigma_floor;  /* lower bound on the adaptive sigma */
    double tv_eps;       /* eps added under the root of Eq. A3 (mm^-1) */
    double armijo_c;     /* sufficient-decrease constant of the Armijo rule */
    double armijo_shrink;/* backtracking factor */
    double armijo_t0;    /* first trial step; <= 0 means 1/lambda */
    int armijo_max_backtracks;
    int p2_start;        /* 0: P2 starts at v (P1's output); 1: at f^(k) */
    int positivity;      /* 1: step 3 of the algorithm (f = max(f, 0)) */
    int stored_matrix;   /* 1: P and P^T from the matrix kept by eptv_plan_store_matrix
                            (the look-up-table strategy of Sec. 2.3); 0: on the fly;
                            2: P on the fly and P^T from the stored matrix (the same
                            float32 matrix either way, so P^T stays P's exact
                            transpose).  1 and 2 need the stored matrix (else
                            EPTV_ERR_ARG) */
    int interp_bp;       /* 1: P1 uses the Eq. 11 interpolating backprojector in place
                            of P^T (the paper's on-the-fly code, Sec. 2.3); 0: the
                            exact transpose */
    int check_every;     /* with stop_rmse > 0 and f_ref given: read the RMSE to f_ref
                            back after every check_every-th outer iteration (0 = 1) */
    double stop_rmse;    /* > 0: stop at the first checked iteration whose RMSE to
                            f_ref is <= stop_rmse (the paper's iteration count is
                            case-dependent, Sec. 2.2); 0: run outer_iters */
    int check_finite;    /* 1: before iterating, scan y (and the warm start f when
                            zero_init = 0) on the device and return EPTV_ERR_NONFINITE,
                            with nothing else enqueued and f untouched, if any value is
                            NaN or infinite (synchronises the stream once); 0: no scan */
} eptv_params;

/* Optional per-iteration records, host arrays filled when a call that takes
 * stats returns (that call synchronises its stream).  Any pointer may be NULL. */
typedef struct {
    float* sigma;        /* [K]   sigma used by each P2 */
    int32_t* armijo_k;   /* [K*T] accepted backtrack index per GD step, -1 = none */
    int32_t* cgls_steps; /* [K]   CGLS steps actually run (breakdown stops early) */
    double* cgls_resid;  /* [K]   ||y - P v||^2 at the end of each CGLS P1 */
    double* rmse;        /* [K]   root-mean-square difference to f_ref, if given */
    int32_t* iters_run;  /* [1]   outer iterations actually run (fewer than K after an
                            early stop); the arrays above hold that many entries */
    /* The Armijo energies of each GD step (Sec. 2.2): Q(h) = lambda/2 ||h - v||^2 +
     * sum_e w_e TV_e(h) with the step's weights, at the step's start point
     * (armijo_q0) and at the accepted point f - t g (armijo_q1; = armijo_q0 when
     * the step is skipped).  Sums in float64 of the float32 terms. */
    double* armijo_q0;   /* [K*T] */
    double* armijo_q1;   /* [K*T] */
    /* CGLS scalars of each P1 (App. I), step m = 0..M-1 of iteration k at
     * [k*M + m]: gamma_m = ||P^T r_m||^2 and delta_m = ||P s_m||^2 as the step
     * computed them; 0 for steps after a breakdown (delta_m is also 0 for the
     * step whose gamma_m stopped CGLS).  Empty for the gradient form of P1. */
    double* cgls_gamma;  /* [K*M] */
    double* cgls_delta;  /* [K*M] */
} eptv_stats;

typedef struct eptv_plan_s* eptv_plan;

/* Precompute the per-ray and per-view tables of a geometry on the current
 * device.  Allocates device memory; the plan owns it until eptv_plan_destroy.
 * A plan is immutable after creation and may be shared by several streams.
 * Sizes: 2 <= nx, ny <= 32768 and n_views x n_bins <= 2^30 (else
 * EPTV_ERR_ARG, checked before any device call); EPTV_ERR_GEOMETRY for a
 * scanner that cannot see the whole image (source inside the circle through
 * its corners, detector nearer than the source, a fan of 180 degrees or more,
 * non-finite values). */
int eptv_plan_create(const eptv_geometry* geom, eptv_plan* out);
int eptv_plan_destroy(eptv_plan plan);

/* Number of (ray, pixel) pairs with a positive intersection length, counted
 * on the host in double precision: the nonzeros of P (Sec. 2.1, Eq. 1). */
int eptv_plan_nnz(eptv_plan plan, long long* nnz);

/* The float32 system matrix of a geometry as the kernels evaluate it, in CSR
 * form by ray (row v*n_bins + b; columns j*nx + i; entries in the order the
 * ray sweeps the image), computed on the host: no GPU is needed.  Pass NULL
 * arrays to get *nnz only; otherwise rowptr holds n_views*n_bins + 1 entries
 * and col/val hold *nnz. */
int eptv_geometry_matrix(const eptv_geometry* geom, long long* nnz, long long* rowptr, int* col, float* val);

/* Store that matrix on the plan's device, by ray (CSR, for P) and by pixel
 * (CSC, for P^T), each ray and pixel padded to a multiple of 4 entries.  The
 * CSC copy takes 8 bytes per entry (index, length).  The CSR copy takes 6
 * (float32 length and a 16-bit index offset within a 128-entry chunk of the
 * ray, plus a 4-byte base per chunk) whenever every chunk's indices span at
 * most 65535, else 8 like the CSC copy (190 MB in all at 512^2 / 40 views x
 * 736 bins).  A ray swept row by row indexes the transposed image, so that its
 * entries lie along the fast axis of the image it reads.  Owned by the plan;
 * built once, later calls only report the size.  Synchronous.  EPTV_ERR_ARG
 * when a copy would hold 2^31 entries or more (int32 offsets); EPTV_ERR_HIP
 * when device memory runs out (nothing is kept then). */
int eptv_plan_store_matrix(eptv_plan plan, size_t* device_bytes);

/* The stored matrix's layout (EPTV_ERR_ARG if it is not stored): *csr_compact
 * 1 for the 6-byte CSR encoding, 0 for the 8-byte one; *csr_bytes and
 * *csc_bytes the device bytes of each copy with its offsets.  Any pointer may
 * be NULL. */
int eptv_plan_stored_layout(eptv_plan plan, int* csr_compact, size_t* csr_bytes, size_t* csc_bytes);

/* q = alpha P x + beta q and z = alpha P^T r + beta z from the stored matrix
 * (EPTV_ERR_ARG if it is not stored).  Same matrix as eptv_project /
 * eptv_backproject bit for bit; only the summation order differs.
 * eptv_project_stored transposes x into the workspace (ws: as for
 * eptv_project); eptv_project_stored_dual takes the transposed image xT
 * ([nx][ny]) from the caller, as eptv_project_dual does, and needs no
 * workspace. */
int eptv_project_stored(eptv_plan plan, const float* x, float* q, float alpha, float beta, void* ws,
                        size_t ws_bytes, void* stream);
int eptv_project_stored_dual(eptv_plan plan, const float* x, const float* xT, float* q, float alpha, float beta,
                             void* stream);
int eptv_backproject_stored(eptv_plan plan, const float* r, float* z, float alpha, float beta, void* stream);

/* Workspace bytes for the calls below (device memory the caller allocates and
 * passes as ws / ws_bytes; a smaller ws_bytes is EPTV_ERR_WORKSPACE).
 * params == NULL gives the size needed by eptv_project / eptv_backproject /
 * eptv_tv_gradient / eptv_select_sigma and by eptv_tv_step with up to 4096
 * steps; eptv_reconstruct needs the size for its params (the per-iteration
 * records grow with outer_iters * tv_iters).  Calls that run concurrently need
 * separate workspaces; the contents need no initialisation. */
int eptv_workspace_bytes(eptv_plan plan, const eptv_params* params, size_t* bytes);

/* q = alpha P x + beta q (Sec. 2.1 Eq. 1): p_ij is the exact length of ray i
 * inside pixel j.  x [ny][nx], q [n_views][n_bins]; beta == 0 never reads q.
 * ws: workspace of eptv_workspace_bytes(plan, NULL). */
int eptv_project(eptv_plan plan, const float* x, float* q, float alpha, float beta,
                 void* ws, size_t ws_bytes, void* stream);

/* eptv_project for callers that keep the image in both layouts: xT is the
 * same image stored transposed, [nx][ny] (y fastest).  Rays closer to the x
 * axis read xT, the others read x, so every wave reads contiguous memory.
 * Needs no workspace; launches the projector kernel only. */
int eptv_project_dual(eptv_plan plan, const float* x, const float* xT, float* q, float alpha, float beta,
                      void* stream);

/* z = alpha P^T r + beta z with P^T the exact transpose of eptv_project's P
 * (Sec. 2.2, below Eq. 6), computed pixel by pixel (Sec. 2.3) without atomics.
 * r [n_views][n_bins], z [ny][nx]; beta == 0 never reads z. */
int eptv_backproject(eptv_plan plan, const float* r, float* z, float alpha, float beta,
                     void* ws, size_t ws_bytes, void* stream);

/* z = alpha B r + beta z with B the pixel-driven interpolating backprojector
 * of Eq. 11 (App. III): per pixel and view, r is interpolated linearly in the
 * bin direction at the angle beta* of the ray through the pixel centre (bins
 * beyond the detector read zero), divided by the source-to-pixel distance l,
 * summed over views and scaled by pixel_mm^2 / dbeta_rad.  A smooth
 * approximation of P^T, not its exact transpose.  r [n_views][n_bins],
 * z [ny][nx]; beta == 0 never reads z.  Needs no workspace. */
int eptv_backproject_interp(eptv_plan plan, const float* r, float* z, float alpha, float beta, void* stream);

/* The P2 descent direction g = lambda (f - v) + (A2 variation of the EPTV
 * term) (Eq. 9-10, App. II Eq. A2) with the half-edge magnitudes and weights
 * w = exp(-TV^2 / sigma^2) of Eq. A3 / Eq. 5 taken at f.  sigma may be +inf
 * (w = 1).  wx [ny][nx+1] and wy [ny+1][nx] receive the weights (may be NULL). */
int eptv_tv_gradient(eptv_plan plan, const float* f, const float* v, float lambda, float sigma,
                     float tv_eps, float* g, float* wx, float* wy, void* ws, size_t ws_bytes,
                     void* stream);

/* out = (dg/df)^T u: the vector-Jacobian product of eptv_tv_gradient's g with
 * respect to f, sigma held fixed (Eq. 9 with the A2 variation; the weights of
 * Eq. 5 / A3 are differentiated along with the magnitudes).  For gradients
 * through unrolled descent steps; the product with respect to v is -lambda u.
 * tv_eps must be > 0 (the magnitudes are then differentiable everywhere).
 * f, u, out [ny][nx]; out must not alias f or u.  ws: workspace of
 * eptv_workspace_bytes(plan, NULL). */
int eptv_tv_gradient_vjp(eptv_plan plan, const float* f, const float* u, float lambda, float sigma, float tv_eps,
                         float* out, void* ws, size_t ws_bytes, void* stream);

/* sigma = max(order statistic of rank ceil(q n) - 1 (0-based, ascending) of
 * the n = ny(nx+1) + (ny+1)nx half-edge magnitudes of f, sigma_floor)
 * (Sec. 2.1: sigma set from the gradient-magnitude histogram).  Exact
 * selection on the float32 magnitudes.  Writes one float to the device
 * pointer sigma_out. */
int eptv_select_sigma(eptv_plan plan, const float* f, double q, float tv_eps, float sigma_floor,
                      float* sigma_out, void* ws, size_t ws_bytes, void* stream);

/* n_steps gradient-descent steps of P2 (Eq. 8) from f towards v, in place:
 * the weights are recomputed at each step and held fixed inside an Armijo
 * backtracking search t = t0 shrink^k, k = 0..max_backtracks, for the first
 * t with Q(f - t g) <= Q(f) - c t ||g||^2, Q(h) = lambda/2 ||h - v||^2 +
 * sum_e w_e TV_e(h); without such t the step is skipped.  sigma < 0 selects
 * sigma from f as eptv_select_sigma does (params->edge_quantile,
 * params->sigma_floor).  No positivity.  stats->sigma[0] and
 * stats->armijo_k[0..n_steps-1] are filled when given (synchronises). */
int eptv_tv_step(eptv_plan plan, const eptv_params* params, float* f, const float* v, float sigma,
                 int n_steps, void* ws, size_t ws_bytes, eptv_stats* stats, void* stream);

/* The EPTV algorithm (Sec. 2.2): from f^(0) = 0 (or the warm start in f),
 * params->outer_iters times: P1 by CGLS started at f^(k) (App. I), sigma
 * from the P2 start image, P2 by eptv_tv_step's descent, positivity; f holds
 * f^(K) on return.  y [n_views][n_bins] are the log-transformed data.
 * f_ref (may be NULL) is an image the per-iteration RMSE is measured
 * against.  The iteration's kernels are launched on the stream one by one;
 * with EPTV_GRAPH=1 in the environment one outer iteration is captured once
 * as a HIP graph and replayed instead (same results bit for bit; on MI355X
 * the direct launches are slightly faster while the host thread is idle). */
int eptv_reconstruct(eptv_plan plan, const eptv_params* params, const float* y, float* f,
                     const float* f_ref, void* ws, size_t ws_bytes, eptv_stats* stats, void* stream);

/* eptv_reconstruct with the Armijo decisions given: armijo_replay (host,
 * [K*T] backtrack indices in -1 .. armijo_max_backtracks, -1 = no step) is
 * taken instead of the search in every descent step (the line search of
 * Sec. 2.2 with a recorded outcome), e.g. to follow another implementation's
 * trajectory through near-ties.  EPTV_ERR_ARG for indices out of range. */
int eptv_reconstruct_replay(eptv_plan plan, const eptv_params* params, const float* y, float* f,
                            const float* f_ref, const int32_t* armijo_replay, void* ws, size_t ws_bytes,
                            eptv_stats* stats, void* stream);

/* eptv_reconstruct with given half-edge weights: during the first
 * frozen_iters outer iterations P2 uses wx [ny][nx+1] / wy [ny+1][nx]
 * (device, the layout of eptv_tv_gradient's weights) in place of Eq. 5's
 * w = exp(-TV^2/sigma^2), and no sigma is chosen (recorded as -1); later
 * iterations are the adaptive ones.  For starting the iteration from proposed
 * weights (e.g. a network's). */
int eptv_reconstruct_weighted(eptv_plan plan, const eptv_params* params, const float* y, float* f,
                              const float* f_ref, const float* wx, const float* wy, int frozen_iters, void* ws,
                              size_t ws_bytes, eptv_stats* stats, void* stream);

/* eptv_reconstruct for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same iteration and results, with the workspace taken from a fixed
 * device array of the library instead of a caller's buffer.  That array
 * (eptv_noalloc_scratch_bytes(), 32 MiB: a 512 x 512 image with thousands of
 * per-iteration records) exists once per GPU until the process ends; params
 * whose eptv_workspace_bytes exceed it are EPTV_ERR_WORKSPACE.  No call here
 * allocates: no hipMalloc, no page-locked staging, no graph (EPTV_GRAPH is
 * ignored; the kernels are launched one by one); stats are copied straight
 * into the caller's host arrays.  The current device must be the plan's.
 * Every call on one GPU shares its array: calls that overlap on one GPU
 * (several streams or threads) race and must be serialised by the caller. */
int eptv_reconstruct_noalloc(eptv_plan plan, const eptv_params* params, const float* y, float* f,
                             const float* f_ref, eptv_stats* stats, void* stream);
size_t eptv_noalloc_scratch_bytes(void);

/* Measurement aid, not part of the method: reads `bytes` of device memory at
 * buf once with 16-byte loads (buf and bytes multiples of 16), the rate a
 * read-only stream reaches, to set beside the stored-matrix products (which
 * mostly read).  sink: one device word, written only in a case no real buffer
 * produces (it keeps the loads from being optimised away).  Asynchronous on
 * the stream; EPTV_ERR_ARG for null pointers, zero size or misalignment. */
int eptv_stream_read(const void* buf, size_t bytes, unsigned* sink, void* stream);

/* ------------------------------------------------------------------ batches
 * Many slices, each with its own geometry (image size, views, bins), iterated
 * together: every phase of the EPTV iteration (Sec. 2.2) is one launch for
 * the whole batch, a persistent grid walking a list of (slice, block) items,
 * and with EPTV_GRAPH=1 one outer iteration of all slices is one captured
 * graph (as for eptv_reconstruct).  Each slice's
 * arithmetic is that of eptv_reconstruct on its own plan; with the
 * projector's launch shape at 16 segments (the one-slice default) the images
 * are identical bit for bit.  The stored-matrix and Eq. 11 variants and the
 * early stop are one-slice only (EPTV_ERR_ARG here). */
typedef struct eptv_batch_s* eptv_batch;

/* One plan per geometry (geoms[0 .. n_slices-1]); owns them. */
int eptv_batch_create(const eptv_geometry* geoms, int n_slices, eptv_batch* out);
int eptv_batch_destroy(eptv_batch batch);
int eptv_batch_size(eptv_batch batch, int* n_slices);
/* The plan of one slice (owned by the batch), for one-slice calls. */
int eptv_batch_plan(eptv_batch batch, int slice, eptv_plan* plan);
/* Workspace bytes for eptv_batch_reconstruct with these params. */
int eptv_batch_workspace_bytes(eptv_batch batch, const eptv_params* params, size_t* bytes);

/* Launch shapes: projector sweep segments per block (4, 8 or 16) and
 * persistent blocks per compute unit for the projector and for the
 * tile-shaped phases (1..64).  eptv_batch_tune chooses them by timing. */
int eptv_batch_set_launch(eptv_batch batch, int proj_seg, int proj_blocks_per_cu, int tile_blocks_per_cu);
int eptv_batch_get_launch(eptv_batch batch, int* proj_seg, int* proj_grid, int* tile_grid);
/* The launch-shape tuner: times the batched projector (sweep segments 4/8/16
 * x 1/2/4 blocks per CU) and backprojector (2/4/8/16 blocks per CU) on
 * scratch data, reps launches each, and keeps the fastest; reports their
 * average times (may be NULL).  Allocates and frees scratch device memory;
 * synchronises the stream. */
int eptv_batch_tune(eptv_batch batch, int reps, void* stream, float* proj_ms, float* backproj_ms);

/* The exact P (Sec. 2.1, Eq. 1) and its transpose P^T (Sec. 2.2) of every
 * slice in one launch each: q[i] = alpha P_i x[i] + beta q[i], and
 * z[i] = alpha P_i^T r[i] + beta z[i] (beta == 0 never reads the output), the
 * same arithmetic as eptv_project / eptv_backproject on each slice's plan in
 * the batch's launch shape.  x[i], z[i] [ny_i][nx_i], q[i], r[i]
 * [n_views_i][n_bins_i], device pointers, one per slice.  ws: workspace of
 * eptv_batch_operator_workspace_bytes (the projector stages each image's
 * transposed copy there).  Asynchronous on the stream. */
int eptv_batch_operator_workspace_bytes(eptv_batch batch, size_t* bytes);
int eptv_batch_project(eptv_batch batch, const float* const* x, float* const* q, float alpha, float beta, void* ws,
                       size_t ws_bytes, void* stream);
int eptv_batch_backproject(eptv_batch batch, const float* const* r, float* const* z, float alpha, float beta,
                           void* ws, size_t ws_bytes, void* stream);

/* params.outer_iters EPTV iterations on every slice: y[i] (device
 * [V_i][B_i]), f[i] (device [ny_i][nx_i], warm start unless zero_init,
 * result), f_ref (NULL, or an array of reference images for the RMSE
 * record); host arrays of n_slices device pointers.  stats: NULL or an array
 * of n_slices records (synchronises the stream).  ws: 256-byte aligned
 * device workspace of eptv_batch_workspace_bytes. */
int eptv_batch_reconstruct(eptv_batch batch, const eptv_params* params, const float* const* y, float* const* f,
                           const float* const* f_ref, void* ws, size_t ws_bytes, eptv_stats* stats, void* stream);

/* ------------------------------------------------------------------ the U-Net
 * A convolutional network (not part of the paper) that maps an early EPTV
 * reconstruction to the half-edge weight maps of Eq. 5 / A3 and to an image,
 * used to start the EPTV iteration of Sec. 2.2 closer to its end.  Encoder
 * levels of two 3x3 convolutions (base << level channels, ReLU) joined by 2x2
 * average pooling; decoder levels of a stride-2 2x2 transposed convolution
 * (ReLU), concatenation with the encoder's output of that level, two 3x3
 * convolutions (ReLU); a final 1x1 convolution.  bf16 weights and
 * activations, fp32 accumulation on the matrix cores, fp32 master weights
 * and Adam.  Tensors at the boundary are device fp32 NHWC [n][h][w][c].
 * Parameters: a flat fp32 array, per layer (encoder levels first, then the
 * decoder from the bottom up, then the 1x1) weights laid out
 * [3][3][C_in][C_out] / [2][2][C_in][C_out] / [C_in][C_out], then the bias. */
typedef struct eptv_unet_s* eptv_unet;

/* height and width must be multiples of 2^(levels-1); base a multiple of 8
 * when levels > 1.  Buffers are sized for max_batch images. */
int eptv_unet_create(int c_in, int c_out, int base, int levels, int max_batch, int height, int width,
                     eptv_unet* out);
int eptv_unet_destroy(eptv_unet net);
int eptv_unet_param_count(eptv_unet net, long long* n);
/* Host arrays of eptv_unet_param_count floats; set_params also clears the
 * Adam moments.  All three synchronise the stream. */
int eptv_unet_set_params(eptv_unet net, const float* params, void* stream);
int eptv_unet_get_params(eptv_unet net, float* params, void* stream);
int eptv_unet_get_grads(eptv_unet net, float* grads, void* stream);
/* y = net(x) for n <= max_batch images; x [n][h][w][c_in], y [n][h][w][c_out]. */
int eptv_unet_forward(eptv_unet net, const float* x, int n, float* y, void* stream);
/* Gradients of sum(dy * y) for the last forward's batch: parameter gradients
 * (overwritten, read with eptv_unet_get_grads) and, if dx is given, the input
 * gradient [n][h][w][c_in]. */
int eptv_unet_backward(eptv_unet net, const float* dy, float* dx, void* stream);
/* One Adam step (Kingma & Ba) on the parameters with the current gradients;
 * step counts from 1. */
int eptv_unet_adam(eptv_unet net, float lr, float beta1, float beta2, float eps, int step, void* stream);
/* loss = mean((y - target)^2) over n floats into a device float; dy (may be
 * NULL) = its gradient 2 (y - target) / n. */
int eptv_unet_mse(eptv_unet net, const float* y, const float* target, size_t n, float* dy, float* loss,
                  void* stream);

/* EPTV images and half-edge weights (Eq. 5 / A3) as network tensors, for
 * n_img images of ny x nx stored one after another: f and f_base
 * [n_img][ny][nx], wx [n_img][ny][nx+1], wy [n_img][ny+1][nx], maps NHWC fp32
 * (all device).  The image channel is scale * (f - f_base) (f_base may be
 * NULL: scale * f); scale > 0 brings the attenuation image (mm^-1), or its
 * change from a base image, to unit order for the network.  With weights,
 * maps has 3 channels: 0 = wx[j][i+1] (the half-edge right of pixel (i, j)),
 * 1 = wy[j+1][i] (the half-edge above it), 2 = the image channel; with
 * wx = wy = NULL, the image channel alone. */
int eptv_maps_from_eptv(int n_img, int ny, int nx, const float* f, const float* f_base, const float* wx,
                        const float* wy, float scale, float* maps, void* stream);
/* The inverse for 3-channel maps: f = max(channel 2 / scale + f_base, 0)
 * (f_base may be NULL), weights clamped to [0, 1]; the half-edges on the left
 * (wx[j][0]) and bottom (wy[0][i]) border, which no pixel's channels hold,
 * take the weight of the adjacent half-edge of their row / column.  The
 * weights are ready for eptv_reconstruct_weighted, f for its warm start. */
int eptv_maps_to_eptv(int n_img, int ny, int nx, const float* maps, float scale, const float* f_base, float* f,
                      float* wx, float* wy, void* stream);

const char* eptv_status_string(int status);

/* Last HIP error text seen by the library on this thread ("" if none). */
const char* eptv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
