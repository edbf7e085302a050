/*
 * ba.h -- C ABI of the MI355X (gfx950) reduced-camera-system solver.
 *
 * Solves the damped Levenberg-Marquardt normal equation of bundle adjustment
 * after its reduction to the camera Schur complement
 *     S dx_p = -b~,  S = U_lambda - W V_lambda^-1 W^T,  b~ = b_p - W V_lambda^-1 b_l
 * (Weber, Demmel, Cremers, "Multidirectional Conjugate Gradients for Scalable
 * Bundle Adjustment", GCPR 2021, Sec. 3.1, eq. (7)-(15)) with block-Jacobi PCG
 * (Sec. 3.2, Algorithm 1) or Multidirectional CG (Sec. 3.2, Algorithm 2).
 *
 * Conventions shared by every call:
 *  - All array arguments are DEVICE pointers (HIP, the device current at
 *    ba_build_system) unless a comment says "host".  Arrays are dense,
 *    row-major C order, FP64 unless stated.
 *  - A pose has d_p parameters (Sec. 3.1): 9 (rotation increment,
 *    translation, focal, two radial terms) or 6 (rotation increment and
 *    translation, intrinsics fixed); the camera space has n = d_p * n_cams
 *    entries, ordered camera by camera.
 *  - Every call runs on the stream given to ba_build_system and returns
 *    after its work is complete (the library synchronises that stream).
 *  - Status codes: 0 success, > 0 warning, < 0 error (ba_status).  No
 *    exception crosses the ABI.  ba_last_error() gives a message for the
 *    last failing call on the calling thread.
 *  - A ba_system must not be used from two host threads at once.
 *  - The library allocates its own device memory (hipMalloc) inside
 *    ba_build_system and the solve calls; ba_free_system releases all of it.
 *    ba_build_system_ws takes the memory from a caller-owned workspace instead
 *    (sized by ba_build_workspace_bytes).  Input arrays are copied into the
 *    system's own layout: the caller may free them once the build has returned.
 */
#ifndef BA_H
#define BA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BA_OK = 0,
    BA_MAXITER = 1,            /* warning: max_iter reached; x holds the last iterate */
    BA_ERR_INVALID_ARG = -1,   /* null pointer, bad size, index out of range, duplicate
                                  (camera, landmark) pair, d_p not 6 or 9, N outside [1, n_cams] */
    BA_ERR_NONFINITE = -2,     /* NaN/Inf in J, r or lambda */
    BA_ERR_NOT_SPD = -3,       /* a V_lambda or D(S) block has a Cholesky pivot <= 0
                                  (e.g. a camera or landmark with no observation) */
    BA_ERR_BREAKDOWN = -4,     /* PCG: P^T S P <= 0; MCG: Delta numerically zero */
    BA_ERR_WORKSPACE = -5,     /* MCG history capacity too small */
    BA_ERR_HIP = -6,           /* a HIP runtime call failed */
    BA_ERR_NOMEM = -7,         /* device or host allocation failed */
    BA_ERR_UNSUPPORTED = -8    /* input outside the supported envelope (see message) */
} ba_status;

typedef struct ba_system ba_system;

/* One linearised BA problem: the per-observation split of J = (J_p J_l) and
 * r0 = r(x0) (Sec. 3.1, eq. (2)-(5)), and the damping coefficient lambda of
 * eq. (6) with diagonal damping D_p^T D_p = diag(J_p^T J_p), D_l^T D_l =
 * diag(J_l^T J_l).  Observation o couples camera obs_cam[o] and landmark
 * obs_lm[o]; each (camera, landmark) pair may appear at most once. */
typedef struct {
    int32_t n_cams;          /* n_p >= 1 */
    int32_t n_lms;           /* n_l >= 1 */
    int64_t n_obs;           /* m >= 1 */
    int32_t d_p;             /* pose dimension (Sec. 3.1): 9 (extrinsics and intrinsics) or 6 (extrinsics
                                only); the explicit S, batches and the learned preconditioner need 9 */
    int32_t reserved0;
    const int32_t *obs_cam;  /* device [m], in [0, n_cams) */
    const int32_t *obs_lm;   /* device [m], in [0, n_lms) */
    const double *J_p;       /* device [m][2][d_p]: d r_o / d (pose of obs_cam[o]) */
    const double *J_l;       /* device [m][2][3]: d r_o / d (landmark obs_lm[o]) */
    const double *r;         /* device [m][2]: residuals r_o at the linearisation point */
    double lambda;           /* >= 0 */
} ba_problem_desc;

typedef struct {
    int32_t store_fp32;      /* also keep an FP32 copy of the Jacobian stream (precision FP32) */
    int32_t store_bf16;      /* also keep a BF16 copy with per-camera column scales (precision BF16) */
    int32_t max_slots;       /* cameras per landmark chunk (0 = default 128; 64..440) */
    int32_t max_tiles;       /* 64-observation tiles per chunk of the S product; 0: as many as make every
                                chunk of the FP64 product resident at once on the device */
    int32_t explicit_schur;  /* also form S explicitly in 9x9 block-sparse rows (the paper's representation,
                                Sec. 3.2 and 4.1); FP64 S products then read it instead of the Jacobians.
                                Rows wider than one wavefront's LDS (251 blocks on gfx950) are assembled in
                                pieces; BA_ERR_UNSUPPORTED only when a row's column list alone exceeds it */
    int32_t max_tiles_multi; /* tiles per chunk of the multidirectional product; 0: max_tiles when that is
                                set, else as many as make every chunk of the FP64 product resident at once */
    int32_t ws_groups;       /* caller-owned workspace only (ba_build_system_ws): the solves it reserves memory
                                for -- PCG always, MCG with this many subsets N (0: none) */
    int32_t ws_max_iter;     /* ... and a direction history for this many iterations (0: 1000) */
} ba_build_opts;

typedef enum { BA_PREC_FP64 = 0, BA_PREC_FP32 = 1, BA_PREC_BF16 = 2 } ba_precision;

typedef struct {
    double eps;              /* relative residual tolerance, stop when |r_i| < eps |r_0| (1e-6) */
    int32_t max_iter;        /* imax (1000) */
    int32_t precision;       /* ba_precision used for the S products (FP64 default) */
    int32_t precond;         /* 0: block Jacobi D(S); 1: block Jacobi plus the low-rank term set by
                                ba_set_lowrank_precond */
    int32_t history_mfma;    /* MCG: 1 runs the history products of multidirectional blocks wider
                                than 16 columns (P_{i+1} = Z - sum_j P_j beta_ij and eq. (19)) on the
                                FP64 matrix cores instead of vector FMAs (0, measured faster) */
    int64_t max_history_cols;/* MCG history capacity in columns (0 = 1 + max_iter * N) */
    double inner_eps;        /* mixed precision: inner tolerance relative to the outer residual
                                (0 = automatic: 1e-3 for FP32 products, 1e-1 for BF16 storage; batches
                                use 1e-2 for FP32).  A single solve's inner tolerance is raised so that
                                the last step stops at half the outer target eps |b~| */
    int32_t max_outer;       /* mixed precision: max refinement steps (20) */
    int32_t max_inner;       /* mixed precision: max inner iterations per step (1000) */
    int32_t history_fp32;    /* mixed-precision MCG: 1 lets the reorthogonalisation (Phi = Q^T Z and the
                                history products of Alg. 2 / eq. (19)) read an FP32 copy of the P and Q
                                history (the storage option of the mixed path); the new block's Gram,
                                x, r and the S products keep FP64.  Ignored for FP64 solves and by
                                the batched solver.  ba_default_solve_opts sets 1 */
    int32_t reserved[3];
} ba_solve_opts;

/* Solve statistics.  The trace pointers are HOST arrays supplied by the caller
 * (nullable); entry i is filled for iteration i < min(iterations, trace_cap). */
typedef struct {
    int32_t iterations;       /* completed alpha-updates (Alg. 1/2, the x-update) */
    int32_t multi_steps;      /* MCG: steps with N directions */
    int32_t history_cols;     /* MCG: columns of the direction history */
    int32_t refinement_steps; /* mixed precision: outer steps */
    int32_t status;
    int32_t trace_cap;
    double rel_res_recursive; /* |r_i| / |r_0| of the recursive residual */
    double rel_res_true;      /* |-b~ - S x| / |b~| recomputed in FP64 */
    double t_solve_ms;        /* wall time of the solve on the stream */
    double *trace_res;        /* host [trace_cap]: |r_{i+1}| / |r_0| */
    double *trace_t;          /* host [trace_cap]: t_i of the tau-test (NaN when not taken) */
    int32_t *trace_k;         /* host [trace_cap]: columns of the next direction block (0 at exit) */
} ba_solve_stats;

/* Fills opts with the defaults (eps 1e-6, max_iter 1000, FP64, block Jacobi). */
void ba_default_solve_opts(ba_solve_opts *opts);

/* Builds the damped normal-equation blocks and the reduced camera system of
 * Sec. 3.1, eq. (8)-(15), and the block-Jacobi preconditioner D(S) (Sec. 3.2,
 * before Alg. 1), in FP64 on the device.  `stream` is a hipStream_t (NULL = the
 * null stream) used by every later call on the returned system.  opts nullable.
 * Errors: INVALID_ARG, NONFINITE, NOT_SPD, UNSUPPORTED (a landmark with more than
 * 64 observations), NOMEM, HIP.  On error *out is NULL. */
ba_status ba_build_system(const ba_problem_desc *desc, const ba_build_opts *opts, void *stream,
                          ba_system **out);

/* Device bytes that ba_build_system_ws carves out of the caller's workspace for this
 * problem and these options (the survey of the boundary: sizing only).  The layout is
 * planned on the host from the observation indices (copied from desc's device arrays on
 * the null stream), the values are not formed and nothing is allocated on the device.
 * The count covers the system (Jacobian stream and its layout, the blocks of eq. (8)-
 * (15), D(S), the explicit S and the FP32 / BF16 copies the options ask for) and the
 * memory of the solves opts->ws_groups and opts->ws_max_iter reserve: PCG (Alg. 1) with
 * a residual trace, MCG (Alg. 2) with ws_groups subsets (its multidirectional layout and
 * a history of 1 + ws_max_iter * ws_groups columns), and the refinement vectors when a
 * reduced-precision copy is stored.  bytes: host.  Errors as ba_build_system. */
ba_status ba_build_workspace_bytes(const ba_problem_desc *desc, const ba_build_opts *opts, size_t *bytes);

/* ba_build_system with every device array of the system in the caller's workspace ws
 * (device, 256-byte aligned, ws_bytes >= ba_build_workspace_bytes of the same desc and
 * opts).  The handle does not own ws: ws must stay allocated until ba_free_system, which
 * releases only the host-side parts.  The input arrays are copied into ws, so they may
 * be freed once the call has returned.  Later calls on the system take device memory
 * only from ws: the reserved solves run without allocating; anything beyond them
 * (another N, a longer history, a reduced precision not stored at build, the low-rank
 * preconditioner) uses what is left of ws or fails with BA_ERR_WORKSPACE.  Errors as
 * ba_build_system, plus INVALID_ARG (ws NULL or misaligned) and WORKSPACE (ws_bytes too
 * small). */
ba_status ba_build_system_ws(const ba_problem_desc *desc, const ba_build_opts *opts, void *ws, size_t ws_bytes,
                             void *stream, ba_system **out);

/* Bytes of the caller's workspace a system built by ba_build_system_ws has used so far
 * (0 for other systems).  bytes: host. */
ba_status ba_system_workspace_used(const ba_system *sys, size_t *bytes);

/* Releases the system and all its device memory (for ba_build_system_ws: the host-side
 * parts only).  Null-safe. */
void ba_free_system(ba_system *sys);

/* y = S v for one camera-space vector (the implicit product of eq. (14)):
 * y = J_p^T (e - J_l V_lambda^-1 J_l^T e) + lambda diag(J_p^T J_p) v with e = J_p v.
 * v, y: device [n].  precision: ba_precision of the Jacobian stream used. */
ba_status ba_schur_matvec(ba_system *sys, const double *v, double *y, int32_t precision);

/* The product of ba_schur_matvec, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, bit for bit, with the
 * product's partial camera rows kept in a file-scope device array of the library
 * (32 MiB, 4,194,304 doubles, one copy per GPU, held until the process ends)
 * instead of the system's own buffer.  The call allocates nothing and calls no
 * allocating routine.  v, y: device [n].  The system's device must be current.
 * Every call on one GPU shares that array, so calls that overlap in time on one GPU
 * (other host threads, other streams) race.  Errors: INVALID_ARG (NULL, precision
 * outside 0..2, another device current), UNSUPPORTED (precision 1 or 2 on a system
 * built without store_fp32 / store_bf16 and not yet used at that precision: the
 * reduced-precision copy would need an allocation), WORKSPACE (the system's partial
 * rows, n_part * d_p doubles, exceed the array), HIP. */
ba_status ba_schur_matvec_noalloc(ba_system *sys, const double *v, double *y, int32_t precision);

/* Y[:, p] = S Z[:, p], p < N, where Z[:, p] equals z on the poses of subset p of
 * the partition into N subsets (ba_partition) and 0 elsewhere -- the
 * multidirectional product of Sec. 3.2, "Optimized implementation", eq. (19).
 * z: device [n]; Y: device [N][n] (column p contiguous). */
ba_status ba_schur_matmat_grouped(ba_system *sys, int32_t n_groups, const double *z, double *Y,
                                  int32_t precision);

/* z = D(S)^-1 r (block-Jacobi preconditioner, one 9x9 Cholesky solve per pose).
 * r, z: device [n]. */
ba_status ba_precond_apply(ba_system *sys, const double *r, double *z);

/* Copies b~ (eq. (15)) into bt: device [n]. */
ba_status ba_get_rhs(ba_system *sys, double *bt);

/* Copies the d_p x d_p blocks of D(S) (row-major, camera by camera) into D: device [n_cams][d_p][d_p]. */
ba_status ba_get_precond_blocks(ba_system *sys, double *D);

/* Block-Jacobi PCG, Algorithm 1, on S dx_p = -b~.  x0: device [n] or NULL (= 0);
 * x: device [n] output.  opts, stats nullable (defaults).  Returns BA_OK,
 * BA_MAXITER or an error. */
ba_status ba_pcg_solve(ba_system *sys, const double *x0, double *x, const ba_solve_opts *opts,
                       ba_solve_stats *stats);

/* Multidirectional CG, Algorithm 2, with N subsets of consecutive poses and the
 * tau-test threshold tau >= 0.  A step is multidirectional iff N > 1 and
 * t_i < tau; the first step is global.  Same argument conventions as
 * ba_pcg_solve.  Errors: INVALID_ARG (N outside [1, n_cams], tau < 0),
 * WORKSPACE (history capacity), BREAKDOWN. */
ba_status ba_mcg_solve(ba_system *sys, int32_t n_groups, double tau, const double *x0, double *x,
                       const ba_solve_opts *opts, ba_solve_stats *stats);

/* Lays out, ahead of the solves, what ba_mcg_solve with N subsets and the given
 * precision needs beyond the build: the partition of the poses (Sec. 3.2,
 * "Optimized implementation"), the layout of the multidirectional product eq. (19)
 * (planned on the host from the observation indices, once per N; an explicit-S
 * system needs the partition only) and the reduced-precision Jacobian copy.  The
 * first ba_mcg_solve with these arguments does the same when it was not called.
 * Errors: INVALID_ARG (N outside [1, n_cams], precision outside 0..2), UNSUPPORTED,
 * NOMEM, HIP. */
ba_status ba_prepare_mcg(ba_system *sys, int32_t n_groups, int32_t precision);

/* Landmark update from a pose update, the second block row of eq. (7):
 * dx_l = -V_lambda^-1 (b_l + W^T dx_p).  (eq. (16) is printed with the sign of
 * b_l flipped.)  dxp: device [n]; dxl: device [n_lms][3], original landmark order. */
ba_status ba_back_substitute(ba_system *sys, const double *dxp, double *dxl);

/* Moore-Penrose pseudo-inverse of a symmetric k x k matrix on the device
 * (Sec. 3.2, "Optimized implementation": Delta_i is inverted or
 * pseudo-inverted): Jacobi eigendecomposition, eigenvalues with
 * |l| <= k 2^-52 max|l| dropped.  A, Ap: device [k][k]; rank: host, nullable.
 * 1 <= k <= 256.  Runs on `stream` (hipStream_t, NULL = null stream). */
ba_status ba_pinv_sym(int32_t k, const double *A, double *Ap, int32_t *rank, void *stream);

/* Partition of the n_cams poses into N subsets of consecutive poses (Sec. 3.2,
 * "Optimized implementation"): s = floor(n_cams / N); subsets 0..N-2 hold s
 * poses each, the last holds the rest.  group: HOST [n_cams]. */
ba_status ba_partition(int32_t n_cams, int32_t n_groups, int32_t *group);

/* Sizes of a built system.  All outputs host, nullable. */
ba_status ba_system_info(const ba_system *sys, int32_t *n_cams, int32_t *n_lms, int64_t *n_obs,
                         int64_t *n_tiles, int32_t *n_chunks, int64_t *matvec_bytes_fp64);

/* ---- Learned low-rank correction of the block-Jacobi preconditioner (an addition
 * to the paper's D(S), Sec. 3.2): M^-1 = D(S)^-1 + U U^T with U (n x 8, row-major),
 * U_c = L_c^-T Uh_c for D(S)_c = L_c L_c^T, and Uh_c (9 x 8, row-major) the output of a
 * 2-layer MLP (47 -> 128 tanh -> 72) on 47 features of camera c.  M^-1 is SPD for
 * any weights.  Solves use it when ba_solve_opts.precond = 1.
 * MLP parameters (FP32, BA_MLP_PARAMS): W1 [128][47], b1 [128], W2 [72][128], b2 [72]. */
#define BA_MLP_FEATURES 47
#define BA_MLP_OUT 72
#define BA_MLP_PARAMS 15432

/* Features of every camera into F (device [n_cams][47], FP32): 36 correlations
 * D_ij / sqrt(D_ii D_jj) (i < j, row-major) of D(S)_c, 9 log D_ii minus their mean,
 * log(1 + covisibility degree), log(max(lambda, 1e-12)). */
ba_status ba_lowrank_features(ba_system *sys, float *F);

/* out (device [rows][72]) = MLP(F) with params (device, FP32).  bf16 = 1: inference on
 * the matrix cores with BF16 operands and FP32 accumulation; 0: FP32.  Runs on stream. */
ba_status ba_mlp_forward(const float *params, const float *F, int32_t rows, float *out, int32_t bf16,
                         void *stream);

/* Sets the system's low-rank term from MLP outputs (device [n_cams][72]). */
ba_status ba_set_lowrank_from_mlp(ba_system *sys, const float *out);

/* Sets the low-rank term to U (device [n][8], copied), or clears it (U = NULL). */
ba_status ba_set_lowrank_precond(ba_system *sys, const double *U);

/* Copies the current low-rank term into U (device [n][8]). */
ba_status ba_get_lowrank(ba_system *sys, double *U);

/* y = L^-1 x (transpose = 0) or L^-T x (transpose = 1), with L the block Cholesky
 * factor of D(S); x, y device [n].  Maps vectors to and from the coordinates in
 * which D(S) is the identity. */
ba_status ba_block_scale(ba_system *sys, const double *x, double *y, int32_t transpose);

/* Training loss and gradient for one system: with Uh = MLP(F) viewed as n x 8 and
 * probes W, Sw (device [n][n_probes], row-major, Sw = L^-1 S L^-T W),
 *   loss = 1/(n_probes n) sum_k |W_k - Sw_k - Uh (Uh^T Sw_k)|^2,
 * an estimate of |I - (I + Uh Uh^T) L^-1 S L^-T|_F^2 / n.  grad: device [BA_MLP_PARAMS];
 * loss: host.  1 <= n_probes <= 8; rows = n_cams.  FP32 network, FP64 loss. */
ba_status ba_mlp_loss_grad(const float *params, const float *F, int32_t rows, const double *W, const double *Sw,
                           int32_t n_probes, float *grad, double *loss, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on params with the gradient grad and
 * moments m, v (all device [BA_MLP_PARAMS], FP32); t >= 1 counts steps. */
ba_status ba_adam_step(float *params, const float *grad, float *m, float *v, int32_t t, float lr, void *stream);

/* Event timing of the dominant kernel, the chunked implicit Schur product of
 * ba_schur_matvec and of the solvers' S v products (the block-sparse product with an
 * explicit S): with on >= 1, every on-th of its launches on this system is bracketed by
 * two HIP events recorded on the system's stream (on = 1: every launch; a larger on
 * samples the launches, so fewer event records sit between kernels); on = 0 turns it
 * off.  ba_profile_read (host outputs, nullable) returns the summed kernel time in ms
 * and the number of timed launches since the last reset.  BA_ERR_INVALID_ARG for
 * on < 0. */
ba_status ba_profile_enable(ba_system *sys, int32_t on);
ba_status ba_profile_read(ba_system *sys, double *ms_total, int64_t *launches, int32_t reset);

/* HOST-ONLY check of the HBM layout plan (no GPU needed): plans the layout of
 * the host index arrays cam, lm [n_obs] exactly as ba_build_system does, and the
 * layout of the multidirectional product for each N in Ns[n_Ns] (host), then
 * checks every invariant the kernels index by.  stats (host, nullable,
 * 4 + 3 n_Ns entries): tiles, chunks, partial rows, largest chunk slot count,
 * then per N: chunks, (camera, subset) partial rows, largest chunk out count.
 * Returns BA_OK, the planner's error, or BA_ERR_INVALID_ARG with
 * ba_plan_validate_error() naming the broken invariant. */
ba_status ba_plan_validate(int32_t n_cams, int32_t n_lms, int64_t n_obs, const int32_t *cam, const int32_t *lm,
                           int32_t max_slots, int32_t max_tiles, const int32_t *Ns, int32_t n_Ns,
                           int64_t *stats);
const char *ba_plan_validate_error(void);

/* ------------------------------------------------------------------ batches
 * Many independent problems solved at once, each by Algorithm 2 (Sec. 3.2) with
 * its own tau-test, Gram blocks, Delta^+ and direction history.  The batch is the
 * block-diagonal system over the concatenated problems: problem p holds cameras
 * [c_p, c_p + cams_per_problem[p]) (c_p the sum of the counts before it) and
 * rows [9 c_p, 9 (c_p + cams_per_problem[p])) of every batch vector. */
typedef struct ba_batch ba_batch;

typedef struct {
    int32_t iterations;       /* inner iterations, all refinement steps together */
    int32_t multi_steps;
    int32_t history_cols;     /* history columns of the last inner solve */
    int32_t refinement_steps; /* mixed precision: inner solves */
    int32_t status;           /* ba_status of this problem */
    int32_t reserved;
    double rel_res_recursive; /* last inner solve, |r_i| / |r_0| */
    double rel_res_true;      /* |b~ + S x| / |b~|, FP64 */
    double done_ms;           /* ms from the solve's start until this problem was seen stopped */
} ba_batch_stats;

/* Builds the batch from the concatenated problem `all` (device arrays as in
 * ba_build_system; camera and landmark indices global over the batch, every
 * landmark observed by cameras of one problem only, one lambda for all) and the
 * HOST array cams_per_problem[n_problems].  Tiles and chunks of the HBM layout
 * never mix problems.  Errors as ba_build_system, plus BA_ERR_INVALID_ARG when
 * the counts do not add up to all->n_cams or a landmark spans two problems. */
ba_status ba_batch_build(const ba_problem_desc *all, int32_t n_problems, const int32_t *cams_per_problem,
                         const ba_build_opts *opts, void *stream, ba_batch **out);
void ba_batch_free(ba_batch *batch);
/* The block-diagonal system of the batch (owned by the batch): S products,
 * right-hand side, preconditioner blocks of all problems at once. */
ba_system *ba_batch_system(ba_batch *batch);

/* Algorithm 2 for every problem of the batch on S_p x_p = -b~_p.  x: device
 * [9 * total cameras] (batch layout); N subsets per problem (1..64, at most the
 * cameras of the smallest problem), tau the threshold of the tau-test.  opts as
 * ba_mcg_solve (precision != FP64: FP64 refinement per problem around inner
 * solves with reduced-precision S products; precond must be 0).  Every
 * iteration is one fixed sequence of launches for all running problems, with all
 * solver state on the device; graph_window > 0 captures that many iterations
 * into one HIP graph per launch (0: eager launches, stop flags read every 8
 * iterations).  stats: HOST array [n_problems] (nullable); elapsed_ms (host,
 * nullable): wall time of the call.  Returns BA_OK when every problem reached
 * eps, BA_MAXITER when some did not, else the first error. */
ba_status ba_batch_mcg_solve(ba_batch *batch, int32_t N, double tau, double *x, const ba_solve_opts *opts,
                             int32_t graph_window, ba_batch_stats *stats, double *elapsed_ms);

/* Explicit S (ba_build_opts.explicit_schur): nonzero 9x9 blocks, bytes of the block
 * values, and the assembly time in ms (host outputs, nullable).  BA_ERR_INVALID_ARG
 * when the system was built without it. */
ba_status ba_explicit_schur_info(const ba_system *sys, int64_t *nnz_blocks, int64_t *bytes, double *assembly_ms);

/* New values for the same observations: the LM loop's relinearisation at a moved
 * state, or its new damping lambda (Sec. 4.1), on a built system.  J_p, J_l, r:
 * device arrays as in ba_problem_desc, in the observation order of the build.  The
 * layout (tiles, chunks, partitions, explicit-S pattern) is kept; every value the
 * build forms is recomputed (eq. (8)-(15), D(S) and its factor, the FP32/BF16
 * copies the system holds, the explicit S).  A low-rank preconditioner term set
 * before stays as set.  Errors: INVALID_ARG (batch systems, lambda < 0),
 * NONFINITE (nothing changed), NOT_SPD (the values are undefined until a
 * successful update). */
ba_status ba_update_system(ba_system *sys, const double *J_p, const double *J_l, const double *r, double lambda);

/* A new damping coefficient lambda (eq. (6), Marquardt damping D^T D = diag(J^T J))
 * for the same linearisation: the LM loop's accept/reject step (Sec. 4.1) after a
 * rejected step.  Recomputes every value that depends on lambda -- V_lambda^-1 and
 * V_lambda^-1 b_l per landmark, U_lambda's damping, D(S), its factor and b~
 * (eq. (9)-(15)), and the explicit S when the system keeps one -- from the undamped
 * blocks J_l^T J_l, J_p^T J_p, b_l and b_p kept at build and the packed Jacobian
 * stream, without reading J or r again.  The result equals, bit for bit, a fresh
 * ba_build_system (or ba_update_system) of the same J and r at this lambda.  A
 * low-rank preconditioner term set before stays as set.  Errors: INVALID_ARG (NULL,
 * lambda < 0, batch systems), NONFINITE (nothing changed), NOT_SPD (the values are
 * undefined until a successful ba_set_lambda or ba_update_system), HIP. */
ba_status ba_set_lambda(ba_system *sys, double lambda);

/* ------------------------------------------------------------------ LM outer loop
 * The Levenberg-Marquardt loop of Sec. 4.1 around the solvers above, for the
 * nine-parameter camera (Sec. 3.1, d_p = 9).  Camera c is 15 doubles: R
 * (row-major 3x3), t (3), f, k1, k2; landmark l is X_l (3).  Observation o of
 * landmark obs_lm[o] in camera obs_cam[o] has the residual
 *   r_o = f s p - u_obs[o],  P = R X + t,  p = P_xy / P_z,  s = 1 + k1 |p|^2 + k2 |p|^4,
 * and F = sum_o |r_o|^2 (eq. (1)).  A step (dx_p, dx_l) moves camera c by a left
 * rigid motion, R <- exp([w]x) R, t <- exp([w]x) t + dt with (w, dt) its first 6
 * entries, adds the last 3 to (f, k1, k2), and adds dx_l to the landmarks. */
typedef struct {
    int32_t n_cams;
    int32_t n_lms;
    int64_t n_obs;
    const int32_t *obs_cam;  /* device [m] */
    const int32_t *obs_lm;   /* device [m]; each (camera, landmark) pair at most once */
    const double *u_obs;     /* device [m][2]: observed pixel positions */
} ba_scene_desc;

typedef struct {
    int32_t max_iter;        /* LM iterations (25) */
    int32_t solver;          /* 0: PCG (Alg. 1); 1: MCG (Alg. 2) */
    int32_t n_groups;        /* MCG: N */
    int32_t reserved0;
    double tau;              /* MCG: tau */
    double lambda0;          /* first damping (1e-4) */
    double ftol;             /* stop after an iteration with |F - F_new| / F < ftol (1e-6) */
    double lambda_factor;    /* lambda / factor after an accepted step, x factor after a rejected one (10) */
    ba_solve_opts solve;     /* the linear solves (ba_default_solve_opts) */
    ba_build_opts build;     /* the reduced camera system (zeros: defaults) */
} ba_lm_opts;

typedef struct {
    int32_t iterations;      /* LM iterations done */
    int32_t accepted;        /* of which moved the state */
    int32_t status;          /* BA_OK, or the error that ended the loop */
    int32_t solver_iterations; /* linear-solver iterations, all LM iterations together */
    double cost0;            /* F at the start */
    double cost;             /* F at the returned state */
    double t_total_ms;       /* wall time of the call */
    double t_solve_ms;       /* of which in the linear solves */
    double t_linearize_ms;   /* of which in residuals, Jacobians and system values */
    int32_t trace_cap;       /* entries of the HOST trace arrays below (nullable) */
    int32_t reserved;
    double *trace_lambda;    /* lambda of iteration i's solve */
    double *trace_cost;      /* F at the moved state of iteration i */
    int32_t *trace_accepted; /* 1 when iteration i moved the state */
    int32_t *trace_solver_iterations;
    double *trace_solve_ms;
} ba_lm_stats;

/* Fills opts with the defaults above (PCG, N = 1, tau = 3.3). */
void ba_default_lm_opts(ba_lm_opts *opts);

/* Residuals r (device [m][2], nullable) and, when J_p is not NULL, the Jacobian
 * blocks J_p (device [m][2][9]) and J_l (device [m][2][3]) in the step coordinates
 * above, at the state (cams: device [n_cams][15], X: device [n_lms][3]); F to
 * *cost (host, nullable).  Runs on `stream` and waits for it. */
ba_status ba_project(const ba_scene_desc *scene, const double *cams, const double *X, double *J_p, double *J_l,
                     double *r, double *cost, void *stream);

/* The state moved by the step: cams_out, X_out (device, the shapes of cams, X) from
 * dxp (device [9 n_cams]) and dxl (device [3 n_lms]).  Asynchronous on `stream`. */
ba_status ba_apply_step(int32_t n_cams, int32_t n_lms, const double *cams, const double *X, const double *dxp,
                        const double *dxl, double *cams_out, double *X_out, void *stream);

/* The LM loop of Sec. 4.1: lambda starts at lambda0; each iteration solves the
 * damped normal equation through the reduced camera system (Alg. 1 or 2 with
 * opts->solve), back-substitutes the landmarks, and evaluates F at the moved state;
 * the move is kept when F decreases (lambda / factor, the system is relinearised)
 * and dropped otherwise (lambda x factor, same linearisation).  It stops after
 * max_iter iterations, after an iteration with |F - F_new| / F < ftol, or at F = 0.
 * cams, X: device, the start state on entry and the final state on return.  A
 * linear solve that ends at its iteration limit still gives a step; any other
 * solver error ends the loop with that status (the state is the last accepted one).
 * stats: host, nullable. */
ba_status ba_lm_solve(const ba_scene_desc *scene, double *cams, double *X, const ba_lm_opts *opts, void *stream,
                      ba_lm_stats *stats);

/* Measurement helper (not part of the method): the HBM read rate in GB/s (host
 * output) of a kernel that streams a zero-filled buffer of `bytes` (device memory
 * allocated and freed by the call) in the S-product kernel's access pattern (one
 * wavefront per 16 tiles of 12 coalesced 1 KiB loads), timed with HIP events over
 * `reps` launches on `stream`.  The practical ceiling for that kernel's bandwidth. */
ba_status ba_stream_read_gbs(int64_t bytes, int32_t reps, double *gbs, void *stream);

/* Measurement helper (not part of the method): y = S v, as ba_schur_matvec, launched
 * `reps` >= 1 times back to back on the system's stream after one untimed launch, with
 * HIP events around the whole sequence and no synchronisation between launches.
 * *ms_per (host) receives the elapsed time divided by reps: the kernel time plus the gaps
 * between consecutive launches, without the host's per-call overhead.  v, y: device [n].
 * Errors as ba_schur_matvec; INVALID_ARG for reps < 1. */
ba_status ba_schur_matvec_timed(ba_system *sys, const double *v, double *y, int32_t precision, int32_t reps,
                                double *ms_per);

const char *ba_status_string(int32_t status);
const char *ba_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BA_H */
