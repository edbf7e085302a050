// Device helpers and kernel launchers of the reduced-camera-system library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace ba {

// slots of the device scalar array of the solvers
enum {
    SC_RR0 = 0,      // |r_0|^2
    SC_RR = 1,       // |r_i|^2
    SC_DELTA = 2,    // Delta_i (PCG)
    SC_GAMMA = 3,    // gamma_i (PCG)
    SC_ALPHA = 4,    // alpha_i (PCG)
    SC_PHI = 5,      // Phi_i (PCG)
    SC_BETA = 6,     // beta_i (PCG)
    SC_BREAK = 7,    // 1 when P^T S P <= 0 (PCG)
    SC_T = 8,        // t_i of the tau-test (MCG)
    SC_RHO = 9,      // r^T D^-1 r (MCG)
    SC_RANK = 10,    // numerical rank of Delta_i (MCG)
    SC_DONE = 11,    // 1 once the PCG loop has stopped (device-side stop test)
    SC_ITER = 12,    // completed PCG iterations
    SC_STATUS = 13,  // ba_status of the PCG loop
    SC_SKIPM = 14,   // MCG: 1 unless the next block is multidirectional (t < tau, not converged)
    SC_KN = 15,      // MCG: width of the next block (0 once converged, N multidirectional, else 1)
    SC_SKIPS = 16,   // MCG: 1 unless the next block has one column
    SC_COUNT = 20    // the last two slots: scratch of the true-residual check
};

// device status word bits
constexpr int32_t kStatusNonfinite = 1;
constexpr int32_t kStatusNotSpdLandmark = 2;
constexpr int32_t kStatusNotSpdCamera = 4;

__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)0x7FC0;   // NaN
    u += 0x7FFFu + ((u >> 16) & 1u);                                   // round to nearest even
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint32_t h) {
    uint32_t u = h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// Values of one observation's record in the tile stream (pose dimension DP = 9, or 6
// for extrinsics only): J_p rows 0, 1 then J_l rows 0, 1; 16-byte words per slot in
// FP64 (pairs), FP32 (quads) and BF16 (octets), the last word zero-padded.
template <int DP>
struct RecordShape {
    static constexpr int kVals = 2 * DP + 6;
    static constexpr int kW64 = kVals / 2;
    static constexpr int kW32 = (kVals + 3) / 4;
    static constexpr int kW16 = (kVals + 7) / 8;
};

// ---- build (k_build.hip); dp = pose dimension (9 or 6)
void launch_check_finite(const double *a, int64_t count, int32_t *status, hipStream_t s);
void launch_pack(const int64_t *slot_obs, int64_t nslots, const double *Jp, const double *Jl, double *J64,
                 float *J32, uint16_t *J16, hipStream_t s, int dp = 9);
void launch_convert(const double *J64, int64_t nslots, float *J32, uint16_t *J16, hipStream_t s, int dp = 9);
// lambda-independent sums (read the caller's J and r): J_l^T J_l and b_l per landmark,
// J_p^T J_p (packed upper triangle) and b_p per camera
void launch_landmarks_base(int nl, const int64_t *first_slot, const int32_t *count, const int64_t *slot_obs,
                           const double *Jl, const double *r, double *Vraw, double *bl, hipStream_t s);
void launch_cameras_base(int np, const int64_t *cam_ptr, const int64_t *cam_obs, const double *Jp, const double *r,
                         double *Uraw, double *bp, hipStream_t s, int dp = 9);
// the values that depend on lambda, from those sums and the packed tile stream
void launch_landmarks_lambda(int nl, const double *Vraw, const double *bl, double lambda, double *vinv, double *h0,
                             int32_t *status, hipStream_t s);
void launch_cameras_lambda(int np, const int64_t *cam_ptr, const int64_t *cam_obs, const int32_t *obs_lm,
                           const int32_t *lmk_store, const int64_t *obs_slot, const double *J64, const double *Uraw,
                           const double *bp, const double *vinv, const double *h0, double lambda, double *dU,
                           double *Dblk, double *Dchol, double *bt, int32_t *status, hipStream_t s, int dp = 9);

// ---- Schur products (k_schur.hip)
struct SchurArgs {
    const void *J = nullptr;                 // tile stream in the chosen precision
    int precision = 0;                       // 0 FP64, 1 FP32, 2 BF16
    const uint32_t *meta = nullptr;
    const int32_t *tile_lmk_base = nullptr;
    const double *vinv = nullptr;
    const int32_t *chunk_tile = nullptr, *chunk_part = nullptr, *part_cam = nullptr, *part_dst = nullptr;
    int n_chunks = 0;
    int max_slots = 0;
    double *partial = nullptr;
    const int32_t *cam_part_ptr = nullptr;
    const double *dU = nullptr;
    int np = 0;
    const double *done = nullptr;            // nullable: when *done != 0 the launch does nothing
    // batches (nullable): a chunk / camera of problem b does nothing when seg_skip[b] != 0
    const int32_t *chunk_seg = nullptr, *cam_seg = nullptr, *seg_skip = nullptr;
    int dp = 9;                              // pose dimension: 9, or 6 for extrinsics only
    // nullable, single systems only: the camera reduction also leaves the partials of
    // y^T v and v^T gram_r, gram[2 b], gram[2 b + 1] for b < schur_gram_blocks(np)
    double *gram = nullptr;
    const double *gram_r = nullptr;
    // nullable: the camera reduction also writes y rounded to FP32 here (the FP32 history
    // copy of mixed-precision MCG)
    float *y32 = nullptr;
};
int schur_gram_blocks(int np);
// FP64 chunk wavefronts of the S product (of the multidirectional product) resident at
// once on the current device (0: unknown)
int schur1_resident_chunks(int dp);
int schur_multi_resident_chunks(int dp);
// y = S v (partials then the camera reduction)
void launch_schur_matvec(const SchurArgs &a, const double *v, double *y, hipStream_t s);
void launch_schur_chunks(const SchurArgs &a, const double *v, hipStream_t s);
void launch_schur_reduce(const SchurArgs &a, const double *v, double *y, hipStream_t s);

struct MultiArgs {
    const void *J = nullptr;
    int precision = 0;
    const uint32_t *meta = nullptr;          // for the landmark index inside the tile
    const uint32_t *mmeta = nullptr;
    const int32_t *slot_cam = nullptr;
    const uint8_t *pair_ll = nullptr;
    const uint32_t *tile_oidx = nullptr;
    const uint16_t *oidx = nullptr;
    const uint16_t *slot_ooff = nullptr;
    const int32_t *tile_lmk_base = nullptr;
    const double *vinv = nullptr;
    const int32_t *chunk_tile = nullptr, *chunk_part = nullptr;
    int n_chunks = 0, max_out = 0;
    double *partial = nullptr;
    const int32_t *part_dst = nullptr;
    const int32_t *cg_ptr = nullptr;
    const double *dU = nullptr;
    const int32_t *group = nullptr;
    int np = 0, N = 0;
    // batches (nullable): a chunk / camera of problem b does nothing when seg_skip[b] != 0
    const int32_t *chunk_seg = nullptr, *cam_seg = nullptr, *seg_skip = nullptr;
    const double *skip = nullptr;             // nullable: when *skip != 0 the launch does nothing
    int dp = 9;                               // pose dimension: 9, or 6 for extrinsics only
};
// Y[p] = S (z restricted to subset p), Y column-major [N][n]
void launch_schur_multi(const MultiArgs &a, const double *z, double *Y, hipStream_t s);

// dx_l = -V^-1 (b_l + W^T dx_p), written in original landmark order
void launch_back_substitute(const double *J64, const uint32_t *meta, const int32_t *tile_lmk_base,
                            const int32_t *chunk_tile, const int32_t *chunk_part, const int32_t *part_cam,
                            int n_chunks, int max_slots, const double *vinv, const double *bl,
                            const int32_t *lmk_order, const double *dxp, double *dxl, hipStream_t s, int dp = 9);

// ---- vectors, reductions, small dense (k_vec.hip)
constexpr int kRedBlocks = 120;    // fixed grid of the deterministic reductions
constexpr int kPhiSeg = 16;        // row segments of a one-column Phi (Alg. 2 reorthogonalisation)

// DP x DP block-Jacobi solves, dp = 9 or 6 (pose dimension)
void launch_precond(int np, const double *Dchol, const double *r, double *z, hipStream_t s, int dp = 9);
// finalize: out[d] = sum_b partials[b * nd + d] (fixed order), d < nd
void launch_finalize(const double *partials, int nd, double *out, hipStream_t s);

// mixed-precision refinement
void launch_residual_refine(int64_t n, const double *bt, const double *Sx, double *r, double *btp,
                            double *partials, hipStream_t s);
void launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s);

// PCG steps (scalars in sc[]: see k_vec.hip for the slot map)
void launch_pcg_init(int64_t n, const double *bt, const double *Sx, double *r, double *partials, hipStream_t s);
// alpha from n_dq pairs of partials of P^T S P and P^T r (the Gram partials the camera
// reduction or the explicit-S product leaves)
void launch_pcg_update_xr(int64_t n, const double *partials_dq, int n_dq, double *sc, double *x, double *r,
                          const double *P, const double *Q, double *partials_rr, hipStream_t s);
void launch_pcg_precond_phi(int np, const double *Dchol, const double *r, const double *Q, double *z,
                            double *partials, const double *done, hipStream_t s, int dp = 9);
void launch_pcg_step_end(const double *partials_rr, double *sc, double eps, int max_iter, double *trace,
                         hipStream_t s);
// partials_phi null: beta from sc[SC_BETA] (stored by launch_pcg_xrz)
void launch_pcg_update_p(int64_t n, const double *partials_phi, double *sc, const double *z, double *P,
                         hipStream_t s);
// Fused end of a PCG iteration with the block-Jacobi preconditioner: alpha, x and r,
// z = D^-1 r, the step-end decisions and beta (launch_pcg_update_xr, launch_pcg_step_end,
// launch_pcg_precond_phi in one launch); partials: 2 mcg_xrz_blocks(np, dp) doubles;
// ticket: a zero counter, left zero
void launch_pcg_xrz(int np, const double *pdq, int npdq, double *sc, double *x, double *r, const double *P,
                    const double *Q, const double *Dchol, double *z, double *partials, uint32_t *ticket, double eps,
                    int max_iter, double *trace, hipStream_t s, int dp = 9);
void launch_pcg_rr(const double *partials_rr, double *sc, hipStream_t s);

// MCG steps
// Gram products of a block of k > 1 columns: partials[b][...] of b < gram_blocks(k)
// blocks, their sums after them, at partials + gram_blocks(k) (k k + k) (one-column blocks
// take theirs from the camera reduction of the product, see XrzGram)
int gram_blocks(int k);
void launch_gram(int64_t n, int k, const double *P, const double *Q, const double *r, double *partials,
                 hipStream_t s);
// history block table entry written by the pseudo-inverse kernel (off == nullptr: none)
struct BlockEntry {
    int32_t *off = nullptr, *k = nullptr;
    int64_t *dp = nullptr;
    int j = 0, first = 0;
    int64_t dpo = 0;
};
// k > 1: Delta^+ and alpha from the Gram sums (nblocks partial blocks before them)
void launch_pinv_alpha(int k, const double *partials, int nblocks, double *Dp, double *gamma, double *alpha,
                       double *sc, hipStream_t s, BlockEntry blk = BlockEntry());
// Fused end of an MCG iteration: x += P alpha, r -= Q alpha, z = D^-1 r, and the scalars of
// Alg. 2's stop and tau tests (sc[SC_RR], [SC_RHO], [SC_T], and the next block's width in
// sc[SC_SKIPM], [SC_KN], [SC_SKIPS]), from
// mcg_xrz_blocks(np, dp) blocks' partials (2 per block) added by the last block to arrive
// (ticket: a zero counter, left zero); that block also copies sc[0, SC_COUNT) to host_sc
// (nullable: mapped host memory of SC_COUNT + 1 doubles) and, once those values are
// released at system scope, writes tag to host_sc[SC_COUNT]
// For a one-column block (g1.part set) the kernel also takes the place of the Gram and
// pseudo-inverse kernels: Delta and gamma from the camera reduction's partials (nb blocks,
// schur_gram_blocks), then Delta^+ into g1.Dp, gamma, alpha, sc[SC_RANK] and the block entry.
struct XrzGram {
    const double *part = nullptr;
    int nb = 0;
    double *Dp = nullptr;
    BlockEntry blk;
};
// The learned low-rank term of the preconditioner, M^-1 = D^-1 + U U^T (U: n x 8,
// row-major; d_p = 9): each block leaves the 8 partial sums of U^T r in part[8 b ..], the
// last block adds them into w (8 doubles) and takes rho = r^T D^-1 r + |w|^2; Z = D^-1 r
// then still needs + U w (launch_lr_zadd, next on the stream).
constexpr int kLowRank = 8;   // columns of the learned low-rank term U
struct XrzLowrank {
    const double *U = nullptr;
    double *part = nullptr;
    double *w = nullptr;
};
int mcg_xrz_blocks(int np, int dp);
void launch_mcg_xrz(int np, int k, const double *P, const double *Q, double *alpha, double *x, double *r,
                    const double *Dchol, double *z, double *partials, uint32_t *ticket, double *gamma,
                    double *sc, double *host_sc, double tag, int N, double tau, double eps, hipStream_t s,
                    int dp = 9, XrzGram g1 = XrzGram(), XrzLowrank lr = XrzLowrank());
// z += U w (n x 8 row-major U, w of 8 doubles)
void launch_lr_zadd(int64_t n, const double *U, const double *w, double *z, hipStream_t s);
// Phi segments per history column: the N subsets when N > 1 (the same for one-column
// and multidirectional steps), kPhiSeg row segments when N = 1
int phi_segments(int N);
// gs: rows of one subset (subset poses times the pose dimension)
template <typename HT>   // history stored in FP64 (double) or, on the mixed path, as an FP32 copy (float)
void launch_phi(int64_t n, int h, const HT *Qh, const double *z, int N, int gs, double *Phi, hipStream_t s);
// row length of beta for a kn-column step: kn = 1 unpadded, else kn rounded up to the
// output block of the history products (16 up to 16 columns, then multiples of 32), the
// padding zero
__host__ __device__ inline int hist_ldb(int kn) { return kn <= 1 ? 1 : kn <= 16 ? 16 : (kn + 31) / 32 * 32; }
// beta = Delta^+ Phi per history block (rows of hist_ldb(kn)) for the next block's width
// kn = sc[SC_KN] as the device decided it (nothing when 0 or above kn_max); kn = 1 adds
// Phi's segments, kn = N takes them apart
void launch_beta(int nb, const int32_t *blk_off, const int32_t *blk_k, const int64_t *blk_dp, const double *Dp,
                 const double *Phi, const double *sc, int kn_max, int N, double *beta, hipStream_t s);
// The new block's P columns (Pn, kn of them), kn = sc[SC_KN] read on the device, and the
// history sums of its Q columns in the scratch (kept for launch_update_q); kn_max is the
// widest block the history has room for.  The scratch holds at least
// hist_scratch_min(n, kn_max) doubles.  mfma: blocks wider than 16 on the FP64 matrix
// cores.  Pn32 (nullable): the new columns also rounded to FP32 there.
template <typename HT>   // Ph, Qh: FP64 history or its FP32 copy
void launch_update_pq(int64_t n, int h, int N, int kn_max, const HT *Ph, const HT *Qh, const double *beta,
                      const double *z, int gs, const double *sc, double *Pn, double *scratch, int64_t scratch_doubles,
                      hipStream_t s, bool mfma = false, float *Pn32 = nullptr);
// FP32 copy of history columns [c0, c0 + k) of P and Q (column-major, n rows)
void launch_hist_copy32(int64_t n, int64_t c0, int k, const double *Ph, const double *Qh, float *P32, float *Q32,
                        hipStream_t s);
// Q columns of a multidirectional block (N of them): Qn holds S Z on entry; the history
// sums are those launch_update_pq left in the scratch with kn_max = N; Qn32 (nullable):
// the columns also rounded to FP32 there
void launch_update_q(int64_t n, int h, int N, const double *sc, double *Qn, const double *scratch,
                     int64_t scratch_doubles, hipStream_t s, float *Qn32 = nullptr);
int64_t hist_scratch_min(int64_t n, int kn_max);
void launch_pinv_sym(int k, const double *A, double *Ap, int32_t *rank, hipStream_t s);

// ---- learned low-rank preconditioner (k_learned.hip)
void launch_features(int np, const double *Dblk, const int32_t *deg, double lambda, float *F, hipStream_t s);
void launch_mlp_forward(const float *P, const float *F, int rows, float *out, float *hid, int bf16, hipStream_t s);
void launch_lowrank_U(int np, const double *Dchol, const float *out, double *U, hipStream_t s);
void launch_block_scale(int np, const double *Dchol, const double *x, double *y, int transpose, hipStream_t s);
// z += U (U^T r) and partial sums of a2^T z (a2, partials nullable); pproj: kRedBlocks x 8
void launch_lowrank_apply(int64_t n, const double *U, const double *r, double *z, const double *a2, double *pproj,
                          double *partials, const double *done, hipStream_t s);
void launch_probe_loss_grad(int64_t n, int Pn, const float *Uh, const double *W, const double *Sw, double *work,
                            float *g_out, hipStream_t s);
size_t probe_work_doubles();
void launch_mlp_backward(const float *P, const float *F, const float *hid, const float *g_out, float *g_pre, int rows,
                         float *grad, hipStream_t s);
void launch_adam(float *P, const float *g, float *m, float *v, int t, float lr, hipStream_t s);


// ---------------------------------------------------------------- explicit S (block-sparse rows)
// The observation structure the explicit S is formed from: observations camera by
// camera, their landmarks' storage index, and each landmark's observation slots
struct BsrGather {
    const int64_t *cam_ptr = nullptr, *cam_obs = nullptr;
    const int32_t *obs_lm = nullptr, *lmk_store = nullptr;
    const int64_t *lmk_first_slot = nullptr;
    const int32_t *lmk_count = nullptr;
    const int32_t *slot_cam = nullptr;        // camera of every observation slot
};
// nonzero blocks per block row; then the rows' columns (ascending) at row_ptr
void launch_bsr_rowcount(int np, const BsrGather &g, int32_t *nnz, hipStream_t s);
void launch_bsr_rowfill(int np, const BsrGather &g, const int32_t *row_ptr, int32_t *col, hipStream_t s);
// blocks of a row that one wavefront of the assembly holds in lds_bytes of LDS (with the
// row's column list); 0 when not even one fits
int bsr_assembly_piece(int max_row, size_t lds_bytes);
// block values (9 x 9, row-major per block); obs_slot: slot of every observation; rows are
// assembled in pieces of at most `piece` blocks (bsr_assembly_piece)
void launch_bsr_assemble(int np, const BsrGather &g, const int64_t *obs_slot, const double *J64, const double *vinv,
                         const double *Dblk, const int32_t *row_ptr, const int32_t *col, int max_row, int piece,
                         double *val, hipStream_t s);
// y = S v; with gram, row j also leaves gram[2 j] = y_j . v_j, gram[2 j + 1] = v_j . gram_r_j
// (np partial pairs, see bsr_gram_blocks)
void launch_bsr_mv(int np, const int32_t *row_ptr, const int32_t *col, const double *val, const double *v, double *y,
                   const double *done, hipStream_t s, double *gram = nullptr, const double *gram_r = nullptr);
inline int bsr_gram_blocks(int np) { return np; }
void launch_bsr_mm_grouped(int np, int N, const int32_t *row_ptr, const int32_t *col, const double *val,
                           const int32_t *group, const double *z, double *Y, hipStream_t s,
                           const double *skip = nullptr);

// ---------------------------------------------------------------- batches (Algorithm 2 per problem)

struct BatchProb {            // problem b of a batch (static)
    int64_t row0;             // first row in the batch vectors (9 x first camera)
    int64_t hbase;            // history column 0 in Ph and Qh (doubles)
    int64_t colbase;          // first history slot: block tables at colbase, Phi / beta / Delta^+ at colbase * N
    int32_t n, np;            // rows, cameras
    int32_t cam0, gs;         // first camera; poses per subset (the last subset takes the rest)
    int32_t cap, pad;         // history capacity (columns)
};

struct BatchDyn {             // per-problem solver state, advanced by the kernels
    int32_t hcols, nblk, cur_off, kcur;   // history columns and blocks; current block (first column, width)
    int32_t kn, multi, done, status;      // width of the next block, tau-test outcome, stopped, ba_status
    int32_t iters, multi_steps, rank, max_it;   // ...; iterations this solve may take
    int64_t dp_used;                      // Delta^+ storage used (doubles)
    double rr0, rr, rho, t;
};

struct BatchLaunch {
    int B = 0, N = 1, max_np = 0;
    int64_t max_n = 0, ntot = 0;
    const BatchProb *prob = nullptr;
    BatchDyn *dyn = nullptr;
    const double *Dchol = nullptr;
    double *x = nullptr, *r = nullptr, *z = nullptr, *pstage = nullptr, *qstage = nullptr, *Y = nullptr;
    double *Ph = nullptr, *Qh = nullptr, *Dp = nullptr, *Phi = nullptr, *beta = nullptr;
    double *alpha = nullptr, *gamma = nullptr, *gpart = nullptr, *upart = nullptr;
    int32_t *blk_off = nullptr, *blk_k = nullptr;
    int64_t *blk_dp = nullptr;
    int32_t *skip_single = nullptr, *skip_multi = nullptr;
};
constexpr int kMaxBlock = 64;         // widest direction block of Algorithm 2
constexpr int kBatchGramBlocks = 16;   // partial blocks per problem of the Gram and update reductions
constexpr int kBatchVecBlocks = 8;
constexpr int kBatchPhiBlocks = 128;   // fixed grids of the history kernels (per problem), whatever the
constexpr int kBatchBetaBlocks = 32;   // history width, so an iteration's launches never change
// r = -bt, x = x0 (or 0), rr0; problems with off[b] != 0 stay stopped; P_0 = D^-1 r_0.  With
// `only`, just the flagged problems are (re)started.  Each may take max_it[b] iterations
// (max_iter when max_it is NULL).
void launch_bstart(const BatchLaunch &L, const double *bt, const double *x0, const int32_t *off, hipStream_t s,
                   const int32_t *only, int max_iter, const int32_t *max_it);
// Gram, Delta^+ / alpha, x / r / z update, stop and tau tests
void launch_biter_head(const BatchLaunch &L, double tau, double eps, hipStream_t s);
// Phi, beta and the new history block
void launch_biter_tail(const BatchLaunch &L, hipStream_t s);
// Q of one-column blocks from the staging product; the new block becomes current (`only`:
// just the flagged problems)
void launch_bqcopy_advance(const BatchLaunch &L, hipStream_t s, const int32_t *only = nullptr);
// per-problem |bt + Sx|^2 and |bt|^2 (out [B][2]) and, when btp is given, btp = bt + Sx
// (`only`: just the flagged problems)
void launch_bresidual(const BatchLaunch &L, const double *bt, const double *Sx, double *btp, double *out,
                      hipStream_t s, const int32_t *only = nullptr);
// FP64 refinement step xprev = x, x += d, and its undoing x = xprev, on the flagged problems
void launch_bouter_step(const BatchLaunch &L, const int32_t *only, double *x, const double *d, double *xprev,
                        hipStream_t s);
void launch_brevert(const BatchLaunch &L, const int32_t *only, double *x, const double *xprev, hipStream_t s);
// LM outer loop (k_lm.hip): residuals, Jacobian blocks and F of a state; the moved state
int project_blocks(int64_t m);   // doubles of `partials` launch_project needs
void launch_project(int64_t m, const int32_t *obs_cam, const int32_t *obs_lm, const double *cams, const double *X,
                    const double *u_obs, double *Jp, double *Jl, double *r, double *partials, double *cost,
                    hipStream_t s);
void launch_apply_step(int np, int nl, const double *cams, const double *X, const double *dxp, const double *dxl,
                       double *cams_out, double *X_out, hipStream_t s);

}  // namespace ba
