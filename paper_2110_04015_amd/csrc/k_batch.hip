// Algorithm 2 for a batch of independent problems, all state on the device.
//
// The batch is one block-diagonal system: the cameras of problem b are a
// contiguous range and its rows [row0_b, row0_b + n_b) of the batch vectors, so
// one S product over all chunks applies every S_b at once (the chunk and camera
// kernels skip problems through per-problem flags).  Everything else of the
// recurrence is per problem: Gram blocks, Delta^+, alpha, the tau-test, the
// direction history with its own width per block, Phi, beta.  Per-problem
// scalars and counters live in BatchDyn and are advanced by the kernels
// themselves, so an iteration is a fixed sequence of launches with no read-back
// and can be captured into a graph.
#include "ba_internal.h"
#include "kernels.h"
#include "dev_la.h"

namespace ba {

constexpr int kBGX = kBatchGramBlocks;
constexpr int kBUX = kBatchVecBlocks;

__device__ __forceinline__ int subset_of(int cam_local, int gs, int N) { return min(cam_local / gs, N - 1); }

// rr0 partials: sum of r^2 over the rows of problem b (r = -bt)
__global__ __launch_bounds__(kNT) void k_bstart_rows(const BatchProb *__restrict__ prob, const double *__restrict__ bt,
                                                     const double *__restrict__ x0, double *__restrict__ x,
                                                     double *__restrict__ r, double *__restrict__ part,
                                                     const int32_t *__restrict__ only) {
    __shared__ double sh[kNT];
    const int b = blockIdx.y;
    if (only && !only[b]) return;
    const BatchProb P = prob[b];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * kNT) {
        const int64_t g = P.row0 + i;
        const double v = -bt[g];
        r[g] = v;
        x[g] = x0 ? x0[g] : 0.0;
        acc += v * v;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)b * kBUX + blockIdx.x] = acc;
}

// resets the per-problem state; problems flagged in `off` start (and stay) stopped.  With
// `only`, just the flagged problems are (re)started and the others keep their state.  A
// problem may take max_it[b] iterations (max_iter when max_it is NULL).
__global__ void k_bstart(int B, const double *__restrict__ part, const int32_t *__restrict__ off,
                         BatchDyn *__restrict__ dyn, int32_t *__restrict__ skip_single,
                         int32_t *__restrict__ skip_multi, const int32_t *__restrict__ only, int max_iter,
                         const int32_t *__restrict__ max_it) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (only && !only[b]) return;
    double rr = 0.0;
    for (int u = 0; u < kBUX; ++u) rr += part[(int64_t)b * kBUX + u];
    BatchDyn d{};
    d.rr0 = rr;
    d.rr = rr;
    d.kn = 1;
    d.status = BA_MAXITER;
    d.max_it = max_it ? max_it[b] : max_iter;
    d.done = (off && off[b]) ? 1 : 0;
    if (!d.done && rr == 0.0) {
        d.done = 1;
        d.status = BA_OK;
    }
    dyn[b] = d;
    skip_single[b] = d.done;
    skip_multi[b] = 1;
}

// P_0 = Z_0 = D^-1 r_0 into history column 0 of each running problem and into the
// staging vector for Q_0 = S P_0
__global__ void k_bseed(int B, const BatchProb *__restrict__ prob, const BatchDyn *__restrict__ dyn,
                        const double *__restrict__ Dchol, const double *__restrict__ r, double *__restrict__ Ph,
                        double *__restrict__ pstage, const int32_t *__restrict__ only) {
    const int b = blockIdx.y;
    if (dyn[b].done || (only && !only[b])) return;
    const BatchProb P = prob[b];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.np) return;
    double rc[9], zc[9];
    const int64_t g = P.row0 + (int64_t)c * 9;
    for (int i = 0; i < 9; ++i) rc[i] = r[g + i];
    chol9_solve(Dchol + (int64_t)(P.cam0 + c) * 45, rc, zc);
    for (int i = 0; i < 9; ++i) {
        Ph[P.hbase + (int64_t)c * 9 + i] = zc[i];
        pstage[g + i] = zc[i];
    }
}

// Delta = Q_cur^T P_cur (k x k) and gamma = P_cur^T r partials over a row range of problem b.
// k = 1: two dot products with two rows per thread in flight.  k > 1: chunks of R rows
// (R k <= kBGramChunk) staged in LDS column by column, each column padded by one double so
// that the threads of an output row read distinct banks.
constexpr int kBGramChunk = 2048;
__global__ __launch_bounds__(kNT) void k_bgram(int N, const BatchProb *__restrict__ prob,
                                               const BatchDyn *__restrict__ dyn, const double *__restrict__ Ph,
                                               const double *__restrict__ Qh, const double *__restrict__ r,
                                               double *__restrict__ part) {
    __shared__ double sP[kBGramChunk + kMaxK], sQ[kBGramChunk + kMaxK], sr[kBGramChunk];
    __shared__ double sh[kNT];
    const int b = blockIdx.y;
    const BatchDyn d = dyn[b];
    if (d.done) return;
    const BatchProb P = prob[b];
    const int k = d.kcur, tot = k * k + k, T = N * N + N;
    const int64_t n = P.n;
    const double *Pc = Ph + P.hbase + (int64_t)d.cur_off * n;
    const double *Qc = Qh + P.hbase + (int64_t)d.cur_off * n;
    const double *rb = r + P.row0;
    const int64_t lo = n * blockIdx.x / kBGX, hi = n * (blockIdx.x + 1) / kBGX;
    double *out = part + ((int64_t)b * kBGX + blockIdx.x) * T;
    if (k == 1) {
        double q0 = 0.0, q1 = 0.0, g0 = 0.0, g1 = 0.0;
        int64_t i = lo + threadIdx.x;
        for (; i + kNT < hi; i += 2 * kNT) {
            const double p0 = Pc[i], p1 = Pc[i + kNT];
            q0 += Qc[i] * p0;
            q1 += Qc[i + kNT] * p1;
            g0 += p0 * rb[i];
            g1 += p1 * rb[i + kNT];
        }
        if (i < hi) {
            q0 += Qc[i] * Pc[i];
            g0 += Pc[i] * rb[i];
        }
        const double qp = block_sum(q0 + q1, sh);
        const double pr = block_sum(g0 + g1, sh);
        if (threadIdx.x == 0) {
            out[0] = qp;
            out[1] = pr;
        }
        return;
    }
    const int R = kBGramChunk / k;   // rows per chunk
    const int ld = R + 1;            // padded column stride
    constexpr int OUT = (kMaxK * kMaxK + kMaxK + kNT - 1) / kNT;
    double acc[OUT];
#pragma unroll
    for (int o = 0; o < OUT; ++o) acc[o] = 0.0;
    for (int64_t r0 = lo; r0 < hi; r0 += R) {
        const int rows = (int)min<int64_t>(R, hi - r0);
        for (int w = threadIdx.x; w < R * k; w += kNT) {
            const int a = w / R, rr = w - a * R;   // consecutive threads: consecutive rows of column a
            const bool in = rr < rows;
            sP[a * ld + rr] = in ? Pc[(int64_t)a * n + r0 + rr] : 0.0;
            sQ[a * ld + rr] = in ? Qc[(int64_t)a * n + r0 + rr] : 0.0;
        }
        for (int rr = threadIdx.x; rr < R; rr += kNT) sr[rr] = rr < rows ? rb[r0 + rr] : 0.0;
        __syncthreads();
#pragma unroll
        for (int o = 0; o < OUT; ++o) {
            const int idx = threadIdx.x + o * kNT;
            if (idx < tot) {
                const bool pr = idx >= k * k;
                const int a = pr ? idx - k * k : idx / k;
                const double *xv = pr ? sP + a * ld : sQ + a * ld;
                const double *yv = pr ? sr : sP + (idx - a * k) * ld;
                double s0 = 0.0, s1 = 0.0;
                int rr = 0;
                for (; rr + 1 < rows; rr += 2) {
                    s0 += xv[rr] * yv[rr];
                    s1 += xv[rr + 1] * yv[rr + 1];
                }
                if (rr < rows) s0 += xv[rr] * yv[rr];
                acc[o] += s0 + s1;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < OUT; ++o) {
        const int idx = threadIdx.x + o * kNT;
        if (idx < tot) out[idx] = acc[o];
    }
}

// Delta^+ (stored as history block nblk), alpha = Delta^+ gamma; rank 0 stops the problem
__global__ __launch_bounds__(kNT) void k_bpinv(int N, const BatchProb *__restrict__ prob, BatchDyn *__restrict__ dyn,
                                               const double *__restrict__ part, double *__restrict__ Dp,
                                               int32_t *__restrict__ blk_off, int32_t *__restrict__ blk_k,
                                               int64_t *__restrict__ blk_dp, double *__restrict__ alpha,
                                               double *__restrict__ gamma) {
    __shared__ double A[kMaxK * kMaxK], V[kMaxK * kMaxK], G[kMaxK * kMaxK];
    __shared__ double gam[kMaxK], sh[kNT];
    __shared__ int rank;
    const int b = blockIdx.x;
    BatchDyn *dp = dyn + b;
    if (dp->done) return;
    const BatchProb P = prob[b];
    const int k = dp->kcur, tot = k * k + k, T = N * N + N;
    for (int idx = threadIdx.x; idx < tot; idx += kNT) {
        double s = 0.0;
        for (int u = 0; u < kBGX; ++u) s += part[((int64_t)b * kBGX + u) * T + idx];
        if (idx < k * k) G[idx] = s;
        else gam[idx - k * k] = s;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < k * k; w += kNT) {
        const int i = w / k, j = w - i * k;
        A[w] = 0.5 * (G[i * k + j] + G[j * k + i]);
    }
    __syncthreads();
    pinv_sym_lds(k, A, V, G, sh, &rank);
    const int64_t dpo = dp->dp_used;
    double *Dout = Dp + P.colbase * N + dpo;
    for (int w = threadIdx.x; w < k * k; w += kNT) Dout[w] = G[w];
    for (int a = threadIdx.x; a < k; a += kNT) {
        double s = 0.0;
        for (int c = 0; c < k; ++c) s += G[a * k + c] * gam[c];
        alpha[(int64_t)b * kMaxK + a] = s;
        gamma[(int64_t)b * kMaxK + a] = gam[a];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int j = dp->nblk;
        blk_off[P.colbase + j] = dp->cur_off;
        blk_k[P.colbase + j] = k;
        blk_dp[P.colbase + j] = dpo;
        dp->nblk = j + 1;
        dp->dp_used = dpo + (int64_t)k * k;
        dp->rank = rank;
        if (rank == 0) {
            dp->done = 1;
            dp->status = BA_ERR_BREAKDOWN;
        }
    }
}

// x += P_cur alpha, r -= Q_cur alpha, z = D^-1 r, and partials of r^T r and r^T z per
// problem.  Each of the kBUX blocks of a problem takes camera blocks of CB = kNT / 9
// poses in turn: a thread per row for the update (the rows stay in LDS), then a
// thread per pose for its 9 x 9 solve.
__global__ __launch_bounds__(kNT) void k_bupdate(const BatchProb *__restrict__ prob, const BatchDyn *__restrict__ dyn,
                                                 const double *__restrict__ Ph, const double *__restrict__ Qh,
                                                 const double *__restrict__ alpha, const double *__restrict__ Dchol,
                                                 double *__restrict__ x, double *__restrict__ r,
                                                 double *__restrict__ z, double *__restrict__ part) {
    constexpr int CB = kNT / 9;
    __shared__ double sr[CB * 9], sh[kNT], al[kMaxK];
    const int b = blockIdx.y;
    const BatchDyn d = dyn[b];
    if (d.done) return;
    const BatchProb P = prob[b];
    const int k = d.kcur;
    const int t = threadIdx.x;
    for (int a = t; a < k; a += kNT) al[a] = alpha[(int64_t)b * kMaxK + a];
    __syncthreads();
    const double *Pc = Ph + P.hbase + (int64_t)d.cur_off * P.n;
    const double *Qc = Qh + P.hbase + (int64_t)d.cur_off * P.n;
    double rr = 0.0, rz = 0.0;
    for (int c0 = blockIdx.x * CB; c0 < P.np; c0 += gridDim.x * CB) {
        const int cams = min(CB, P.np - c0);
        if (t < cams * 9) {
            const int64_t row = (int64_t)c0 * 9 + t;
            double dx = 0.0, dr = 0.0;
            for (int a = 0; a < k; ++a) {
                dx += Pc[(int64_t)a * P.n + row] * al[a];
                dr += Qc[(int64_t)a * P.n + row] * al[a];
            }
            const int64_t g = P.row0 + row;
            x[g] += dx;
            const double v = r[g] - dr;
            r[g] = v;
            sr[t] = v;
            rr += v * v;
        }
        __syncthreads();
        if (t < cams) {
            double rc[9], zc[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) rc[e] = sr[t * 9 + e];
            chol9_solve(Dchol + (int64_t)(P.cam0 + c0 + t) * 45, rc, zc);
            const int64_t g = P.row0 + (int64_t)(c0 + t) * 9;
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                z[g + e] = zc[e];
                rz += rc[e] * zc[e];
            }
        }
        __syncthreads();
    }
    rr = block_sum(rr, sh);
    rz = block_sum(rz, sh);
    if (t == 0) {
        part[((int64_t)b * kBUX + blockIdx.x) * 2] = rr;
        part[((int64_t)b * kBUX + blockIdx.x) * 2 + 1] = rz;
    }
}

// stop test, tau-test (t = gamma^T alpha / r^T D^-1 r), width of the next block, the
// history capacity check and the per-problem launch flags of the S products
__global__ void k_bscalars(int B, int N, double tau, double eps, const BatchProb *__restrict__ prob,
                           BatchDyn *__restrict__ dyn, const double *__restrict__ part,
                           const double *__restrict__ alpha, const double *__restrict__ gamma,
                           int32_t *__restrict__ skip_single, int32_t *__restrict__ skip_multi) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    BatchDyn d = dyn[b];
    if (d.done) {
        skip_single[b] = 1;
        skip_multi[b] = 1;
        return;
    }
    double rr = 0.0, rho = 0.0;
    for (int u = 0; u < kBUX; ++u) {
        rr += part[((int64_t)b * kBUX + u) * 2];
        rho += part[((int64_t)b * kBUX + u) * 2 + 1];
    }
    double ga = 0.0;
    for (int a = 0; a < d.kcur; ++a) ga += gamma[(int64_t)b * kMaxK + a] * alpha[(int64_t)b * kMaxK + a];
    d.rr = rr;
    d.rho = rho;
    d.iters += 1;
    d.multi = 0;
    d.kn = 1;
    if (sqrt(rr) < eps * sqrt(d.rr0)) {
        d.done = 1;
        d.status = BA_OK;
    } else {
        // the tau-test is taken (and counted) on the last allowed iteration too, as in
        // the single-problem solver, whose count includes the block it would build next
        d.t = rho > 0.0 ? ga / rho : INFINITY;
        d.multi = (N > 1 && d.t < tau) ? 1 : 0;
        d.kn = d.multi ? N : 1;
        if (d.hcols + d.kn > prob[b].cap) {
            d.done = 1;
            d.status = BA_ERR_WORKSPACE;
            d.multi = 0;
        } else {
            d.multi_steps += d.multi;
            if (d.iters >= d.max_it) {
                d.done = 1;
                d.status = BA_MAXITER;
            }
        }
    }
    dyn[b] = d;
    skip_single[b] = d.done || d.multi;
    skip_multi[b] = d.done || !d.multi;
}

// Phi[col][p] = Q_hist[:, col]^T z restricted to subset p, for every history column of
// every running problem (one wavefront per subset, fixed-order reductions)
__global__ __launch_bounds__(kNT) void k_bphi(int N, const BatchProb *__restrict__ prob,
                                              const BatchDyn *__restrict__ dyn, const double *__restrict__ Qh,
                                              const double *__restrict__ z, double *__restrict__ Phi) {
    const int b = blockIdx.y;
    const BatchDyn d = dyn[b];
    if (d.done) return;
    const BatchProb P = prob[b];
    const double *zb = z + P.row0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // a fixed grid whatever the history width: block x takes columns x, x + gridDim.x, ...
    for (int col = blockIdx.x; col < d.hcols; col += gridDim.x) {
    const double *q = Qh + P.hbase + (int64_t)col * P.n;
    for (int p = wave; p < N; p += kNT / 64) {
        const int64_t lo = (int64_t)p * P.gs * 9;
        const int64_t hi = (p == N - 1) ? (int64_t)P.n : (int64_t)(p + 1) * P.gs * 9;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;   // four rows per lane in flight
        int64_t i = lo + lane;
        for (; i + 192 < hi; i += 256) {
            a0 += q[i] * zb[i];
            a1 += q[i + 64] * zb[i + 64];
            a2 += q[i + 128] * zb[i + 128];
            a3 += q[i + 192] * zb[i + 192];
        }
        for (; i < hi; i += 64) a0 += q[i] * zb[i];
        const double acc = wave_sum((a0 + a1) + (a2 + a3));
        if (lane == 0) Phi[(P.colbase + col) * N + p] = acc;
    }
    }
}

// beta rows of history block j: beta[off_j + a][p] = sum_c Delta_j^+[a][c] Phi_(off_j + c, p);
// for a one-column next block the subsets' Phi are summed first (Z = D^-1 r)
__global__ __launch_bounds__(kNT) void k_bbeta(int N, const BatchProb *__restrict__ prob,
                                               const BatchDyn *__restrict__ dyn, const int32_t *__restrict__ blk_off,
                                               const int32_t *__restrict__ blk_k, const int64_t *__restrict__ blk_dp,
                                               const double *__restrict__ Dp, const double *__restrict__ Phi,
                                               double *__restrict__ beta) {
    const int b = blockIdx.y;
    const BatchDyn d = dyn[b];
    if (d.done) return;
    const BatchProb P = prob[b];
    // a fixed grid whatever the number of blocks: block x takes blocks x, x + gridDim.x, ...
    for (int j = blockIdx.x; j < d.nblk; j += gridDim.x) {
    const int off = blk_off[P.colbase + j], kj = blk_k[P.colbase + j];
    const double *D = Dp + P.colbase * N + blk_dp[P.colbase + j];
    const double *F = Phi + P.colbase * N;
    const int kn = d.kn;
    // rows of hist_ldb(N) values; a multidirectional block's are padded with zeros
    const int ldb = hist_ldb(N), w_row = kn == 1 ? 1 : ldb;
    for (int w = threadIdx.x; w < kj * w_row; w += kNT) {
        const int a = w / w_row, p = w - a * w_row;
        double s = 0.0;
        if (p < kn) {
            for (int c = 0; c < kj; ++c) {
                double f;
                if (kn == 1) {
                    f = 0.0;
                    for (int q = 0; q < N; ++q) f += F[(int64_t)(off + c) * N + q];
                } else {
                    f = F[(int64_t)(off + c) * N + p];
                }
                s += D[a * kj + c] * f;
            }
        }
        beta[(P.colbase + off + a) * ldb + p] = s;
    }
    }
}

// Sums over the history of one row: ap[j] += sum_col P_hist[row, col] beta[col][j]
// (and aq with Q_hist), four columns per step so that four loads per lane are in flight.
// beta rows are ldb long; outputs beyond the block's width read the zero padding.
template <int KB, bool WITH_Q>
__device__ inline void bhist_rows(const double *__restrict__ ph, const double *__restrict__ qh, int64_t n, int h,
                                  const double *__restrict__ bt, int ldb, double *ap, double *aq) {
    int col = 0;
    for (; col + 4 <= h; col += 4) {
        double hp[4], hq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            hp[u] = ph[(int64_t)(col + u) * n];
            if (WITH_Q) hq[u] = qh[(int64_t)(col + u) * n];
        }
        const double *bc = bt + (int64_t)col * ldb;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                ap[j] += hp[u] * bc[u * ldb + j];
                if (WITH_Q) aq[j] += hq[u] * bc[u * ldb + j];
            }
        }
    }
    for (; col < h; ++col) {
        const double hp = ph[(int64_t)col * n];
        const double hq = WITH_Q ? qh[(int64_t)col * n] : 0.0;
        const double *bc = bt + (int64_t)col * ldb;
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            ap[j] += hp * bc[j];
            if (WITH_Q) aq[j] += hq * bc[j];
        }
    }
}

// New block: P_new[:, p] = Z_p - sum_col P_hist[:, col] beta[col][p] into history columns
// hcols.. (and the staging vector of the one-column S product); multidirectional blocks
// also Q_new[:, p] = (S Z)_p - sum_col Q_hist[:, col] beta[col][p] (eq. (19)).
// One wavefront per 64 rows of a problem and KB next-block columns.
template <int KB>
__global__ __launch_bounds__(64) void k_bhist(int N, int64_t ntot, const BatchProb *__restrict__ prob,
                                              const BatchDyn *__restrict__ dyn, double *__restrict__ Ph,
                                              double *__restrict__ Qh, const double *__restrict__ beta,
                                              const double *__restrict__ z, const double *__restrict__ Y,
                                              double *__restrict__ pstage) {
    const int b = blockIdx.y;
    const BatchDyn d = dyn[b];
    if (d.done) return;
    const int p0 = blockIdx.z * KB;
    if (p0 >= d.kn) return;
    const BatchProb P = prob[b];
    const int64_t row = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (row >= P.n) return;
    const int ldb = hist_ldb(N);
    const double *bt = beta + P.colbase * ldb;
    const double *ph = Ph + P.hbase + row;
    const double *qh = Qh + P.hbase + row;
    const double zr = z[P.row0 + row];
    if (!d.multi) {   // one-column block: P only; S P_new is formed from the staging vector
        double ap = 0.0;
        bhist_rows<1, false>(ph, qh, P.n, d.hcols, bt, ldb, &ap, nullptr);
        const double pn = zr - ap;
        Ph[P.hbase + (int64_t)d.hcols * P.n + row] = pn;
        pstage[P.row0 + row] = pn;
        return;
    }
    double ap[KB], aq[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        ap[j] = 0.0;
        aq[j] = 0.0;
    }
    bhist_rows<KB, true>(ph, qh, P.n, d.hcols, bt + p0, ldb, ap, aq);
    const int grp = subset_of((int)(row / 9), P.gs, N);
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        const int p = p0 + j;
        if (p >= d.kn) continue;
        const double base = grp == p ? zr : 0.0;
        Ph[P.hbase + (int64_t)(d.hcols + p) * P.n + row] = base - ap[j];
        Qh[P.hbase + (int64_t)(d.hcols + p) * P.n + row] = Y[(int64_t)p * ntot + P.row0 + row] - aq[j];
    }
}

// Q of a one-column block: copy S P_new from the staging vector into the history
__global__ void k_bqcopy(const BatchProb *__restrict__ prob, const BatchDyn *__restrict__ dyn,
                         const double *__restrict__ qstage, double *__restrict__ Qh, const int32_t *__restrict__ only) {
    const int b = blockIdx.y;
    const BatchDyn d = dyn[b];
    if (d.done || d.multi || (only && !only[b])) return;
    const BatchProb P = prob[b];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * blockDim.x)
        Qh[P.hbase + (int64_t)d.hcols * P.n + i] = qstage[P.row0 + i];
}

// the new block becomes the current one
__global__ void k_badvance(int B, BatchDyn *__restrict__ dyn, const int32_t *__restrict__ only) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || dyn[b].done || (only && !only[b])) return;
    BatchDyn d = dyn[b];
    d.cur_off = d.hcols;
    d.kcur = d.kn;
    d.hcols += d.kn;
    dyn[b] = d;
}

// per-problem |bt + Sx|^2 and |bt|^2; btp = bt + Sx (the right-hand side of the
// correction equation S d = -bt - S x, in the solvers' S x = -bt form) when given
__global__ __launch_bounds__(kNT) void k_bresid_rows(const BatchProb *__restrict__ prob, const double *__restrict__ bt,
                                                     const double *__restrict__ Sx, double *__restrict__ btp,
                                                     double *__restrict__ part, const int32_t *__restrict__ only) {
    __shared__ double sh[kNT];
    const int b = blockIdx.y;
    if (only && !only[b]) return;
    const BatchProb P = prob[b];
    double a0 = 0.0, a1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * kNT) {
        const int64_t g = P.row0 + i;
        const double v = bt[g] + Sx[g];
        if (btp) btp[g] = v;
        a0 += v * v;
        a1 += bt[g] * bt[g];
    }
    a0 = block_sum(a0, sh);
    a1 = block_sum(a1, sh);
    if (threadIdx.x == 0) {
        part[((int64_t)b * kBUX + blockIdx.x) * 2] = a0;
        part[((int64_t)b * kBUX + blockIdx.x) * 2 + 1] = a1;
    }
}

__global__ void k_bresid_sum(int B, const double *__restrict__ part, double *__restrict__ out,
                             const int32_t *__restrict__ only) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || (only && !only[b])) return;
    double a0 = 0.0, a1 = 0.0;
    for (int u = 0; u < kBUX; ++u) {
        a0 += part[((int64_t)b * kBUX + u) * 2];
        a1 += part[((int64_t)b * kBUX + u) * 2 + 1];
    }
    out[2 * b] = a0;
    out[2 * b + 1] = a1;
}

// FP64 refinement step of the problems flagged in `only`: xprev = x, x += d on their rows
__global__ void k_bouter_step(const BatchProb *__restrict__ prob, const int32_t *__restrict__ only,
                              double *__restrict__ x, const double *__restrict__ d, double *__restrict__ xprev) {
    const int b = blockIdx.y;
    if (!only[b]) return;
    const BatchProb P = prob[b];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = P.row0 + i;
        const double v = x[g];
        xprev[g] = v;
        x[g] = v + d[g];
    }
}

// x = xprev on the rows of the problems flagged in `only` (a correction that did not help)
__global__ void k_brevert(const BatchProb *__restrict__ prob, const int32_t *__restrict__ only,
                          double *__restrict__ x, const double *__restrict__ xprev) {
    const int b = blockIdx.y;
    if (!only[b]) return;
    const BatchProb P = prob[b];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * blockDim.x)
        x[P.row0 + i] = xprev[P.row0 + i];
}

// ---------------------------------------------------------------- launchers

void launch_bouter_step(const BatchLaunch &L, const int32_t *only, double *x, const double *d, double *xprev,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_bouter_step, dim3(kBUX, L.B), dim3(256), 0, s, L.prob, only, x, d, xprev);
}

void launch_brevert(const BatchLaunch &L, const int32_t *only, double *x, const double *xprev, hipStream_t s) {
    hipLaunchKernelGGL(k_brevert, dim3(kBUX, L.B), dim3(256), 0, s, L.prob, only, x, xprev);
}

void launch_bresidual(const BatchLaunch &L, const double *bt, const double *Sx, double *btp, double *out,
                      hipStream_t s, const int32_t *only) {
    hipLaunchKernelGGL(k_bresid_rows, dim3(kBUX, L.B), dim3(kNT), 0, s, L.prob, bt, Sx, btp, L.upart, only);
    hipLaunchKernelGGL(k_bresid_sum, dim3((L.B + 63) / 64), dim3(64), 0, s, L.B, L.upart, out, only);
}

void launch_bstart(const BatchLaunch &L, const double *bt, const double *x0, const int32_t *off, hipStream_t s,
                   const int32_t *only, int max_iter, const int32_t *max_it) {
    hipLaunchKernelGGL(k_bstart_rows, dim3(kBUX, L.B), dim3(kNT), 0, s, L.prob, bt, x0, L.x, L.r, L.upart, only);
    hipLaunchKernelGGL(k_bstart, dim3((L.B + 63) / 64), dim3(64), 0, s, L.B, L.upart, off, L.dyn, L.skip_single,
                       L.skip_multi, only, max_iter, max_it);
    hipLaunchKernelGGL(k_bseed, dim3((L.max_np + 127) / 128, L.B), dim3(128), 0, s, L.B, L.prob, L.dyn, L.Dchol, L.r,
                       L.Ph, L.pstage, only);
}

void launch_bqcopy_advance(const BatchLaunch &L, hipStream_t s, const int32_t *only) {
    hipLaunchKernelGGL(k_bqcopy, dim3((unsigned)((L.max_n + 255) / 256), L.B), dim3(256), 0, s, L.prob, L.dyn,
                       L.qstage, L.Qh, only);
    hipLaunchKernelGGL(k_badvance, dim3((L.B + 63) / 64), dim3(64), 0, s, L.B, L.dyn, only);
}

void launch_biter_head(const BatchLaunch &L, double tau, double eps, hipStream_t s) {
    hipLaunchKernelGGL(k_bgram, dim3(kBGX, L.B), dim3(kNT), 0, s, L.N, L.prob, L.dyn, L.Ph, L.Qh, L.r, L.gpart);
    hipLaunchKernelGGL(k_bpinv, dim3(L.B), dim3(kNT), 0, s, L.N, L.prob, L.dyn, L.gpart, L.Dp, L.blk_off, L.blk_k,
                       L.blk_dp, L.alpha, L.gamma);
    hipLaunchKernelGGL(k_bupdate, dim3(kBUX, L.B), dim3(kNT), 0, s, L.prob, L.dyn, L.Ph, L.Qh, L.alpha, L.Dchol, L.x,
                       L.r, L.z, L.upart);
    hipLaunchKernelGGL(k_bscalars, dim3((L.B + 63) / 64), dim3(64), 0, s, L.B, L.N, tau, eps, L.prob, L.dyn,
                       L.upart, L.alpha, L.gamma, L.skip_single, L.skip_multi);
}

void launch_biter_tail(const BatchLaunch &L, hipStream_t s) {
    hipLaunchKernelGGL(k_bphi, dim3(kBatchPhiBlocks, L.B), dim3(kNT), 0, s, L.N, L.prob, L.dyn, L.Qh, L.z, L.Phi);
    hipLaunchKernelGGL(k_bbeta, dim3(kBatchBetaBlocks, L.B), dim3(kNT), 0, s, L.N, L.prob, L.dyn, L.blk_off, L.blk_k,
                       L.blk_dp, L.Dp, L.Phi, L.beta);
    const unsigned tiles = (unsigned)((L.max_n + 63) / 64);
    if (L.N <= 16)
        hipLaunchKernelGGL((k_bhist<16>), dim3(tiles, L.B, 1), dim3(64), 0, s, L.N, L.ntot, L.prob, L.dyn, L.Ph,
                           L.Qh, L.beta, L.z, L.Y, L.pstage);
    else
        hipLaunchKernelGGL((k_bhist<16>), dim3(tiles, L.B, (L.N + 15) / 16), dim3(64), 0, s, L.N, L.ntot, L.prob,
                           L.dyn, L.Ph, L.Qh, L.beta, L.z, L.Y, L.pstage);
}

}  // namespace ba
