// Camera-space vector kernels of the Krylov solvers: block-Jacobi
// preconditioner, deterministic reductions (fixed grid, fixed-order trees),
// the PCG recurrences of Algorithm 1, and the block recurrences of Algorithm 2
// (Gram matrices, pseudo-inverse, tau-test, full reorthogonalisation).
// All FP64.
#include "ba_internal.h"
#include "kernels.h"
#include "dev_la.h"

namespace ba {

// ---------------------------------------------------------------- preconditioner

// DP x DP blocks (pose dimension 9, or 6 for extrinsics only); the factors are packed,
// DP (DP + 1) / 2 values per camera
template <int DP>
__global__ void k_precond(int np, const double *__restrict__ Dchol, const double *__restrict__ r,
                          double *__restrict__ z) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= np) return;
    double rc[DP], zc[DP];
    for (int i = 0; i < DP; ++i) rc[i] = r[(int64_t)c * DP + i];
    chol_solve_packed<DP>(Dchol + (int64_t)c * (DP * (DP + 1) / 2), rc, zc);
    for (int i = 0; i < DP; ++i) z[(int64_t)c * DP + i] = zc[i];
}

void launch_precond(int np, const double *Dchol, const double *r, double *z, hipStream_t s, int dp) {
    if (dp == 6) hipLaunchKernelGGL(k_precond<6>, dim3((np + 127) / 128), dim3(128), 0, s, np, Dchol, r, z);
    else hipLaunchKernelGGL(k_precond<9>, dim3((np + 127) / 128), dim3(128), 0, s, np, Dchol, r, z);
}

// z = D^-1 r and per-block partial sums of sum_i a[i] * z[i]
template <int DP>
__global__ __launch_bounds__(kNT) void k_precond_dot(int np, const double *__restrict__ Dchol,
                                                     const double *__restrict__ r, const double *__restrict__ a,
                                                     double *__restrict__ z, double *__restrict__ partials,
                                                     const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    __shared__ double sh[kNT];
    double acc = 0.0;
    for (int c = blockIdx.x * kNT + threadIdx.x; c < np; c += gridDim.x * kNT) {
        double rc[DP], zc[DP];
        for (int i = 0; i < DP; ++i) rc[i] = r[(int64_t)c * DP + i];
        chol_solve_packed<DP>(Dchol + (int64_t)c * (DP * (DP + 1) / 2), rc, zc);
        for (int i = 0; i < DP; ++i) {
            z[(int64_t)c * DP + i] = zc[i];
            acc += a[(int64_t)c * DP + i] * zc[i];
        }
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

void launch_pcg_precond_phi(int np, const double *Dchol, const double *r, const double *Q, double *z,
                            double *partials, const double *done, hipStream_t s, int dp) {
    if (dp == 6)
        hipLaunchKernelGGL(k_precond_dot<6>, dim3(kRedBlocks), dim3(kNT), 0, s, np, Dchol, r, Q, z, partials, done);
    else
        hipLaunchKernelGGL(k_precond_dot<9>, dim3(kRedBlocks), dim3(kNT), 0, s, np, Dchol, r, Q, z, partials, done);
}


// ---------------------------------------------------------------- reductions

// one wavefront per output d
__global__ __launch_bounds__(64) void k_finalize(const double *__restrict__ partials, int nd,
                                                 double *__restrict__ out) {
    const int d = blockIdx.x;
    const double s = wave_partials(partials + d, nd, kRedBlocks);
    if (threadIdx.x == 0) out[d] = s;
}

void launch_finalize(const double *partials, int nd, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(nd), dim3(64), 0, s, partials, nd, out);
}

// ---------------------------------------------------------------- refinement

// r = -bt - Sx, btp = -r; partials of |r|^2 and |bt|^2 (2 per block)
__global__ __launch_bounds__(kNT) void k_residual_refine(int64_t n, const double *__restrict__ bt,
                                                         const double *__restrict__ Sx, double *__restrict__ r,
                                                         double *__restrict__ btp, double *__restrict__ partials) {
    __shared__ double sh[kNT];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
        const double v = -bt[i] - Sx[i];
        r[i] = v;
        btp[i] = -v;
        a += v * v;
        b += bt[i] * bt[i];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x * 2] = a;
        partials[blockIdx.x * 2 + 1] = b;
    }
}

void launch_residual_refine(int64_t n, const double *bt, const double *Sx, double *r, double *btp,
                            double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_residual_refine, dim3(kRedBlocks), dim3(kNT), 0, s, n, bt, Sx, r, btp, partials);
}

__global__ void k_axpy(int64_t n, double a, const double *__restrict__ x, double *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

void launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(kRedBlocks), dim3(kNT), 0, s, n, a, x, y);
}

// ---------------------------------------------------------------- Algorithm 1

// r0 = -b~ - S x0 (Sx nullable for x0 = 0); partial |r0|^2
__global__ __launch_bounds__(kNT) void k_pcg_init(int64_t n, const double *__restrict__ bt,
                                                  const double *__restrict__ Sx, double *__restrict__ r,
                                                  double *__restrict__ partials) {
    __shared__ double sh[kNT];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
        double v = -bt[i] - (Sx ? Sx[i] : 0.0);
        r[i] = v;
        acc += v * v;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

void launch_pcg_init(int64_t n, const double *bt, const double *Sx, double *r, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_init, dim3(kRedBlocks), dim3(kNT), 0, s, n, bt, Sx, r, partials);
}

// sc[SC_RR] = sum of the partials; the first call (sc[SC_RR0] < 0) also sets SC_RR0
__global__ __launch_bounds__(64) void k_pcg_rr(const double *__restrict__ partials, double *__restrict__ sc) {
    const double s = wave_partials(partials, 1, kRedBlocks);
    if (threadIdx.x != 0) return;
    sc[SC_RR] = s;
    if (sc[SC_RR0] < 0.0) sc[SC_RR0] = s;
}

void launch_pcg_rr(const double *partials_rr, double *sc, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_rr, dim3(1), dim3(64), 0, s, partials_rr, sc);
}

// End of a PCG iteration on the device: |r_{i+1}|^2 from the partials, the
// iteration count, the stop test |r_{i+1}| < eps |r_0| (Alg. 1) and the iteration
// cap.  Sets sc[SC_DONE] (after which every kernel of later iterations returns at
// once) and sc[SC_STATUS].  trace (nullable) receives |r_{i+1}| / |r_0|.
__global__ __launch_bounds__(64) void k_pcg_step_end(const double *__restrict__ partials, double *__restrict__ sc,
                                                     double eps, int max_iter, double *__restrict__ trace) {
    if (sc[SC_DONE] != 0.0) return;
    const double s = wave_partials(partials, 1, kRedBlocks);
    if (threadIdx.x != 0) return;
    if (sc[SC_BREAK] != 0.0) {
        sc[SC_DONE] = 1.0;
        sc[SC_STATUS] = (double)BA_ERR_BREAKDOWN;
        return;
    }
    const double it = sc[SC_ITER] + 1.0;
    sc[SC_ITER] = it;
    sc[SC_RR] = s;
    const double rr0 = sc[SC_RR0];
    if (trace) trace[(int)it - 1] = sqrt(s / rr0);
    if (sqrt(s) < eps * sqrt(rr0)) {
        sc[SC_DONE] = 1.0;
        sc[SC_STATUS] = (double)BA_OK;
    } else if (it >= (double)max_iter) {
        sc[SC_DONE] = 1.0;
        sc[SC_STATUS] = (double)BA_MAXITER;
    }
}

void launch_pcg_step_end(const double *partials_rr, double *sc, double eps, int max_iter, double *trace,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_step_end, dim3(1), dim3(64), 0, s, partials_rr, sc, eps, max_iter, trace);
}

// Delta = Q^T P, gamma = P^T r from the partials; alpha = gamma / Delta;
// x += alpha P, r -= alpha Q; partial |r|^2
__global__ __launch_bounds__(kNT) void k_pcg_update_xr(int64_t n, const double *__restrict__ pdq, int npdq,
                                                       double *__restrict__ sc, double *__restrict__ x,
                                                       double *__restrict__ r, const double *__restrict__ P,
                                                       const double *__restrict__ Q,
                                                       double *__restrict__ partials) {
    if (sc[SC_DONE] != 0.0) return;
    __shared__ double sh[kNT];
    __shared__ double s_alpha;
    if (threadIdx.x < 64) {
        const double D = wave_partials(pdq, 2, npdq);
        const double g = wave_partials(pdq + 1, 2, npdq);
        const double al = D > 0.0 ? g / D : 0.0;
        if (threadIdx.x == 0) s_alpha = al;
        if (threadIdx.x == 0 && blockIdx.x == 0) {
            sc[SC_DELTA] = D;
            sc[SC_GAMMA] = g;
            sc[SC_ALPHA] = al;
            if (!(D > 0.0)) sc[SC_BREAK] = 1.0;
        }
    }
    __syncthreads();
    const double al = s_alpha;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
        x[i] += al * P[i];
        double v = r[i] - al * Q[i];
        r[i] = v;
        acc += v * v;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

void launch_pcg_update_xr(int64_t n, const double *partials_dq, int n_dq, double *sc, double *x, double *r,
                          const double *P, const double *Q, double *partials_rr, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_update_xr, dim3(kRedBlocks), dim3(kNT), 0, s, n, partials_dq, n_dq, sc, x, r, P, Q,
                       partials_rr);
}

// One kernel for the end of a PCG iteration (Alg. 1) with the block-Jacobi
// preconditioner: alpha = gamma / Delta from npdq pairs of partials (pdq), x += alpha P,
// r -= alpha Q, Z = D^-1 r, and the partial sums of |r|^2 and Phi = Q^T Z.  Block b owns
// the poses [b CB, (b + 1) CB) (CB = kNT / DP), whose rows it updates and whose D^-1
// solves it takes.  The block that arrives last (an agent-scope counter, left zero) adds
// the partials in block order and takes the step-end decisions of k_pcg_step_end (on a
// breakdown flag, the stop test, the iteration cap), then beta = Phi / Delta into the
// scalars for k_pcg_update_p.  As in k_mcg_xrz, the loads that need nothing formed here
// (x, r, P, Q and the Cholesky factor of the thread's camera; threads without a row or a
// camera read the block's first and ignore them) go before the reduction of the partials,
// which are read as pairs with eight loads in flight.
template <int DP>
__global__ __launch_bounds__(kNT) void k_pcg_xrz(int np, const double *__restrict__ pdq, int npdq,
                                                 double *__restrict__ sc, double *__restrict__ x,
                                                 double *__restrict__ r, const double *__restrict__ P,
                                                 const double *__restrict__ Q, const double *__restrict__ Dchol,
                                                 double *__restrict__ z, double *__restrict__ partials,
                                                 uint32_t *__restrict__ ticket, double eps, int max_iter,
                                                 double *__restrict__ trace) {
    if (sc[SC_DONE] != 0.0) return;
    constexpr int CB = kNT / DP;
    constexpr int NL = DP * (DP + 1) / 2;
    __shared__ double sr[CB * DP], sq[CB * DP];
    __shared__ double sh[kNT];
    __shared__ double s_alpha;
    __shared__ int last;
    const int c0 = blockIdx.x * CB;
    const int cams = min(CB, np - c0);
    const int t = threadIdx.x;
    const bool row = t < cams * DP;
    const int64_t i = (int64_t)c0 * DP + (row ? t : 0);
    const double xi = x[i], ri = r[i], pi = P[i], qi = Q[i];
    double Lc[NL];
    {
        const double *Lp = Dchol + (int64_t)(c0 + (t < cams ? t : 0)) * NL;
#pragma unroll
        for (int e = 0; e < NL; ++e) Lc[e] = Lp[e];
    }
    if (t < 64) {
        double D, g;
        wave_pair_sums(pdq, npdq, D, g);
        const double al = D > 0.0 ? g / D : 0.0;
        if (t == 0) {
            s_alpha = al;
            if (blockIdx.x == 0) {
                sc[SC_DELTA] = D;
                sc[SC_GAMMA] = g;
                sc[SC_ALPHA] = al;
                if (!(D > 0.0)) sc[SC_BREAK] = 1.0;
            }
        }
    }
    __syncthreads();
    const double al = s_alpha;
    double rr = 0.0;
    if (row) {
        x[i] = xi + al * pi;
        const double v = ri - al * qi;
        r[i] = v;
        sr[t] = v;
        sq[t] = qi;
        rr = v * v;
    }
    __syncthreads();
    double phi = 0.0;
    if (t < cams) {
        double rc[DP], zc[DP];
#pragma unroll
        for (int e = 0; e < DP; ++e) rc[e] = sr[t * DP + e];
        chol_solve_packed<DP>(Lc, rc, zc);
#pragma unroll
        for (int e = 0; e < DP; ++e) {
            z[(int64_t)(c0 + t) * DP + e] = zc[e];
            phi += sq[t * DP + e] * zc[e];
        }
    }
    rr = block_sum(rr, sh);
    phi = block_sum(phi, sh);
    if (t == 0) {
        partials[2 * blockIdx.x] = rr;
        partials[2 * blockIdx.x + 1] = phi;
        const uint32_t prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || t >= 64) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double srr, sphi;
    wave_pair_sums(partials, gridDim.x, srr, sphi);
    if (t != 0) return;
    __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (sc[SC_BREAK] != 0.0) {
        sc[SC_DONE] = 1.0;
        sc[SC_STATUS] = (double)BA_ERR_BREAKDOWN;
        return;
    }
    const double it = sc[SC_ITER] + 1.0;
    sc[SC_ITER] = it;
    sc[SC_RR] = srr;
    const double rr0 = sc[SC_RR0];
    if (trace) trace[(int)it - 1] = sqrt(srr / rr0);
    if (sqrt(srr) < eps * sqrt(rr0)) {
        sc[SC_DONE] = 1.0;
        sc[SC_STATUS] = (double)BA_OK;
    } else if (it >= (double)max_iter) {
        sc[SC_DONE] = 1.0;
        sc[SC_STATUS] = (double)BA_MAXITER;
    } else {
        sc[SC_PHI] = sphi;
        sc[SC_BETA] = sphi / sc[SC_DELTA];
    }
}

void launch_pcg_xrz(int np, const double *pdq, int npdq, double *sc, double *x, double *r, const double *P,
                    const double *Q, const double *Dchol, double *z, double *partials, uint32_t *ticket, double eps,
                    int max_iter, double *trace, hipStream_t s, int dp) {
    const unsigned nb = (unsigned)mcg_xrz_blocks(np, dp);
    if (dp == 6)
        hipLaunchKernelGGL(k_pcg_xrz<6>, dim3(nb), dim3(kNT), 0, s, np, pdq, npdq, sc, x, r, P, Q, Dchol, z, partials,
                           ticket, eps, max_iter, trace);
    else
        hipLaunchKernelGGL(k_pcg_xrz<9>, dim3(nb), dim3(kNT), 0, s, np, pdq, npdq, sc, x, r, P, Q, Dchol, z, partials,
                           ticket, eps, max_iter, trace);
}

// Phi = Q^T Z from the partials; beta = Phi / Delta; P = Z - beta P.  Without partials
// (pphi null) beta is the one k_pcg_xrz stored.
__global__ __launch_bounds__(kNT) void k_pcg_update_p(int64_t n, const double *__restrict__ pphi,
                                                      double *__restrict__ sc, const double *__restrict__ z,
                                                      double *__restrict__ P) {
    if (sc[SC_DONE] != 0.0) return;
    __shared__ double s_beta;
    if (!pphi) {
        if (threadIdx.x == 0) s_beta = sc[SC_BETA];
    } else if (threadIdx.x < 64) {
        const double phi = wave_partials(pphi, 1, kRedBlocks);
        const double be = phi / sc[SC_DELTA];
        if (threadIdx.x == 0) s_beta = be;
        if (threadIdx.x == 0 && blockIdx.x == 0) {
            sc[SC_PHI] = phi;
            sc[SC_BETA] = be;
        }
    }
    __syncthreads();
    const double be = s_beta;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT)
        P[i] = z[i] - be * P[i];
}

void launch_pcg_update_p(int64_t n, const double *partials_phi, double *sc, const double *z, double *P,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_update_p, dim3(kRedBlocks), dim3(kNT), 0, s, n, partials_phi, sc, z, P);
}

// ---------------------------------------------------------------- Algorithm 2

constexpr int kGramOut = (kMaxK * kMaxK + kMaxK + kNT - 1) / kNT;   // outputs per thread
constexpr int kGramLds = 64 * 1024;                                   // bytes of one row chunk
constexpr int kGramBlocksWide = kRedBlocks;                          // blocks of a k > 1 Gram

// Rows [r0, r0 + rows) of the n x k blocks P and Q (column-major) into LDS row-major
// (sP[rr * k + a]) and of r into sr, by the work-group: consecutive threads take
// consecutive rows of a column, eight elements of each block per thread are loaded before
// any is stored (elements past the end read element 0 and are dropped), so that a
// thread's loads are in flight together rather than one round trip each.
__device__ __forceinline__ void gram_stage(int64_t n, int k, int rows, int64_t r0, const double *__restrict__ P,
                                           const double *__restrict__ Q, const double *__restrict__ r, double *sP,
                                           double *sQ, double *sr) {
    const int tid = threadIdx.x;
    const int tot = rows * k;
    const double rv = r[r0 + (tid < rows ? tid : 0)];
    for (int w0 = tid; w0 < tot; w0 += 8 * kNT) {
        double vp[8], vq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int w = w0 + u * kNT < tot ? w0 + u * kNT : 0;
            const int a = w / rows, rr = w - a * rows;
            vp[u] = P[(int64_t)a * n + r0 + rr];
            vq[u] = Q[(int64_t)a * n + r0 + rr];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int w = w0 + u * kNT;
            if (w < tot) {
                const int a = w / rows, rr = w - a * rows;
                sP[rr * k + a] = vp[u];
                sQ[rr * k + a] = vq[u];
            }
        }
    }
    if (tid < rows) sr[tid] = rv;
    for (int rr = tid + kNT; rr < rows; rr += kNT) sr[rr] = r[r0 + rr];
}

// k > 1: partials[b][a * k + c] = sum_rows Q[:, a] . P[:, c] ; partials[b][k*k + a] = sum_rows P[:, a] . r
// over block b's contiguous row range.  The range is staged through LDS in chunks of R
// rows (R (2k + 1) doubles fit kGramLds), each chunk loaded in one pass so that all its
// loads are in flight together.
__global__ __launch_bounds__(kNT) void k_gram(int64_t n, int k, int R, const double *__restrict__ P,
                                              const double *__restrict__ Q, const double *__restrict__ r,
                                              double *__restrict__ partials) {
    extern __shared__ double gsm[];
    double *sP = gsm, *sQ = gsm + (int64_t)R * k, *sr = sQ + (int64_t)R * k;
    const int tot = k * k + k;
    double acc[kGramOut];
#pragma unroll
    for (int o = 0; o < kGramOut; ++o) acc[o] = 0.0;
    const int64_t lo = n * blockIdx.x / gridDim.x, hi = n * (blockIdx.x + 1) / gridDim.x;
    for (int64_t r0 = lo; r0 < hi; r0 += R) {
        const int rows = (int)(hi - r0 < R ? hi - r0 : R);
        gram_stage(n, k, rows, r0, P, Q, r, sP, sQ, sr);
        __syncthreads();
#pragma unroll
        for (int o = 0; o < kGramOut; ++o) {
            const int idx = threadIdx.x + o * kNT;
            if (idx < tot) {
                // Q[:, a] . P[:, c], or P[:, a] . r for the last k outputs; four running sums
                // keep four LDS reads of each operand in flight
                const bool pr = idx >= k * k;
                const int a = pr ? idx - k * k : idx / k;
                const double *x = pr ? sP + a : sQ + a;
                const double *y = pr ? sr : sP + (idx - a * k);
                const int sy = pr ? 1 : k;
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                int rr = 0;
                for (; rr + 4 <= rows; rr += 4) {
                    s0 += x[rr * k] * y[rr * sy];
                    s1 += x[(rr + 1) * k] * y[(rr + 1) * sy];
                    s2 += x[(rr + 2) * k] * y[(rr + 2) * sy];
                    s3 += x[(rr + 3) * k] * y[(rr + 3) * sy];
                }
                for (; rr < rows; ++rr) s0 += x[rr * k] * y[rr * sy];
                acc[o] += (s0 + s1) + (s2 + s3);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < kGramOut; ++o) {
        const int idx = threadIdx.x + o * kNT;
        if (idx < tot) partials[(int64_t)blockIdx.x * tot + idx] = acc[o];
    }
}

// k >= 16: the same partials with the k x k part on the matrix cores.  Delta's 16 x 16
// tiles (k padded to a multiple of 16) are dealt to the four wavefronts; for each 4 rows of
// a staged chunk a wavefront issues one v_mfma_f64_16x16x4f64 per tile, with
// A[i][kk] = Q[row kk][a0 + i] and B[kk][j] = P[row kk][c0 + j] read from LDS (lane l
// supplies element (l mod 16, l / 16) of A and (l / 16, l mod 16) of B, and holds
// D[l / 16 + 4 e][l mod 16] in accumulator e).  P^T r stays on the vector units.
typedef double dbl4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kNT) void k_gram_mfma(int64_t n, int k, int R, const double *__restrict__ P,
                                                   const double *__restrict__ Q, const double *__restrict__ r,
                                                   double *__restrict__ partials) {
    extern __shared__ double gsm[];
    double *sP = gsm, *sQ = gsm + (int64_t)R * k, *sr = sQ + (int64_t)R * k;
    const int tot = k * k + k;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int T = (k + 15) / 16;
    const int li = lane & 15, lk = lane >> 4;
    dbl4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = dbl4_t{0.0, 0.0, 0.0, 0.0};
    double gacc = 0.0;
    const int64_t lo = n * blockIdx.x / gridDim.x, hi = n * (blockIdx.x + 1) / gridDim.x;
    for (int64_t r0 = lo; r0 < hi; r0 += R) {
        const int rows = (int)(hi - r0 < R ? hi - r0 : R);
        gram_stage(n, k, rows, r0, P, Q, r, sP, sQ, sr);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int tt = wv + 4 * t;
            if (tt < T * T) {
                const int a = (tt / T) * 16 + li, c = (tt - (tt / T) * T) * 16 + li;
                for (int rr = 0; rr < rows; rr += 4) {
                    const int row = rr + lk;
                    const double av = (row < rows && a < k) ? sQ[row * k + a] : 0.0;
                    const double bv = (row < rows && c < k) ? sP[row * k + c] : 0.0;
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
                }
            }
        }
        if (tid < k)
            for (int rr = 0; rr < rows; ++rr) gacc += sP[rr * k + tid] * sr[rr];
        __syncthreads();
    }
    double *out = partials + (int64_t)blockIdx.x * tot;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int tt = wv + 4 * t;
        if (tt < T * T) {
            const int c = (tt - (tt / T) * T) * 16 + li;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int a = (tt / T) * 16 + lk + 4 * e;
                if (a < k && c < k) out[a * k + c] = acc[t][e];
            }
        }
    }
    if (tid < k) out[k * k + tid] = gacc;
}

// sums[idx] = sum over b < nb of partials[b][idx] (idx < tot), one thread per output in
// a fixed order: eight running sums over batches of 24 blocks (24 loads in flight), the
// remainder into the first, then a fixed tree.  Spread over many work-groups, so the
// k (k + 1) sums of a wide block do not wait on one work-group's load latency.
__global__ __launch_bounds__(64) void k_gram_sum(int tot, int nb, const double *__restrict__ partials,
                                                 double *__restrict__ sums) {
    const int idx = blockIdx.x * 64 + threadIdx.x;
    if (idx >= tot) return;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = 0;
    for (; b + 24 <= nb; b += 24) {
        double v[24];
#pragma unroll
        for (int u = 0; u < 24; ++u) v[u] = partials[(int64_t)(b + u) * tot + idx];
#pragma unroll
        for (int u = 0; u < 24; ++u) acc[u & 7] += v[u];
    }
    for (; b < nb; ++b) acc[0] += partials[(int64_t)b * tot + idx];
    sums[idx] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// blocks of the Gram partials (k > 1)
int gram_blocks(int) { return kGramBlocksWide; }

void launch_gram(int64_t n, int k, const double *P, const double *Q, const double *r, double *partials,
                 hipStream_t s) {
    const int nb = gram_blocks(k);
    const int64_t per = (n + nb - 1) / nb;
    const int64_t cap = kGramLds / (int64_t)((2 * k + 1) * sizeof(double));
    const int R = (int)std::max<int64_t>(1, std::min(per, cap));
    const size_t lds = (size_t)R * (2 * k + 1) * sizeof(double);
    if (k >= 16) hipLaunchKernelGGL(k_gram_mfma, dim3(nb), dim3(kNT), lds, s, n, k, R, P, Q, r, partials);
    else hipLaunchKernelGGL(k_gram, dim3(nb), dim3(kNT), lds, s, n, k, R, P, Q, r, partials);
    const int tot = k * k + k;
    hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)((tot + 63) / 64)), dim3(64), 0, s, tot, nb, partials,
                       partials + (int64_t)nb * tot);
}

// Delta (symmetrised) and gamma from the Gram sums (sums[a k + c], then gamma at k k + a);
// Delta^+; alpha = Delta^+ gamma
__global__ __launch_bounds__(kNT) void k_pinv_alpha(int k, const double *__restrict__ sums,
                                                    double *__restrict__ Dp, double *__restrict__ gamma,
                                                    double *__restrict__ alpha, double *__restrict__ sc,
                                                    BlockEntry blk) {
    __shared__ double A[kMaxK * kMaxK], V[kMaxK * kMaxK], G[kMaxK * kMaxK];
    __shared__ double gam[kMaxK], sh[kNT];
    __shared__ int rank;
    const int tid = threadIdx.x;
    const int tot = k * k + k;
    // eight sums per thread in flight (indices past tot read sum 0 and are dropped)
    for (int i0 = tid; i0 < tot; i0 += 8 * kNT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = sums[i0 + u * kNT < tot ? i0 + u * kNT : 0];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * kNT;
            if (idx < k * k) G[idx] = v[u];
            else if (idx < tot) gam[idx - k * k] = v[u];
        }
    }
    __syncthreads();
    for (int w = tid; w < k * k; w += kNT) {
        int i = w / k, j = w - i * k;
        A[w] = 0.5 * (G[i * k + j] + G[j * k + i]);
    }
    __syncthreads();
    pinv_sym_lds(k, A, V, G, sh, &rank);
    for (int w = tid; w < k * k; w += kNT) Dp[w] = G[w];
    for (int a = tid; a < k; a += kNT) {
        double s = 0.0;
        for (int b = 0; b < k; ++b) s += G[a * k + b] * gam[b];
        alpha[a] = s;
        gamma[a] = gam[a];
    }
    if (tid == 0) {
        sc[SC_RANK] = (double)rank;
        if (blk.off) {   // history block table entry of the current block
            blk.off[blk.j] = blk.first;
            blk.k[blk.j] = k;
            blk.dp[blk.j] = blk.dpo;
        }
    }
}

void launch_pinv_alpha(int k, const double *partials, int nblocks, double *Dp, double *gamma, double *alpha,
                       double *sc, hipStream_t s, BlockEntry blk) {
    hipLaunchKernelGGL(k_pinv_alpha, dim3(1), dim3(kNT), 0, s, k, partials + (int64_t)nblocks * (k * k + k), Dp,
                       gamma, alpha, sc, blk);
}

// Stand-alone symmetric pseudo-inverse (test entry point).
__global__ __launch_bounds__(kNT) void k_pinv_sym(int k, const double *__restrict__ Ain, double *__restrict__ Ap,
                                                  int32_t *__restrict__ rank_out) {
    __shared__ double A[kMaxK * kMaxK], V[kMaxK * kMaxK], G[kMaxK * kMaxK];
    __shared__ double sh[kNT];
    __shared__ int rank;
    for (int w = threadIdx.x; w < k * k; w += kNT) A[w] = Ain[w];
    __syncthreads();
    pinv_sym_lds(k, A, V, G, sh, &rank);
    for (int w = threadIdx.x; w < k * k; w += kNT) Ap[w] = G[w];
    if (threadIdx.x == 0 && rank_out) *rank_out = rank;
}

void launch_pinv_sym(int k, const double *A, double *Ap, int32_t *rank, hipStream_t s) {
    hipLaunchKernelGGL(k_pinv_sym, dim3(1), dim3(kNT), 0, s, k, A, Ap, rank);
}

// Alg. 2's stop test and tau-test from |r_{i+1}|^2 and rho = r_{i+1}^T M^-1 r_{i+1}:
// t_i = gamma_i^T alpha_i / rho (ga = gamma_i^T alpha_i); sc[SC_SKIPM], sc[SC_KN] and
// sc[SC_SKIPS] give the next block's width to the kernels launched ahead of the host's
// read-back.  One thread; the values are also returned in v (indexed by SC_*).
struct McgScalars {
    double rr, rho, t, skipm, kn, skips;
};
__device__ inline McgScalars mcg_scalars_form(double rr, double rho, double ga, double rr0, int N, double tau,
                                              double eps) {
    McgScalars v;
    v.rr = rr;
    v.rho = rho;
    v.t = rho > 0.0 ? ga / rho : INFINITY;
    const bool converged = sqrt(rr) < eps * sqrt(rr0);
    const bool multi = N > 1 && v.t < tau && !converged;
    v.skipm = multi ? 0.0 : 1.0;
    v.kn = converged ? 0.0 : multi ? (double)N : 1.0;
    v.skips = (!converged && !multi) ? 0.0 : 1.0;
    return v;
}
__device__ inline void mcg_scalars_put(const McgScalars &v, double *__restrict__ sc) {
    sc[SC_RR] = v.rr;
    sc[SC_RHO] = v.rho;
    sc[SC_T] = v.t;
    sc[SC_SKIPM] = v.skipm;
    sc[SC_KN] = v.kn;
    sc[SC_SKIPS] = v.skips;
}

// One kernel for the end of an iteration of Alg. 2 with the block-Jacobi preconditioner:
// x += P alpha, r -= Q alpha (n x k blocks, column-major), Z = D^-1 r, and the scalars.
// Block b owns the poses [b CB, (b + 1) CB) (CB = kNT / DP), so the rows it updates are
// the rows its D^-1 solves read (kept in LDS).  Each block leaves its |r|^2 and r^T z in
// partials[2 b], [2 b + 1]; the block that arrives last (an agent-scope counter, reset to
// zero by that block) adds them in block order and stores the scalars.
// The kernel is a chain of dependent memory round trips, so every load that needs nothing
// formed here goes first, unconditionally (threads without a row read row 0 and a camera
// without the block's first camera, and ignore them): x, r, the block's first P and Q
// columns, the Cholesky factor of the thread's camera, the scalars already in sc, and
// gamma of a block formed by the pseudo-inverse kernel.  Their latencies then overlap
// the reduction of the Gram partials.
// LR: with the learned low-rank term (XrzLowrank): the rows' U are loaded with the other
// early loads, and the block's 8 sums of U^T r go beside its |r|^2 and r^T D^-1 r.
template <int DP, bool LR>
__global__ __launch_bounds__(kNT) void k_mcg_xrz(int np, int k, const double *__restrict__ P,
                                                 const double *__restrict__ Q, double *alpha,
                                                 double *__restrict__ x, double *__restrict__ r,
                                                 const double *__restrict__ Dchol, double *__restrict__ z,
                                                 double *__restrict__ partials, uint32_t *__restrict__ ticket,
                                                 double *gamma, double *__restrict__ sc,
                                                 double *__restrict__ host_sc, double tag, int N, double tau,
                                                 double eps, XrzGram g1, XrzLowrank lr) {
    constexpr int CB = kNT / DP;
    constexpr int NL = DP * (DP + 1) / 2;
    __shared__ double sr[CB * DP];
    __shared__ double sh[kNT];
    __shared__ double al[kMaxK], ga_sh[kMaxK];
    __shared__ double rank_sh;
    __shared__ double ush[4 * kLowRank];
    __shared__ int last;
    const int64_t n = (int64_t)np * DP;
    const int c0 = blockIdx.x * CB;
    const int cams = min(CB, np - c0);
    const int t = threadIdx.x;
    const bool row = t < cams * DP;
    const int64_t i = (int64_t)c0 * DP + (row ? t : 0);
    const double xi = x[i], ri = r[i], p0 = P[i], q0 = Q[i];
    double Lc[NL];
    {
        const double *Lp = Dchol + (int64_t)(c0 + (t < cams ? t : 0)) * NL;
#pragma unroll
        for (int e = 0; e < NL; ++e) Lc[e] = Lp[e];
    }
    const double scv = sc[t < SC_COUNT ? t : 0];
    double ul[kLowRank];
    if constexpr (LR) {
#pragma unroll
        for (int a = 0; a < kLowRank; ++a) ul[a] = lr.U[i * kLowRank + a];
    }
    if (g1.part) {
        // one-column block: Delta = Q^T P and gamma = P^T r from the camera reduction's
        // partials, added in the same order by every block; Delta^+ = 1 / Delta unless
        // Delta is zero (or not finite), the 1 x 1 case of the pseudo-inverse's rank rule.
        // Block 0 stores Delta^+, gamma, alpha, the rank and the history block entry.
        if (t < 64) {
            double d, gg;
            wave_pair_sums(g1.part, g1.nb, d, gg);
            if (t == 0) {
                const bool nz = fabs(d) > 2.220446049250313e-16 * fabs(d);
                const double dpv = nz ? 1.0 / d : 0.0;
                al[0] = dpv * gg;
                ga_sh[0] = gg;
                rank_sh = nz ? 1.0 : 0.0;
                if (blockIdx.x == 0) {
                    g1.Dp[0] = dpv;
                    gamma[0] = gg;
                    alpha[0] = al[0];
                    sc[SC_RANK] = rank_sh;
                    if (g1.blk.off) {
                        g1.blk.off[g1.blk.j] = g1.blk.first;
                        g1.blk.k[g1.blk.j] = 1;
                        g1.blk.dp[g1.blk.j] = g1.blk.dpo;
                    }
                }
            }
        }
    } else {
        for (int a = t; a < k; a += kNT) {
            al[a] = alpha[a];
            ga_sh[a] = gamma[a];
        }
        if (t == SC_RANK) rank_sh = scv;
    }
    __syncthreads();
    double rr = 0.0, rv = 0.0;
    if (row) {
        double dx = 0.0, dr = 0.0;
        dx += p0 * al[0];
        dr += q0 * al[0];
        // the other columns of a wide block, eight of each matrix in flight (columns past
        // k read column 0 and are dropped)
        for (int a0 = 1; a0 < k; a0 += 8) {
            double pv[8], qv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int a = a0 + u < k ? a0 + u : 0;
                pv[u] = P[(int64_t)a * n + i];
                qv[u] = Q[(int64_t)a * n + i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (a0 + u < k) {
                    dx += pv[u] * al[a0 + u];
                    dr += qv[u] * al[a0 + u];
                }
            }
        }
        x[i] = xi + dx;
        const double v = ri - dr;
        r[i] = v;
        sr[t] = v;
        rr = v * v;
        rv = v;
    }
    if constexpr (LR) {   // the block's U^T r: a butterfly per wavefront, the four in order below
#pragma unroll
        for (int a = 0; a < kLowRank; ++a) {
            const double s = wave_sum(ul[a] * rv);
            if ((t & 63) == 0) ush[(t >> 6) * kLowRank + a] = s;
        }
    }
    __syncthreads();
    double rho = 0.0;
    if (t < cams) {
        double rc[DP], zc[DP];
#pragma unroll
        for (int e = 0; e < DP; ++e) rc[e] = sr[t * DP + e];
        chol_solve_packed<DP>(Lc, rc, zc);
#pragma unroll
        for (int e = 0; e < DP; ++e) {
            z[(int64_t)(c0 + t) * DP + e] = zc[e];
            rho += rc[e] * zc[e];
        }
    }
    rr = block_sum(rr, sh);
    rho = block_sum(rho, sh);
    if (t == 0) {
        partials[2 * blockIdx.x] = rr;
        partials[2 * blockIdx.x + 1] = rho;
        if constexpr (LR) {
#pragma unroll
            for (int a = 0; a < kLowRank; ++a)
                lr.part[blockIdx.x * kLowRank + a] =
                    (ush[a] + ush[kLowRank + a]) + (ush[2 * kLowRank + a] + ush[3 * kLowRank + a]);
        }
        const uint32_t prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || t >= 64) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double srr, srho;
    wave_pair_sums(partials, gridDim.x, srr, srho);
    if constexpr (LR) {
        // w = U^T r over the blocks in order (lane l: blocks l, l + 64, ...), then
        // rho = r^T M^-1 r = r^T D^-1 r + |w|^2; lane a stores w_a for the z update
        double wa[kLowRank];
#pragma unroll
        for (int a = 0; a < kLowRank; ++a) wa[a] = 0.0;
        for (int b = t; b < (int)gridDim.x; b += 64) {
#pragma unroll
            for (int a = 0; a < kLowRank; ++a) wa[a] += lr.part[b * kLowRank + a];
        }
        double wmine = 0.0, ww = 0.0;
#pragma unroll
        for (int a = 0; a < kLowRank; ++a) {
            const double s = wave_sum(wa[a]);
            ww += s * s;
            if (t == a) wmine = s;
        }
        if (t < kLowRank) lr.w[t] = wmine;
        srho += ww;
    }
    // lane 0 forms and stores the scalars; every lane takes them by cross-lane broadcast
    // (never by reading what lane 0 just stored), the rest of sc from its early load
    McgScalars v{};
    if (t == 0) {
        double ga = 0.0;
        for (int a = 0; a < k; ++a) ga += ga_sh[a] * al[a];
        static_assert(SC_RR0 == 0, "lane 0 loaded |r_0|^2 early");
        v = mcg_scalars_form(srr, srho, ga, scv, N, tau, eps);
        mcg_scalars_put(v, sc);
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (host_sc) {   // all the scalars, for the host's read-back: lane i writes scalar i
        const double b_rr = __shfl(v.rr, 0, 64), b_rho = __shfl(v.rho, 0, 64), b_t = __shfl(v.t, 0, 64);
        const double b_sm = __shfl(v.skipm, 0, 64), b_kn = __shfl(v.kn, 0, 64), b_ss = __shfl(v.skips, 0, 64);
        double mine = t == SC_RANK ? rank_sh : scv;
        mine = t == SC_RR ? b_rr : t == SC_RHO ? b_rho : t == SC_T ? b_t : mine;
        mine = t == SC_SKIPM ? b_sm : t == SC_KN ? b_kn : t == SC_SKIPS ? b_ss : mine;
        if (t < SC_COUNT) host_sc[t] = mine;
        __threadfence_system();   // the values reach the host before the tag
        if (t == 0) host_sc[SC_COUNT] = tag;
    }
}

int mcg_xrz_blocks(int np, int dp) { return (np + kNT / dp - 1) / (kNT / dp); }

void launch_mcg_xrz(int np, int k, const double *P, const double *Q, double *alpha, double *x, double *r,
                    const double *Dchol, double *z, double *partials, uint32_t *ticket, double *gamma,
                    double *sc, double *host_sc, double tag, int N, double tau, double eps, hipStream_t s, int dp,
                    XrzGram g1, XrzLowrank lr) {
    const unsigned nb = (unsigned)mcg_xrz_blocks(np, dp);
    if (dp == 6)
        hipLaunchKernelGGL((k_mcg_xrz<6, false>), dim3(nb), dim3(kNT), 0, s, np, k, P, Q, alpha, x, r, Dchol, z,
                           partials, ticket, gamma, sc, host_sc, tag, N, tau, eps, g1, lr);
    else if (lr.U)
        hipLaunchKernelGGL((k_mcg_xrz<9, true>), dim3(nb), dim3(kNT), 0, s, np, k, P, Q, alpha, x, r, Dchol, z,
                           partials, ticket, gamma, sc, host_sc, tag, N, tau, eps, g1, lr);
    else
        hipLaunchKernelGGL((k_mcg_xrz<9, false>), dim3(nb), dim3(kNT), 0, s, np, k, P, Q, alpha, x, r, Dchol, z,
                           partials, ticket, gamma, sc, host_sc, tag, N, tau, eps, g1, lr);
}

// z += U w: the learned low-rank part of Z = M^-1 r after k_mcg_xrz formed D^-1 r and w = U^T r
__global__ __launch_bounds__(kNT) void k_lr_zadd(int64_t n, const double *__restrict__ U,
                                                 const double *__restrict__ w, double *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < kLowRank; ++a) s += U[i * kLowRank + a] * w[a];
    z[i] = z[i] + s;
}

void launch_lr_zadd(int64_t n, const double *U, const double *w, double *z, hipStream_t s) {
    hipLaunchKernelGGL(k_lr_zadd, dim3((unsigned)((n + kNT - 1) / kNT)), dim3(kNT), 0, s, n, U, w, z);
}

// Phi[col][p] = Q_hist[:, col]^T z restricted to segment p: with N > 1 subsets the
// segments are the subsets (gs rows each -- the rows of gs poses --, the last takes the
// rest), which is Phi of a multidirectional Z; a one-column Z = D^-1 r needs their sum,
// which k_beta forms.  So Phi does not depend on the tau-test and can run before its
// outcome is known.  With N = 1 the rows are split into kPhiSeg equal segments (for
// parallelism only).  One wavefront per (group of kPhiCols columns, segment), segments
// of a group on consecutive wavefronts; each lane keeps four rows of every column of the
// group in flight and loads z once for them.
constexpr int kPhiCols = 4;

template <int NC, typename HT>
__device__ inline void phi_group(int64_t n, int64_t lo, int64_t hi, const HT *__restrict__ q,
                                 const double *__restrict__ z, double *acc) {
    const int lane = threadIdx.x & 63;
    double a[NC][4];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int u = 0; u < 4; ++u) a[c][u] = 0.0;
    int64_t i = lo + lane;
    for (; i + 192 < hi; i += 256) {
        double zv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) zv[u] = z[i + 64 * u];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int u = 0; u < 4; ++u) a[c][u] += (double)q[(int64_t)c * n + i + 64 * u] * zv[u];
    }
    for (; i < hi; i += 64) {
        const double zv = z[i];
#pragma unroll
        for (int c = 0; c < NC; ++c) a[c][0] += (double)q[(int64_t)c * n + i] * zv;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = wave_sum((a[c][0] + a[c][1]) + (a[c][2] + a[c][3]));
}

template <typename HT>
__global__ __launch_bounds__(kNT) void k_phi(int64_t n, int h, int seg, const HT *__restrict__ Qh,
                                             const double *__restrict__ z, int N, int gs,
                                             double *__restrict__ Phi) {
    const int64_t w = (int64_t)blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t groups = (h + kPhiCols - 1) / kPhiCols;
    if (w >= groups * seg) return;
    const int64_t g = w / seg;
    const int p = (int)(w - g * seg);
    int64_t lo, hi;
    if (N > 1) {
        lo = (int64_t)p * gs;
        hi = (p == N - 1) ? n : (int64_t)(p + 1) * gs;
    } else {
        lo = n * p / seg;
        hi = n * (p + 1) / seg;
    }
    const int64_t c0 = g * kPhiCols;
    const int nc = (int)min<int64_t>(kPhiCols, h - c0);
    const HT *q = Qh + c0 * n;
    double acc[kPhiCols];
    switch (nc) {
    case 4: phi_group<4, HT>(n, lo, hi, q, z, acc); break;
    case 3: phi_group<3, HT>(n, lo, hi, q, z, acc); break;
    case 2: phi_group<2, HT>(n, lo, hi, q, z, acc); break;
    default: phi_group<1, HT>(n, lo, hi, q, z, acc); break;
    }
    if (lane == 0)
        for (int c = 0; c < nc; ++c) Phi[(c0 + c) * seg + p] = acc[c];
}

int phi_segments(int N) { return N > 1 ? N : kPhiSeg; }

template <typename HT>
void launch_phi(int64_t n, int h, const HT *Qh, const double *z, int N, int gs, double *Phi, hipStream_t s) {
    if (h <= 0) return;
    const int seg = phi_segments(N);
    const int64_t waves = (int64_t)(h + kPhiCols - 1) / kPhiCols * seg;
    const int per = kNT / 64;
    hipLaunchKernelGGL(k_phi<HT>, dim3((unsigned)((waves + per - 1) / per)), dim3(kNT), 0, s, n, h, seg, Qh, z, N, gs,
                       Phi);
}
template void launch_phi<double>(int64_t, int, const double *, const double *, int, int, double *, hipStream_t);
template void launch_phi<float>(int64_t, int, const float *, const double *, int, int, double *, hipStream_t);

// Width of the block being built, as the device decided it (sc[SC_KN]: 0 once converged,
// N for a multidirectional block, else 1); 0 as well when it exceeds kn_max, the widest
// block the host has room for (the host then stops with a workspace error).
__device__ inline int next_kn(const double *__restrict__ sc, int kn_max) {
    const int kn = (int)sc[SC_KN];
    return kn > kn_max ? 0 : kn;
}

// beta rows of history block j: beta[off_j + a][p] = sum_b Delta_j^+[a][b] Phi[off_j + b][p]
// for the next block's width kn (next_kn); rows of hist_ldb(kn) values.  One work-group
// per history block.  A block wider than one column first stages Delta_j^+ (transposed)
// and its Phi rows in LDS with coalesced loads; each output is then one running sum over
// b in ascending order, taken from LDS (a multidirectional block's outputs in 4 x 4 tiles
// per thread).  For a one-column Z, Phi of a history column is the sum of its segments
// and beta_j = Delta_j^+ Phi, each output by four threads and two shuffles.
__global__ __launch_bounds__(kNT) void k_beta(const int32_t *__restrict__ blk_off, const int32_t *__restrict__ blk_k,
                                              const int64_t *__restrict__ blk_dp, const double *__restrict__ Dp,
                                              const double *__restrict__ Phi, const double *__restrict__ sc,
                                              int kn_max, int seg, double *__restrict__ beta) {
    __shared__ double sDt[kMaxK * kMaxK];   // sDt[b * kj + a] = Delta_j^+[a][b]
    __shared__ double sF[kMaxK * kMaxK];    // sF[b * kn + p] = Phi[off + b][p] (kn > 1; kn == 1: all seg values)
    const int kn = next_kn(sc, kn_max);
    if (kn == 0) return;
    const int j = blockIdx.x;
    const int off = blk_off[j], kj = blk_k[j];
    const double *D = Dp + blk_dp[j];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if (kj == 1) {   // a one-column history block: Delta^+ is a scalar
        const double d = D[0];
        if (kn == 1) {   // one-column Z: Phi of the column is the sum of its seg <= 64 segments
            if (tid < 64) {
                const double f = wave_sum(lane < seg ? Phi[(int64_t)off * seg + lane] : 0.0);
                if (lane == 0) beta[off] = d * f;
            }
            return;
        }
        const int ldb = hist_ldb(kn);
        for (int p = tid; p < ldb; p += kNT) beta[(int64_t)off * ldb + p] = p < kn ? d * Phi[(int64_t)off * seg + p] : 0.0;
        return;
    }
    // staging: every load of a thread is issued before its first LDS store (at most
    // kMaxK * kMaxK / kNT = 16 of each)
    constexpr int SU = kMaxK * kMaxK / kNT;
    {
        double v[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int w = tid + u * kNT;
            v[u] = w < kj * kj ? D[w] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int w = tid + u * kNT;
            if (w < kj * kj) {
                const int a = w / kj, b = w - a * kj;
                sDt[b * kj + a] = v[u];
            }
        }
    }
    const int fcols = kn == 1 ? seg : kn;   // Phi values staged per history column
    {
        double v[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int w = tid + u * kNT;
            const int b = w / fcols, p = w - b * fcols;
            v[u] = w < kj * fcols ? Phi[(int64_t)(off + b) * seg + p] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int w = tid + u * kNT;
            if (w < kj * fcols) sF[w] = v[u];
        }
    }
    __syncthreads();
    if (kn == 1) {   // one-column Z: Phi of column off + b is the sum of its segments
        // four threads per column (or per output row): strided partial sums, then two
        // shuffles within the four, a fixed order
        __shared__ double f1[kMaxK];
        const int r4 = tid >> 2, q4 = tid & 3;
        double f = 0.0;
        if (r4 < kj)
            for (int g = q4; g < seg; g += 4) f += sF[r4 * seg + g];
        f += __shfl_xor(f, 1, 64);
        f += __shfl_xor(f, 2, 64);
        if (q4 == 0 && r4 < kj) f1[r4] = f;
        __syncthreads();
        double s = 0.0;
        if (r4 < kj)
            for (int b = q4; b < kj; b += 4) s += sDt[b * kj + r4] * f1[b];
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        if (q4 == 0 && r4 < kj) beta[off + r4] = s;
        return;
    }
    // multidirectional: segment p is subset p; rows are padded with zeros to hist_ldb(kn)
    const int ldb = hist_ldb(kn);
    const int ta = (kj + 3) / 4, tp = ldb / 4;
    for (int t = tid; t < ta * tp; t += kNT) {
        const int a0 = (t / tp) * 4, p0 = (t - (t / tp) * tp) * 4;
        double acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
        for (int b = 0; b < kj; ++b) {
            double dv[4], fv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) dv[u] = a0 + u < kj ? sDt[b * kj + a0 + u] : 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) fv[v] = p0 + v < kn ? sF[b * kn + p0 + v] : 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += dv[u] * fv[v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (a0 + u >= kj) break;
#pragma unroll
            for (int v = 0; v < 4; ++v) beta[(int64_t)(off + a0 + u) * ldb + p0 + v] = acc[u][v];
        }
    }
}

void launch_beta(int nb, const int32_t *blk_off, const int32_t *blk_k, const int64_t *blk_dp, const double *Dp,
                 const double *Phi, const double *sc, int kn_max, int N, double *beta, hipStream_t s) {
    hipLaunchKernelGGL(k_beta, dim3(nb), dim3(kNT), 0, s, blk_off, blk_k, blk_dp, Dp, Phi, sc, kn_max,
                       phi_segments(N), beta);
}

// History products of the reorthogonalisation, Out[:, p] = Base[:, p] - sum_col H[:, col] beta[col][p]
// (Alg. 2: P_{i+1} = Z - sum_j P_j beta_{i,j}; eq. (19): Q_{i+1} = S Z - sum_j Q_j beta_{i,j}).
// The width kn of the new block is read on the device (next_kn), so the launches go
// ahead of the host's read-back of the tau-test.  Pass 1: one wavefront per (64-row tile,
// column slice, matrix, block of outputs) accumulates its slice; beta is wave-uniform
// (scalar loads) and its rows, hist_ldb(kn) long, are padded with zeros, so the inner
// loops carry no per-output test; blocks wider than 16 columns take the matrix-core path
// (hist_slice_mfma).  Pass 2 adds the slices in slice order and subtracts
// from the base, so the result is independent of scheduling.
template <int KB, typename HT>
__device__ inline void hist_slice(int64_t n, int64_t row, int c0, int c1, int kn, int p0,
                                  const HT *__restrict__ H, const double *__restrict__ beta,
                                  double *__restrict__ out) {
    const int ldb = hist_ldb(kn);
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    const HT *hp = H + row;
    int c = c0;
    // CU columns per step: CU loads of the history in flight per lane (fewer for wide
    // output blocks, whose beta values fill the scalar registers)
    constexpr int CU = KB > 16 ? 4 : 8;
    for (; c + CU <= c1; c += CU) {
        double hv[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) hv[u] = (double)hp[(int64_t)(c + u) * n];
        const double *b0 = beta + (int64_t)c * ldb + p0;
#pragma unroll
        for (int u = 0; u < CU; ++u) {
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += hv[u] * b0[u * ldb + j];
        }
    }
    for (; c < c1; ++c) {
        const double hv = (double)hp[(int64_t)c * n];
        const double *b0 = beta + (int64_t)c * ldb + p0;
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] += hv * b0[j];
    }
#pragma unroll
    for (int j = 0; j < KB; ++j)
        if (p0 + j < kn) out[(int64_t)(p0 + j) * n + row] = acc[j];
}

// The same sums for a multidirectional block on the matrix cores: one wavefront covers 64
// rows x 32 outputs (8 tiles of 16 x 16) of its column slice; for every 4 history columns
// it issues one v_mfma_f64_16x16x4f64 per tile with A[i][kk] = H[row0 + 16 m + i][c + kk]
// and B[kk][j] = beta[c + kk][p0 + 16 q + j] (lane layouts as in the Gram kernel),
// 4 kHistMG columns' loads in flight.  Rows past n and columns past c1 load zeros.
constexpr int kHistMG = 2;   // groups of 4 history columns per loop trip
template <typename HT>
__device__ inline void hist_slice_mfma(int64_t n, int64_t row0, int c0, int c1, int kn, int p0,
                                       const HT *__restrict__ H, const double *__restrict__ beta,
                                       double *__restrict__ out) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int ldb = hist_ldb(kn);
    dbl4_t acc[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[m][q] = dbl4_t{0.0, 0.0, 0.0, 0.0};
    for (int c = c0; c < c1; c += 4 * kHistMG) {
        double hv[kHistMG][4], bv[kHistMG][2];
#pragma unroll
        for (int g = 0; g < kHistMG; ++g) {
            const int col = c + 4 * g + lk;
            const bool okc = col < c1;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int64_t row = row0 + 16 * m + li;
                hv[g][m] = (okc && row < n) ? (double)H[(int64_t)col * n + row] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int p = p0 + 16 * q + li;
                bv[g][q] = (okc && p < ldb) ? beta[(int64_t)col * ldb + p] : 0.0;
            }
        }
#pragma unroll
        for (int g = 0; g < kHistMG; ++g)
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(hv[g][m], bv[g][q], acc[m][q], 0, 0, 0);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = row0 + 16 * m + lk + 4 * e;
                const int p = p0 + 16 * q + li;
                if (row < n && p < kn) out[(int64_t)p * n + row] = acc[m][q][e];
            }
}

// Column slices of the history products for the block width the device chose: a
// one-column block (P only, one output) splits the history into many more slices than a
// multidirectional one, whose kn partial outputs per slice fill the scratch much sooner.
struct HistSlices {
    int one, one_cols;     // kn == 1
    int multi, multi_cols; // kn > 1
};

// grid (row tiles, max slices, 2 * zb): z < zb the P history, z >= zb the Q history (used
// by multidirectional blocks only); zb output blocks of KBW columns.  KBW = 16: blocks of
// any width up to 16; KBW = 32: one-column blocks only (wider ones are left to
// k_hist_wide, launched beside it, so that this kernel keeps few registers and many
// wavefronts in flight for the one-column blocks, the most frequent).
template <int KBW, typename HT>
__global__ __launch_bounds__(64) void k_hist_partial(int64_t n, int h, HistSlices hs, int zb,
                                                     const HT *__restrict__ Ph, const HT *__restrict__ Qh,
                                                     const double *__restrict__ beta, const double *__restrict__ sc,
                                                     int kn_max, double *__restrict__ scratch) {
    const int kn = next_kn(sc, kn_max);
    const int64_t row = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int mat = (int)blockIdx.z / zb, p0 = ((int)blockIdx.z - mat * zb) * KBW;
    if (kn == 0 || row >= n || p0 >= kn || (mat == 1 && kn == 1) || (KBW == 32 && kn > 1)) return;
    const int nslices = kn == 1 ? hs.one : hs.multi;
    const int slice_cols = kn == 1 ? hs.one_cols : hs.multi_cols;
    const int ks = blockIdx.y;
    if (ks >= nslices) return;
    const int c0 = ks * slice_cols;
    const int c1 = min(h, c0 + slice_cols);
    double *out = scratch + ((int64_t)mat * nslices + ks) * kn * n;
    if (kn == 1) hist_slice<1, HT>(n, row, c0, c1, 1, 0, Ph, beta, out);
    else if (KBW == 16) hist_slice<16, HT>(n, row, c0, c1, kn, p0, mat ? Qh : Ph, beta, out);
}

// Multidirectional blocks wider than 16 columns: 32-output blocks of the same grid and
// outputs as k_hist_partial<32>, with vector FMAs (MFMA = false: hist_slice<32>, beta
// from scalar loads) or on the matrix cores (MFMA = true: hist_slice_mfma; every lane of
// a wavefront takes part, rows past n load zeros); one-column blocks return at once.
template <bool MFMA, typename HT>
__global__ __launch_bounds__(64) void k_hist_wide(int64_t n, int h, HistSlices hs, int zb,
                                                  const HT *__restrict__ Ph, const HT *__restrict__ Qh,
                                                  const double *__restrict__ beta, const double *__restrict__ sc,
                                                  int kn_max, double *__restrict__ scratch) {
    const int kn = next_kn(sc, kn_max);
    const int mat = (int)blockIdx.z / zb, p0 = ((int)blockIdx.z - mat * zb) * 32;
    if (kn <= 1 || p0 >= kn) return;
    const int ks = blockIdx.y;
    if (ks >= hs.multi) return;
    const int64_t row0 = (int64_t)blockIdx.x * 64;
    if (!MFMA && row0 + threadIdx.x >= n) return;
    const int c0 = ks * hs.multi_cols;
    const int c1 = min(h, c0 + hs.multi_cols);
    double *out = scratch + ((int64_t)mat * hs.multi + ks) * kn * n;
    if (MFMA) hist_slice_mfma<HT>(n, row0, c0, c1, kn, p0, mat ? Qh : Ph, beta, out);
    else hist_slice<32, HT>(n, row0 + threadIdx.x, c0, c1, kn, p0, mat ? Qh : Ph, beta, out);
}

// y = 0 (mat0 = 0): P_new from the P slices; mat0 = 1: Q_new from the Q slices
// (multidirectional blocks only, their base Y = S Z already in the Q columns); no
// slices: P_new = Z_p.  The slices are added in ascending order, eight loads in flight
// at a time (issued unconditionally: slices past the last read slice 0 and are dropped).
// With out32 the new column is also written rounded to FP32 (mixed precision's history copy).
__global__ void k_hist_final(int64_t n, HistSlices hs, const double *__restrict__ scratch,
                             const double *__restrict__ z, int gs, int N, const double *__restrict__ sc, int kn_max,
                             int mat, double *__restrict__ Pn, double *__restrict__ Qn, float *__restrict__ out32) {
    const int kn = next_kn(sc, kn_max);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (kn == 0 || i >= n * kn || (mat == 1 && kn == 1)) return;
    const int nslices = kn == 1 ? hs.one : hs.multi;
    const int p = (int)(i / n);
    const int64_t row = i - (int64_t)p * n;
    const double *sp = scratch + (int64_t)mat * nslices * kn * n + (int64_t)p * n + row;
    const int64_t sstride = (int64_t)kn * n;
    double s = 0.0;
    for (int k0 = 0; k0 < nslices; k0 += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = sp[(k0 + u < nslices ? k0 + u : 0) * sstride];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (k0 + u < nslices) s += v[u];
    }
    double *out = mat ? Qn : Pn;
    double base;
    if (mat) {
        base = out[i];
    } else {
        const int grp = kn > 1 ? min((int)(row / gs), N - 1) : 0;
        base = (kn == 1 || grp == p) ? z[row] : 0.0;
    }
    const double o = base - s;
    out[i] = o;
    if (out32) out32[i] = (float)o;
}

// column slices of the history products for a block of width kn: enough (row tile, slice)
// wavefronts to fill the device, at least 16 columns each, and the partials of a
// kn-wide block (both matrices) within the scratch (the caller guarantees room for one
// slice of the widest block)
int hist_slices(int64_t n, int h, int kn, int64_t scratch_doubles) {
    const int64_t tiles = (n + 63) / 64;
    int s = (int)std::max<int64_t>(1, (2048 + tiles - 1) / tiles);
    s = std::min(s, std::max(1, h / 16));
    s = std::min(s, 64);
    const int64_t per = 2 * (int64_t)kn * n;
    if (per > 0) s = (int)std::max<int64_t>(1, std::min<int64_t>(s, scratch_doubles / per));
    return std::max(1, s);
}

static HistSlices hist_slicing(int64_t n, int h, int kn_max, int64_t scratch_doubles) {
    HistSlices hs{0, 1, 0, 1};
    if (h <= 0) return hs;
    hs.one = hist_slices(n, h, 1, scratch_doubles);
    hs.one_cols = (h + hs.one - 1) / hs.one;
    hs.multi = hist_slices(n, h, std::max(kn_max, 1), scratch_doubles);
    hs.multi_cols = (h + hs.multi - 1) / hs.multi;
    return hs;
}

int64_t hist_scratch_min(int64_t n, int kn_max) { return 2 * (int64_t)kn_max * n; }

template <typename HT>
void launch_update_pq(int64_t n, int h, int N, int kn_max, const HT *Ph, const HT *Qh, const double *beta,
                      const double *z, int gs, const double *sc, double *Pn, double *scratch, int64_t scratch_doubles,
                      hipStream_t s, bool mfma, float *Pn32) {
    if (kn_max <= 0) return;
    const HistSlices hs = hist_slicing(n, h, kn_max, scratch_doubles);
    if (h > 0) {
        const unsigned tiles = (unsigned)((n + 63) / 64);
        const unsigned ys = (unsigned)std::max(hs.one, hs.multi);
        if (kn_max <= 16) {
            hipLaunchKernelGGL((k_hist_partial<16, HT>), dim3(tiles, ys, 2), dim3(64), 0, s, n, h, hs, 1, Ph, Qh, beta, sc,
                               kn_max, scratch);
        } else {
            const int zb = (kn_max + 31) / 32;
            hipLaunchKernelGGL((k_hist_partial<32, HT>), dim3(tiles, hs.one, 1), dim3(64), 0, s, n, h, hs, zb, Ph, Qh,
                               beta, sc, kn_max, scratch);
            if (mfma)
                hipLaunchKernelGGL((k_hist_wide<true, HT>), dim3(tiles, hs.multi, 2 * zb), dim3(64), 0, s, n, h, hs, zb,
                                   Ph, Qh, beta, sc, kn_max, scratch);
            else
                hipLaunchKernelGGL((k_hist_wide<false, HT>), dim3(tiles, hs.multi, 2 * zb), dim3(64), 0, s, n, h, hs, zb,
                                   Ph, Qh, beta, sc, kn_max, scratch);
        }
    }
    const int64_t tot = n * kn_max;
    hipLaunchKernelGGL(k_hist_final, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, hs, scratch, z, gs, N,
                       sc, kn_max, 0, Pn, nullptr, Pn32);
}

template void launch_update_pq<double>(int64_t, int, int, int, const double *, const double *, const double *,
                                       const double *, int, const double *, double *, double *, int64_t, hipStream_t,
                                       bool, float *);
template void launch_update_pq<float>(int64_t, int, int, int, const float *, const float *, const double *,
                                      const double *, int, const double *, double *, double *, int64_t, hipStream_t,
                                      bool, float *);

// FP32 copy of history columns [c0, c0 + k) of P and Q (mixed precision: the
// reorthogonalisation reads the copy, the block's own Gram and updates the FP64 columns)
__global__ __launch_bounds__(kNT) void k_hist_copy32(int64_t n, int64_t c0, int k, const double *__restrict__ Ph,
                                                     const double *__restrict__ Qh, float *__restrict__ P32,
                                                     float *__restrict__ Q32) {
    const int64_t tot = (int64_t)k * n, base = c0 * n;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < tot; i += (int64_t)gridDim.x * kNT) {
        P32[base + i] = (float)Ph[base + i];
        Q32[base + i] = (float)Qh[base + i];
    }
}

void launch_hist_copy32(int64_t n, int64_t c0, int k, const double *Ph, const double *Qh, float *P32, float *Q32,
                        hipStream_t s) {
    const int64_t tot = (int64_t)k * n;
    const unsigned g = (unsigned)std::min<int64_t>((tot + kNT - 1) / kNT, 2048);
    if (g > 0) hipLaunchKernelGGL(k_hist_copy32, dim3(g), dim3(kNT), 0, s, n, c0, k, Ph, Qh, P32, Q32);
}

void launch_update_q(int64_t n, int h, int N, const double *sc, double *Qn, const double *scratch,
                     int64_t scratch_doubles, hipStream_t s, float *Qn32) {
    const HistSlices hs = hist_slicing(n, h, N, scratch_doubles);
    const int64_t tot = n * N;
    hipLaunchKernelGGL(k_hist_final, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, hs, scratch, nullptr, 0,
                       N, sc, N, 1, nullptr, Qn, Qn32);
}

}  // namespace ba
