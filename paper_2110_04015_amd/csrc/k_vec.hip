// Camera-space vector kernels of the Krylov solvers: block-Jacobi
// preconditioner, deterministic reductions (fixed grid, fixed-order trees),
// the PCG recurrences of Algorithm 1, and the block recurrences of Algorithm 2
// (Gram matrices, pseudo-inverse, tau-test, full reorthogonalisation).
// All FP64.
#include "ba_internal.h"
#include "kernels.h"

namespace ba {

constexpr int kNT = 256;   // threads of the reduction blocks

__device__ __forceinline__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kNT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// z_c = D_c^-1 r_c with the packed lower Cholesky factor (row i holds L[i][0..i])
__device__ __forceinline__ void chol9_solve(const double *__restrict__ L, const double *r, double *z) {
    double x[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        double s = r[i];
#pragma unroll
        for (int p = 0; p < i; ++p) s -= L[i * (i + 1) / 2 + p] * x[p];
        x[i] = s / L[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int i = 8; i >= 0; --i) {
        double s = x[i];
#pragma unroll
        for (int p = i + 1; p < 9; ++p) s -= L[p * (p + 1) / 2 + i] * x[p];
        x[i] = s / L[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) z[i] = x[i];
}

// ---------------------------------------------------------------- preconditioner

__global__ void k_precond(int np, const double *__restrict__ Dchol, const double *__restrict__ r,
                          double *__restrict__ z) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= np) return;
    double rc[9], zc[9];
    for (int i = 0; i < 9; ++i) rc[i] = r[(int64_t)c * 9 + i];
    chol9_solve(Dchol + (int64_t)c * 45, rc, zc);
    for (int i = 0; i < 9; ++i) z[(int64_t)c * 9 + i] = zc[i];
}

void launch_precond(int np, const double *Dchol, const double *r, double *z, hipStream_t s) {
    hipLaunchKernelGGL(k_precond, dim3((np + 127) / 128), dim3(128), 0, s, np, Dchol, r, z);
}

// z = D^-1 r and per-block partial sums of sum_i a[i] * z[i]
__global__ __launch_bounds__(kNT) void k_precond_dot(int np, const double *__restrict__ Dchol,
                                                     const double *__restrict__ r, const double *__restrict__ a,
                                                     double *__restrict__ z, double *__restrict__ partials) {
    __shared__ double sh[kNT];
    double acc = 0.0;
    for (int c = blockIdx.x * kNT + threadIdx.x; c < np; c += gridDim.x * kNT) {
        double rc[9], zc[9];
        for (int i = 0; i < 9; ++i) rc[i] = r[(int64_t)c * 9 + i];
        chol9_solve(Dchol + (int64_t)c * 45, rc, zc);
        for (int i = 0; i < 9; ++i) {
            z[(int64_t)c * 9 + i] = zc[i];
            acc += a[(int64_t)c * 9 + i] * zc[i];
        }
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

void launch_pcg_precond_phi(int np, const double *Dchol, const double *r, const double *Q, double *z,
                            double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_precond_dot, dim3(kRedBlocks), dim3(kNT), 0, s, np, Dchol, r, Q, z, partials);
}

void launch_precond_rho(int np, const double *Dchol, const double *r, double *z, double *partials,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_precond_dot, dim3(kRedBlocks), dim3(kNT), 0, s, np, Dchol, r, r, z, partials);
}

// ---------------------------------------------------------------- reductions

__global__ __launch_bounds__(kNT) void k_dot2(int64_t n, const double *__restrict__ a0, const double *__restrict__ b0,
                                              const double *__restrict__ a1, const double *__restrict__ b1,
                                              double *__restrict__ partials) {
    __shared__ double sh[kNT];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
        s0 += a0[i] * b0[i];
        s1 += a1[i] * b1[i];
    }
    s0 = block_sum(s0, sh);
    s1 = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x * 2] = s0;
        partials[blockIdx.x * 2 + 1] = s1;
    }
}

void launch_dot2(int64_t n, const double *a0, const double *b0, const double *a1, const double *b1,
                 double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_dot2, dim3(kRedBlocks), dim3(kNT), 0, s, n, a0, b0, a1, b1, partials);
}

__global__ void k_finalize(const double *__restrict__ partials, int nd, double *__restrict__ out) {
    int d = threadIdx.x;
    if (d >= nd) return;
    double s = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) s += partials[b * nd + d];
    out[d] = s;
}

void launch_finalize(const double *partials, int nd, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, partials, nd, out);
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
__global__ void k_pcg_rr(const double *__restrict__ partials, double *__restrict__ sc) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) s += partials[b];
    sc[SC_RR] = s;
    if (sc[SC_RR0] < 0.0) sc[SC_RR0] = s;
}

void launch_pcg_rr(const double *partials_rr, double *sc, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_rr, dim3(1), dim3(64), 0, s, partials_rr, sc);
}

// Delta = Q^T P, gamma = P^T r from the partials; alpha = gamma / Delta;
// x += alpha P, r -= alpha Q; partial |r|^2
__global__ __launch_bounds__(kNT) void k_pcg_update_xr(int64_t n, const double *__restrict__ pdq,
                                                       double *__restrict__ sc, double *__restrict__ x,
                                                       double *__restrict__ r, const double *__restrict__ P,
                                                       const double *__restrict__ Q,
                                                       double *__restrict__ partials) {
    __shared__ double sh[kNT];
    __shared__ double s_alpha;
    if (threadIdx.x == 0) {
        double D = 0.0, g = 0.0;
        for (int b = 0; b < kRedBlocks; ++b) {
            D += pdq[b * 2];
            g += pdq[b * 2 + 1];
        }
        double al = D > 0.0 ? g / D : 0.0;
        s_alpha = al;
        if (blockIdx.x == 0) {
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

void launch_pcg_update_xr(int64_t n, const double *partials_dq, double *sc, double *x, double *r,
                          const double *P, const double *Q, double *partials_rr, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_update_xr, dim3(kRedBlocks), dim3(kNT), 0, s, n, partials_dq, sc, x, r, P, Q,
                       partials_rr);
}

// Phi = Q^T Z from the partials; beta = Phi / Delta; P = Z - beta P
__global__ __launch_bounds__(kNT) void k_pcg_update_p(int64_t n, const double *__restrict__ pphi,
                                                      double *__restrict__ sc, const double *__restrict__ z,
                                                      double *__restrict__ P) {
    __shared__ double s_beta;
    if (threadIdx.x == 0) {
        double phi = 0.0;
        for (int b = 0; b < kRedBlocks; ++b) phi += pphi[b];
        double be = phi / sc[SC_DELTA];
        s_beta = be;
        if (blockIdx.x == 0) {
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

constexpr int kGramRows = 16;
constexpr int kMaxK = 64;
constexpr int kGramOut = (kMaxK * kMaxK + kMaxK + kNT - 1) / kNT;   // outputs per thread

// partials[b][a * k + c] = sum_rows Q[:, a] . P[:, c] ; partials[b][k*k + a] = sum_rows P[:, a] . r
__global__ __launch_bounds__(kNT) void k_gram(int64_t n, int k, const double *__restrict__ P,
                                              const double *__restrict__ Q, const double *__restrict__ r,
                                              double *__restrict__ partials) {
    __shared__ double sP[kGramRows][kMaxK], sQ[kGramRows][kMaxK], sr[kGramRows];
    const int tot = k * k + k;
    double acc[kGramOut];
#pragma unroll
    for (int o = 0; o < kGramOut; ++o) acc[o] = 0.0;
    const int64_t ntiles = (n + kGramRows - 1) / kGramRows;
    for (int64_t it = blockIdx.x; it < ntiles; it += gridDim.x) {
        const int64_t r0 = it * kGramRows;
        for (int w = threadIdx.x; w < kGramRows * k; w += kNT) {
            int a = w / kGramRows, rr = w % kGramRows;
            int64_t row = r0 + rr;
            bool in = row < n;
            sP[rr][a] = in ? P[(int64_t)a * n + row] : 0.0;
            sQ[rr][a] = in ? Q[(int64_t)a * n + row] : 0.0;
        }
        if (threadIdx.x < kGramRows) {
            int64_t row = r0 + threadIdx.x;
            sr[threadIdx.x] = row < n ? r[row] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < kGramOut; ++o) {
            int idx = threadIdx.x + o * kNT;
            if (idx < k * k) {
                int a = idx / k, c = idx - a * k;
                double s = 0.0;
                for (int rr = 0; rr < kGramRows; ++rr) s += sQ[rr][a] * sP[rr][c];
                acc[o] += s;
            } else if (idx < tot) {
                int a = idx - k * k;
                double s = 0.0;
                for (int rr = 0; rr < kGramRows; ++rr) s += sP[rr][a] * sr[rr];
                acc[o] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < kGramOut; ++o) {
        int idx = threadIdx.x + o * kNT;
        if (idx < tot) partials[(int64_t)blockIdx.x * tot + idx] = acc[o];
    }
}

void launch_gram(int64_t n, int k, const double *P, const double *Q, const double *r, double *partials,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_gram, dim3(kRedBlocks), dim3(kNT), 0, s, n, k, P, Q, r, partials);
}

// Symmetric Jacobi eigendecomposition of the k x k matrix in LDS (k <= 64), with
// disjoint rotations applied in parallel (round-robin ordering).  A rotation of
// the pair (p, q) is skipped when |a_pq| <= (eps / 2) sqrt(|a_pp a_qq|); sweeps stop
// when a sweep rotates nothing.  On return A holds the eigenvalues on its
// diagonal and V the eigenvectors in its columns.
__device__ void jacobi_eig(int k, double *A, double *V, double *cs, double *sn, int *flag) {
    const int tid = threadIdx.x;
    const int kp = k + (k & 1);
    for (int w = tid; w < k * k; w += kNT) V[w] = (w / k == w % k) ? 1.0 : 0.0;
    __syncthreads();
    if (k < 2) return;
    const int half = kp / 2;
    for (int sweep = 0; sweep < 100; ++sweep) {
        if (tid == 0) *flag = 0;
        __syncthreads();
        for (int step = 0; step < kp - 1; ++step) {
            // pair t of this step: (step, kp-1) for t = 0, otherwise (step+t, step-t) mod (kp-1)
            if (tid < half) {
                int p, q;
                if (tid == 0) {
                    p = step;
                    q = kp - 1;
                } else {
                    p = (step + tid) % (kp - 1);
                    q = (step - tid + (kp - 1)) % (kp - 1);
                }
                if (p > q) {
                    int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, s = 0.0;
                if (q < k) {
                    double apq = A[p * k + q], app = A[p * k + p], aqq = A[q * k + q];
                    if (!(fabs(apq) <= 1e-300) && !(fabs(apq) <= 2.2e-16 * 0.5 * sqrt(fabs(app) * fabs(aqq)))) {
                        double theta = (aqq - app) / (2.0 * apq);
                        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                        *flag = 1;
                    }
                }
                cs[tid] = c;
                sn[tid] = s;
            }
            __syncthreads();
            // columns: A <- A J and V <- V J
            for (int w = tid; w < k * half; w += kNT) {
                int row = w / half, t = w - row * half;
                int p, q;
                if (t == 0) {
                    p = step;
                    q = kp - 1;
                } else {
                    p = (step + t) % (kp - 1);
                    q = (step - t + (kp - 1)) % (kp - 1);
                }
                if (p > q) {
                    int tt = p;
                    p = q;
                    q = tt;
                }
                if (q >= k) continue;
                double c = cs[t], s = sn[t];
                if (s == 0.0) continue;
                double arp = A[row * k + p], arq = A[row * k + q];
                A[row * k + p] = c * arp - s * arq;
                A[row * k + q] = s * arp + c * arq;
                double vrp = V[row * k + p], vrq = V[row * k + q];
                V[row * k + p] = c * vrp - s * vrq;
                V[row * k + q] = s * vrp + c * vrq;
            }
            __syncthreads();
            // rows: A <- J^T A, rotated off-diagonal entries set to zero
            for (int w = tid; w < k * half; w += kNT) {
                int col = w / half, t = w - col * half;
                int p, q;
                if (t == 0) {
                    p = step;
                    q = kp - 1;
                } else {
                    p = (step + t) % (kp - 1);
                    q = (step - t + (kp - 1)) % (kp - 1);
                }
                if (p > q) {
                    int tt = p;
                    p = q;
                    q = tt;
                }
                if (q >= k) continue;
                double c = cs[t], s = sn[t];
                if (s == 0.0) continue;
                double apc = A[p * k + col], aqc = A[q * k + col];
                A[p * k + col] = (col == q) ? 0.0 : c * apc - s * aqc;
                A[q * k + col] = (col == p) ? 0.0 : s * apc + c * aqc;
            }
            __syncthreads();
        }
        if (*flag == 0) break;
        __syncthreads();
    }
}

// A^+ = sum over |l_e| > k 2^-52 max|l| of v_e v_e^T / l_e ; returns rank via *rank_out
__device__ void pinv_from_eig(int k, const double *A, const double *V, double *Ap, int *rank_sh) {
    const int tid = threadIdx.x;
    double lmax = 0.0;
    for (int e = 0; e < k; ++e) lmax = fmax(lmax, fabs(A[e * k + e]));
    const double thr = (double)k * 2.220446049250313e-16 * lmax;
    if (tid == 0) {
        int rk = 0;
        for (int e = 0; e < k; ++e) rk += fabs(A[e * k + e]) > thr;
        *rank_sh = rk;
    }
    for (int w = tid; w < k * k; w += kNT) {
        int i = w / k, j = w - i * k;
        double s = 0.0;
        for (int e = 0; e < k; ++e) {
            double l = A[e * k + e];
            if (fabs(l) > thr) s += V[i * k + e] * (1.0 / l) * V[j * k + e];
        }
        Ap[w] = s;
    }
    __syncthreads();
}

// Delta (symmetrised) and gamma from the Gram partials; Delta^+; alpha = Delta^+ gamma
__global__ __launch_bounds__(kNT) void k_pinv_alpha(int k, const double *__restrict__ partials, int nblocks,
                                                    double *__restrict__ Dp, double *__restrict__ gamma,
                                                    double *__restrict__ alpha, double *__restrict__ sc) {
    __shared__ double A[kMaxK * kMaxK], V[kMaxK * kMaxK], G[kMaxK * kMaxK];
    __shared__ double gam[kMaxK], cs[kMaxK], sn[kMaxK];
    __shared__ int flag, rank;
    const int tid = threadIdx.x;
    const int tot = k * k + k;
    for (int idx = tid; idx < tot; idx += kNT) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * tot + idx];
        if (idx < k * k) G[idx] = s;
        else gam[idx - k * k] = s;
    }
    __syncthreads();
    for (int w = tid; w < k * k; w += kNT) {
        int i = w / k, j = w - i * k;
        A[w] = 0.5 * (G[i * k + j] + G[j * k + i]);
    }
    __syncthreads();
    jacobi_eig(k, A, V, cs, sn, &flag);
    pinv_from_eig(k, A, V, G, &rank);
    for (int w = tid; w < k * k; w += kNT) Dp[w] = G[w];
    for (int a = tid; a < k; a += kNT) {
        double s = 0.0;
        for (int b = 0; b < k; ++b) s += G[a * k + b] * gam[b];
        alpha[a] = s;
        gamma[a] = gam[a];
    }
    if (tid == 0) sc[SC_RANK] = (double)rank;
}

void launch_pinv_alpha(int k, const double *partials, int nblocks, double *Dp, double *gamma, double *alpha,
                       double *sc, hipStream_t s) {
    hipLaunchKernelGGL(k_pinv_alpha, dim3(1), dim3(kNT), 0, s, k, partials, nblocks, Dp, gamma, alpha, sc);
}

// Stand-alone symmetric pseudo-inverse (test entry point).
__global__ __launch_bounds__(kNT) void k_pinv_sym(int k, const double *__restrict__ Ain, double *__restrict__ Ap,
                                                  int32_t *__restrict__ rank_out) {
    __shared__ double A[kMaxK * kMaxK], V[kMaxK * kMaxK];
    __shared__ double cs[kMaxK], sn[kMaxK];
    __shared__ int flag, rank;
    for (int w = threadIdx.x; w < k * k; w += kNT) A[w] = Ain[w];
    __syncthreads();
    jacobi_eig(k, A, V, cs, sn, &flag);
    pinv_from_eig(k, A, V, Ap, &rank);
    if (threadIdx.x == 0 && rank_out) *rank_out = rank;
}

void launch_pinv_sym(int k, const double *A, double *Ap, int32_t *rank, hipStream_t s) {
    hipLaunchKernelGGL(k_pinv_sym, dim3(1), dim3(kNT), 0, s, k, A, Ap, rank);
}

// x += P alpha ; r -= Q alpha (n x k blocks, column-major) ; partial |r|^2
__global__ __launch_bounds__(kNT) void k_update_xr_blk(int64_t n, int k, const double *__restrict__ P,
                                                       const double *__restrict__ Q,
                                                       const double *__restrict__ alpha, double *__restrict__ x,
                                                       double *__restrict__ r, double *__restrict__ partials) {
    __shared__ double sh[kNT];
    __shared__ double al[kMaxK];
    for (int a = threadIdx.x; a < k; a += kNT) al[a] = alpha[a];
    __syncthreads();
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
        double dx = 0.0, dr = 0.0;
        for (int a = 0; a < k; ++a) {
            dx += P[(int64_t)a * n + i] * al[a];
            dr += Q[(int64_t)a * n + i] * al[a];
        }
        x[i] += dx;
        double v = r[i] - dr;
        r[i] = v;
        acc += v * v;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

void launch_update_xr_blk(int64_t n, int k, const double *P, const double *Q, const double *alpha, double *x,
                          double *r, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_update_xr_blk, dim3(kRedBlocks), dim3(kNT), 0, s, n, k, P, Q, alpha, x, r, partials);
}

// rho = r^T D^-1 r from the partials; t = gamma^T alpha / rho (the tau-test of Alg. 2)
__global__ void k_tau(int k, const double *__restrict__ prho, const double *__restrict__ gamma,
                      const double *__restrict__ alpha, double *__restrict__ sc) {
    if (threadIdx.x != 0) return;
    double rho = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) rho += prho[b];
    double ga = 0.0;
    for (int a = 0; a < k; ++a) ga += gamma[a] * alpha[a];
    sc[SC_RHO] = rho;
    sc[SC_T] = rho > 0.0 ? ga / rho : INFINITY;
}

void launch_tau(int k, const double *partials_rho, const double *gamma, const double *alpha, double *sc,
                hipStream_t s) {
    hipLaunchKernelGGL(k_tau, dim3(1), dim3(64), 0, s, k, partials_rho, gamma, alpha, sc);
}

// Phi[col][p] = Q_hist[:, col]^T Z[:, p]: for a multidirectional Z only the rows of
// subset p contribute (gs poses per subset, the last subset takes the rest).
__global__ __launch_bounds__(kNT) void k_phi(int64_t n, const double *__restrict__ Qh,
                                             const double *__restrict__ z, int multi, int N, int gs,
                                             double *__restrict__ Phi) {
    __shared__ double sh[kNT];
    const int col = blockIdx.x;
    const int p = blockIdx.y;
    int64_t lo = 0, hi = n;
    if (multi) {
        lo = (int64_t)p * gs * 9;
        hi = (p == N - 1) ? n : (int64_t)(p + 1) * gs * 9;
    }
    const double *q = Qh + (int64_t)col * n;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kNT) acc += q[i] * z[i];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) Phi[(int64_t)col * (multi ? N : 1) + p] = acc;
}

void launch_phi(int64_t n, int h, const double *Qh, const double *z, int multi, int N, int gs, double *Phi,
                hipStream_t s) {
    hipLaunchKernelGGL(k_phi, dim3(h, multi ? N : 1), dim3(kNT), 0, s, n, Qh, z, multi, N, gs, Phi);
}

// beta rows of history block j: beta[off_j + a][p] = sum_b Delta_j^+[a][b] Phi[off_j + b][p]
__global__ __launch_bounds__(kNT) void k_beta(const int32_t *__restrict__ blk_off, const int32_t *__restrict__ blk_k,
                                              const int64_t *__restrict__ blk_dp, const double *__restrict__ Dp,
                                              const double *__restrict__ Phi, int kn, double *__restrict__ beta) {
    const int j = blockIdx.x;
    const int off = blk_off[j], kj = blk_k[j];
    const double *D = Dp + blk_dp[j];
    for (int w = threadIdx.x; w < kj * kn; w += kNT) {
        int a = w / kn, p = w - a * kn;
        double s = 0.0;
        for (int b = 0; b < kj; ++b) s += D[a * kj + b] * Phi[(int64_t)(off + b) * kn + p];
        beta[(int64_t)(off + a) * kn + p] = s;
    }
}

void launch_beta(int nb, const int32_t *blk_off, const int32_t *blk_k, const int64_t *blk_dp, const double *Dp,
                 const double *Phi, int kn, double *beta, hipStream_t s) {
    hipLaunchKernelGGL(k_beta, dim3(nb), dim3(kNT), 0, s, blk_off, blk_k, blk_dp, Dp, Phi, kn, beta);
}

// Out[:, p] = Base[:, p] - sum_col H[:, col] beta[col][p] for p in [p0, p0 + 16).
// Base is Z (z restricted to subset p, or z itself for one column) when Y is null,
// otherwise the block Y (S Z, eq. (19)).
constexpr int kUpdCols = 16;
__global__ __launch_bounds__(kNT) void k_update_hist(int64_t n, int h, int kn, const double *__restrict__ H,
                                                     const double *__restrict__ beta,
                                                     const double *__restrict__ z, int multi, int gs, int N,
                                                     const double *__restrict__ Y, double *__restrict__ Out) {
    __shared__ double sb[64][kUpdCols];
    const int64_t row = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const int p0 = blockIdx.y * kUpdCols;
    const int pc = min(kUpdCols, kn - p0);
    double acc[kUpdCols];
#pragma unroll
    for (int j = 0; j < kUpdCols; ++j) acc[j] = 0.0;
    for (int c0 = 0; c0 < h; c0 += 64) {
        const int cc = min(64, h - c0);
        __syncthreads();
        for (int w = threadIdx.x; w < 64 * kUpdCols; w += kNT) {
            int c = w / kUpdCols, j = w - c * kUpdCols;
            sb[c][j] = (c < cc && j < pc) ? beta[(int64_t)(c0 + c) * kn + p0 + j] : 0.0;
        }
        __syncthreads();
        if (row < n) {
            for (int c = 0; c < cc; ++c) {
                const double hv = H[(int64_t)(c0 + c) * n + row];
#pragma unroll
                for (int j = 0; j < kUpdCols; ++j) acc[j] += hv * sb[c][j];
            }
        }
    }
    if (row >= n) return;
    int cam_grp = multi ? min((int)(row / 9) / gs, N - 1) : 0;
    for (int j = 0; j < pc; ++j) {
        const int p = p0 + j;
        double base;
        if (Y) base = Y[(int64_t)p * n + row];
        else base = (!multi || cam_grp == p) ? z[row] : 0.0;
        Out[(int64_t)p * n + row] = base - acc[j];
    }
}

void launch_update_pq(int64_t n, int h, int kn, const double *Ph, const double *Qh, const double *beta,
                      const double *z, int multi, int gs, int N, const double *Y, double *Pn, double *Qn,
                      hipStream_t s) {
    dim3 grid((unsigned)((n + kNT - 1) / kNT), (unsigned)((kn + kUpdCols - 1) / kUpdCols));
    hipLaunchKernelGGL(k_update_hist, grid, dim3(kNT), 0, s, n, h, kn, Ph, beta, z, multi, gs, N,
                       (const double *)nullptr, Pn);
    if (Y && Qn) hipLaunchKernelGGL(k_update_hist, grid, dim3(kNT), 0, s, n, h, kn, Qh, beta, z, multi, gs, N, Y, Qn);
}

}  // namespace ba
