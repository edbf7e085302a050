// Device linear algebra shared by the FP64 solver kernels: fixed-order block
// reductions, the 9x9 block-Jacobi solve, and the LDS pseudo-inverse of the k x k
// Gram matrices of Algorithm 2 (a Gauss-Jordan inverse when a norm bound proves that no
// eigenvalue lies below the pseudo-inverse's threshold, else a Jacobi eigendecomposition).
#pragma once
#include <hip/hip_runtime.h>

namespace ba {

constexpr int kMaxK = 64;   // widest direction block (Delta_i is at most 64 x 64)

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

// Sum over the lanes of a wavefront by a fixed butterfly.  Partners add the same two
// values (in swapped order, which is exact), so every lane ends with the same sum,
// independent of scheduling.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of nb block partials a[b * stride] by the calling wavefront (all 64 lanes must
// call): lane l adds entries l, l + 64, ... into four running sums (entry l + 64 i goes
// to sum i mod 4, so that four loads per lane are in flight), then the butterfly.  The
// order is fixed by nb alone.
__device__ __forceinline__ double wave_partials(const double *__restrict__ a, int64_t stride, int nb) {
    const int lane = threadIdx.x & 63;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int b = lane;
    for (; b + 192 < nb; b += 256) {
        s0 += a[(int64_t)b * stride];
        s1 += a[(int64_t)(b + 64) * stride];
        s2 += a[(int64_t)(b + 128) * stride];
        s3 += a[(int64_t)(b + 192) * stride];
    }
    if (b < nb) s0 += a[(int64_t)b * stride];
    if (b + 64 < nb) s1 += a[(int64_t)(b + 64) * stride];
    if (b + 128 < nb) s2 += a[(int64_t)(b + 128) * stride];
    return wave_sum((s0 + s1) + (s2 + s3));
}

// z_c = D_c^-1 r_c with the packed lower Cholesky factor of a DP x DP block (row i
// holds L[i][0..i]; DP (DP + 1) / 2 values)
template <int DP>
__device__ __forceinline__ void chol_solve_packed(const double *__restrict__ L, const double *r, double *z) {
    double x[DP];
#pragma unroll
    for (int i = 0; i < DP; ++i) {
        double s = r[i];
#pragma unroll
        for (int p = 0; p < i; ++p) s -= L[i * (i + 1) / 2 + p] * x[p];
        x[i] = s / L[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int i = DP - 1; i >= 0; --i) {
        double s = x[i];
#pragma unroll
        for (int p = i + 1; p < DP; ++p) s -= L[p * (p + 1) / 2 + i] * x[p];
        x[i] = s / L[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int i = 0; i < DP; ++i) z[i] = x[i];
}

__device__ __forceinline__ void chol9_solve(const double *__restrict__ L, const double *r, double *z) {
    chol_solve_packed<9>(L, r, z);
}

// Symmetric Jacobi eigendecomposition of the k x k matrix in LDS (k <= 64), with
// disjoint rotations applied in parallel (round-robin ordering).  A rotation of
// the pair (p, q) is skipped when |a_pq| <= (eps / 2) sqrt(|a_pp a_qq|); sweeps stop
// when a sweep rotates nothing.  On return A holds the eigenvalues on its
// diagonal and V the eigenvectors in its columns.
__device__ __forceinline__ void jacobi_eig(int k, double *A, double *V, double *cs, double *sn, int *flag) {
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

// Cross-lane move of a double by a DPP control (lanes whose source lies outside the
// control's reach, or outside row_mask, read 0).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Segments of a wavefront's lanes by a key that is equal on runs of consecutive lanes
// (each lane's segment is the run holding its key; a key must not recur after its run
// ends).  end is the segment's last lane; up<d> tells whether lane - d still lies in the
// lane's segment, for the steps of the scan below.
struct Segs {
    int end;
    bool up1, up2, up4, up8, row15, row31;
};

__device__ __forceinline__ Segs key_segments(int key, int lane) {
    const int prev = __shfl_up(key, 1, 64);
    const uint64_t heads = __ballot(lane == 0 || prev != key);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    const int start = 63 - __clzll(heads & upto);
    const uint64_t above = heads & ~upto;
    Segs g;
    g.end = above ? __ffsll((unsigned long long)above) - 2 : 63;
    g.up1 = lane - 1 >= start;
    g.up2 = lane - 2 >= start;
    g.up4 = lane - 4 >= start;
    g.up8 = lane - 8 >= start;
    g.row15 = (lane & 16) && start <= (lane & ~15) - 1;   // rows 1, 3 take lane 15 / 47 of the row before
    g.row31 = lane >= 32 && start <= 31;                  // rows 2, 3 take lane 31
    return g;
}

// Segmented inclusive scan of x: shifts by 1, 2, 4, 8 inside rows of 16 lanes, then the
// row sums carried across rows by the row broadcasts of lanes 15 and 31, each step added
// only where the source lane lies in the same segment.  The segment's last lane holds
// the segment total.  Fixed order: deterministic.
__device__ __forceinline__ double segment_scan(double x, const Segs &g) {
    double t;
    t = dpp_move<0x111>(x);   // row_shr:1
    if (g.up1) x += t;
    t = dpp_move<0x112>(x);   // row_shr:2
    if (g.up2) x += t;
    t = dpp_move<0x114>(x);   // row_shr:4
    if (g.up4) x += t;
    t = dpp_move<0x118>(x);   // row_shr:8
    if (g.up8) x += t;
    t = dpp_move<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
    if (g.row15) x += t;
    t = dpp_move<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
    if (g.row31) x += t;
    return x;
}

// Sum of x over the lane's segment, returned in every lane of the segment.
__device__ __forceinline__ double segment_sum(double x, const Segs &g) {
    return __shfl(segment_scan(x, g), g.end, 64);
}

// Sum over the block's threads: wavefront butterflies, then the wavefronts in order
// (one barrier); every thread gets the sum.  sh holds kNT / 64 doubles.
__device__ __forceinline__ double block_sum_waves(double v, double *sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kNT / 64; ++w) s += sh[w];
    __syncthreads();
    return s;
}

// Value of v in lane l of the wavefront (l wave-uniform).
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Gauss-Jordan inversion of the k x k matrix A (k <= KP, LDS, row-major) by one
// wavefront, held in registers: lane c keeps column c of A padded to KP x KP with the
// identity.  Step j, pivot p = a_jj, replaces a_jj by 1 / p, the rest of row j by
// a_jc / p, the rest of column j by -a_ij / p and every other element by
// a_ic - a_ij (a_jc / p).  Column j is broadcast from lane j (readlane) and row j is kept
// in register 0 of every lane: each step moves register i to i - 1 and the new pivot row
// to register KP - 1, so after the k steps register r holds row (r + k) mod KP.  The
// result goes to G (row-major k x k); *bad is set when a pivot is not positive.
template <int KP>
__device__ __forceinline__ void gj_wave(int k, const double *A, double *G, int *bad) {
    const int c = threadIdx.x & 63;
    double col[KP];
#pragma unroll
    for (int i = 0; i < KP; ++i) col[i] = (i < k && c < k) ? A[i * k + c] : (i == c ? 1.0 : 0.0);
    bool nonpos = false;
    for (int j = 0; j < k; ++j) {
        const double p = readlane_f64(col[0], j);
        nonpos |= !(p > 0.0);
        const double ip = 1.0 / (p > 0.0 ? p : 1.0);
        const bool piv = c == j;
        const double t = (piv ? 1.0 : col[0]) * ip;
#pragma unroll
        for (int i = 1; i < KP; ++i) {
            const double aij = readlane_f64(col[i], j);
            col[i - 1] = (piv ? 0.0 : col[i]) - aij * t;
        }
        col[KP - 1] = t;
    }
    if (c < k) {
#pragma unroll
        for (int r = 0; r < KP; ++r) {
            int row = r + k;
            row -= row >= KP ? KP : 0;
            if (row < k) G[row * k + c] = col[r];
        }
    }
    if (c == 0) *bad = nonpos;
}

// Inverse of the symmetric k x k matrix A (k <= 64, LDS) into G: Gauss-Jordan elimination
// on the diagonal pivots by the first wavefront (gj_wave), then the result is
// symmetrised by the whole block.  Returns (the same in every thread) whether every
// pivot was positive (A positive definite) and |A|_F |A^-1|_F < 1e-4 / (k eps): then
// every eigenvalue lies above the drop threshold k eps max|l| (l_min >= 1 / |A^-1|_F,
// l_max <= |A|_F), so A^+ = A^-1.
__device__ __forceinline__ bool inv_gj(int k, const double *A, double *G, double *sh) {
    constexpr int U = kMaxK * kMaxK / kNT;   // elements per thread at most
    __shared__ int nonpos;
    const int tid = threadIdx.x;
    const int kk = k * k;
    if (tid < 64) {
        if (k <= 16) gj_wave<16>(k, A, G, &nonpos);
        else if (k <= 32) gj_wave<32>(k, A, G, &nonpos);
        else gj_wave<64>(k, A, G, &nonpos);
    }
    __syncthreads();
    double fa = 0.0, fi = 0.0;
    double sym[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int w = tid + u * kNT;
        sym[u] = 0.0;
        if (w < kk) {
            const int i = w / k, c = w - i * k;
            sym[u] = 0.5 * (G[w] + G[c * k + i]);
            fa += A[w] * A[w];
            fi += sym[u] * sym[u];
        }
    }
    fa = block_sum_waves(fa, sh);   // its barriers also separate the reads above from the writes below
    fi = block_sum_waves(fi, sh);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int w = tid + u * kNT;
        if (w < kk) G[w] = sym[u];
    }
    const bool pos = nonpos == 0;
    __syncthreads();
    return pos && sqrt(fa) * sqrt(fi) < 1e-4 / ((double)k * 2.220446049250313e-16);
}

// Moore-Penrose pseudo-inverse of the symmetric k x k matrix A (LDS, left intact),
// result in G; V is scratch.  The Gauss-Jordan inverse (inv_gj) is taken when it is
// accepted; otherwise the Jacobi eigendecomposition decides.
__device__ __forceinline__ void pinv_sym_lds(int k, const double *A, double *V, double *G, double *sh, double *cs, double *sn,
                             int *flag, int *rank_sh) {
    const int tid = threadIdx.x;
    if (inv_gj(k, A, G, sh)) {
        if (tid == 0) *rank_sh = k;
        __syncthreads();
        return;
    }
    // V and G are free again: eigendecomposition of a copy of A
    for (int w = tid; w < k * k; w += kNT) G[w] = A[w];
    __syncthreads();
    jacobi_eig(k, G, V, cs, sn, flag);
    // eigenvalues (diagonal of G) are copied out before G is overwritten
    __shared__ double lam[kMaxK];
    for (int e = tid; e < k; e += kNT) lam[e] = G[e * k + e];
    __syncthreads();
    const double *Lm = lam;
    double lmax = 0.0;
    for (int e = 0; e < k; ++e) lmax = fmax(lmax, fabs(Lm[e]));
    const double thr = (double)k * 2.220446049250313e-16 * lmax;
    if (tid == 0) {
        int rk = 0;
        for (int e = 0; e < k; ++e) rk += fabs(Lm[e]) > thr;
        *rank_sh = rk;
    }
    for (int w = tid; w < k * k; w += kNT) {
        const int i = w / k, j = w - i * k;
        double s = 0.0;
        for (int e = 0; e < k; ++e)
            if (fabs(Lm[e]) > thr) s += V[i * k + e] * (1.0 / Lm[e]) * V[j * k + e];
        G[w] = s;
    }
    __syncthreads();
}

}  // namespace ba
