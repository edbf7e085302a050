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

// Sums of the pairs (a[2 b], a[2 b + 1]) over b < nb (16-byte aligned a) by the calling
// wavefront (all 64 lanes must call): lane l adds pairs l, l + 64, ... in that order, eight
// 16-byte loads in flight at a time (issued unconditionally, pairs past nb read pair 0 and
// are dropped), then the butterfly.  The order is fixed by nb alone.
__device__ __forceinline__ void wave_pair_sums(const double *__restrict__ a, int nb, double &s0, double &s1) {
    typedef double d2_t __attribute__((ext_vector_type(2)));
    const int lane = threadIdx.x & 63;
    const d2_t *p = reinterpret_cast<const d2_t *>(a);
    double x0 = 0.0, x1 = 0.0;
    for (int b0 = 0; b0 < nb; b0 += 512) {
        d2_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int b = b0 + 64 * j + lane;
            v[j] = p[b < nb ? b : 0];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (b0 + 64 * j + lane < nb) {
                x0 += v[j].x;
                x1 += v[j].y;
            }
        }
    }
    s0 = wave_sum(x0);
    s1 = wave_sum(x1);
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

// Value of v in lane l of the wavefront (l wave-uniform).
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Eigendecomposition of the symmetric k x k matrix A in LDS (k <= 64, row-major) by the
// block's 256 threads: on return the diagonal of A holds the eigenvalues and the columns
// of V the eigenvectors.
//  1. Householder tridiagonalisation, Q^T A Q = T: for column j, the reflector
//     H = I - b v v^T with H x = alpha e_1 for x = A[j+1.., j]; the trailing block becomes
//     A - v w^T - w v^T with p = b A v, w = p - (b/2)(v^T p) v.  v_1.. stays in the zeroed
//     part of column j, v_0 and b in LDS.  Four barriers per column.
//  2. Q = H_0 H_1 ... formed in V, the reflectors applied from the last to the first.
//  3. Implicit-shift QL iterations on T (the shift from the leading 2 x 2 block, the
//     bulge chased with Givens rotations from the bottom of the unreduced block up), by
//     the first wavefront: lane i keeps d_i and e_i in registers, every lane reads them
//     with readlane and runs the same scalar recurrence, and lane r applies each rotation
//     to row r of V.  A subdiagonal entry counts as zero when |e_m| <= eps (|d_m| + |d_m+1|).
__device__ __forceinline__ void sym_eig(int k, double *A, double *V) {
    __shared__ double hv0[kMaxK], hb[kMaxK], hp[kMaxK], hd[kMaxK], he[kMaxK + 1];
    __shared__ double s_alpha, s_K;
    const int tid = threadIdx.x, lane = tid & 63;
    const int r4 = tid >> 2, q4 = tid & 3;   // 4 threads per row (or column) of a trailing block
    for (int w = tid; w < k * k; w += kNT) V[w] = (w / k == w % k) ? 1.0 : 0.0;
    if (tid < kMaxK) hb[tid] = 0.0;
    __syncthreads();
    // 1. tridiagonalisation
    for (int j = 0; j + 2 < k; ++j) {
        const int m = k - j - 1, o = j + 1;
        if (tid < 64) {
            const double xi = lane < m ? A[(o + lane) * k + j] : 0.0;
            const double sigma = wave_sum(lane >= 1 && lane < m ? xi * xi : 0.0);
            if (lane == 0) {
                if (sigma == 0.0) {
                    hb[j] = 0.0;
                } else {
                    const double alpha = -copysign(sqrt(xi * xi + sigma), xi);
                    const double v0 = xi - alpha;
                    hv0[j] = v0;
                    hb[j] = 2.0 / (sigma + v0 * v0);
                    s_alpha = alpha;
                }
            }
        }
        __syncthreads();
        const double b = hb[j];
        if (b == 0.0) continue;   // column already reduced (uniform)
        const double v0 = hv0[j];
        // p = b A_sub v: row r4 of the m x m trailing block, four partial sums per row
        {
            double sum = 0.0;
            if (r4 < m)
                for (int c = q4; c < m; c += 4) sum += A[(o + r4) * k + o + c] * (c == 0 ? v0 : A[(o + c) * k + j]);
            sum += __shfl_xor(sum, 1, 64);
            sum += __shfl_xor(sum, 2, 64);
            if (q4 == 0 && r4 < m) hp[r4] = b * sum;
        }
        __syncthreads();
        if (tid < 64) {
            const double vr = lane == 0 ? v0 : A[(o + lane) * k + j];
            const double t = wave_sum(lane < m ? vr * hp[lane] : 0.0);
            if (lane == 0) s_K = 0.5 * b * t;
        }
        __syncthreads();
        {
            const double K = s_K;
            if (r4 < m) {
                const double vr = r4 == 0 ? v0 : A[(o + r4) * k + j];
                const double wr = hp[r4] - K * vr;
                for (int c = q4; c < m; c += 4) {
                    const double vc = c == 0 ? v0 : A[(o + c) * k + j];
                    const double wc = hp[c] - K * vc;
                    A[(o + r4) * k + o + c] -= vr * wc + wr * vc;
                }
            }
            if (tid == 0) {
                A[o * k + j] = s_alpha;
                A[j * k + o] = s_alpha;
            }
            if (tid >= 64 && tid - 64 < m - 1) A[j * k + o + 1 + (tid - 64)] = 0.0;   // row j past the band
        }
        __syncthreads();
    }
    for (int i = tid; i < k; i += kNT) {
        hd[i] = A[i * k + i];
        he[i] = i + 1 < k ? A[(i + 1) * k + i] : 0.0;
    }
    __syncthreads();
    // 2. Q = H_0 ... H_{k-3} into V, from the last reflector to the first
    for (int j = k - 3; j >= 0; --j) {
        const double b = hb[j];
        if (b == 0.0) continue;
        const int m = k - j - 1, o = j + 1;
        const double v0 = hv0[j];
        // u_c = v^T V_sub[:, c], four partial sums per column
        double u = 0.0;
        if (r4 < m)
            for (int r = q4; r < m; r += 4) u += (r == 0 ? v0 : A[(o + r) * k + j]) * V[(o + r) * k + o + r4];
        u += __shfl_xor(u, 1, 64);
        u += __shfl_xor(u, 2, 64);
        if (q4 == 0 && r4 < m) hp[r4] = b * u;
        __syncthreads();
        if (r4 < m) {
            const double vr = r4 == 0 ? v0 : A[(o + r4) * k + j];
            for (int c = q4; c < m; c += 4) V[(o + r4) * k + o + c] -= vr * hp[c];
        }
        __syncthreads();
    }
    // 3. implicit QL on (d, e): lane i keeps d_i and e_i in registers, every lane reads
    // them with readlane and runs the same scalar recurrence, and lane r applies each
    // rotation to row r of V
    if (tid < 64) {
        const double eps = 2.220446049250313e-16;
        double dl = lane < k ? hd[lane] : 0.0, el = lane < k ? he[lane] : 0.0;
        auto setl = [&](double &reg, int i, double v) {
            if (lane == i) reg = v;
        };
        for (int l = 0; l < k; ++l) {
            for (int iter = 0; iter < 64; ++iter) {
                // first m >= l with a negligible e_m (m = k - 1 when none)
                const double dn = __shfl_down(dl, 1, 64);
                const bool small = lane + 1 < k && fabs(el) <= eps * (fabs(dl) + fabs(dn));
                const uint64_t sm = __ballot(small && lane >= l);
                const int m = sm ? __ffsll((unsigned long long)sm) - 1 : k - 1;
                if (m == l) break;
                const double dlv = readlane_f64(dl, l), el_l = readlane_f64(el, l);
                double g = (readlane_f64(dl, l + 1) - dlv) / (2.0 * el_l);
                double r = sqrt(g * g + 1.0);
                g = readlane_f64(dl, m) - dlv + el_l / (g + copysign(r, g));
                double sn = 1.0, cn = 1.0, p = 0.0;
                bool early = false;
                // row `lane` of V: column i + 1 of the rotation in hand is carried in a
                // register (the previous rotation's new column i), so LDS is only read
                // ahead and written once per column
                double carry = lane < k ? V[lane * k + m] : 0.0;
                int i = m - 1;
                for (; i >= l; --i) {
                    const double zi = lane < k ? V[lane * k + i] : 0.0;
                    const double ei = readlane_f64(el, i);
                    const double f = sn * ei, bb = cn * ei;
                    // r = |(f, g)| and 1 / r from the hardware reciprocal square root and one
                    // Newton step (y <- y + y (1 - x y^2) / 2), which keeps the recurrence's
                    // dependency chain short
                    const double x = f * f + g * g;
                    double ir = __builtin_amdgcn_rsq(x);
                    ir = fma(0.5 * ir, fma(-x * ir, ir, 1.0), ir);
                    r = x > 0.0 ? x * ir : 0.0;
                    setl(el, i + 1, r);
                    if (r == 0.0) {   // exact split: deflate and restart the block
                        setl(dl, i + 1, readlane_f64(dl, i + 1) - p);
                        setl(el, m, 0.0);
                        early = true;
                        break;
                    }
                    sn = f * ir;
                    cn = g * ir;
                    g = readlane_f64(dl, i + 1) - p;
                    r = (readlane_f64(dl, i) - g) * sn + 2.0 * cn * bb;
                    p = sn * r;
                    setl(dl, i + 1, g + p);
                    g = cn * r - bb;
                    if (lane < k) V[lane * k + i + 1] = sn * zi + cn * carry;
                    carry = cn * zi - sn * carry;
                }
                if (lane < k) V[lane * k + i + 1] = carry;   // column l, or the split's i + 1
                if (!early) {
                    setl(dl, l, readlane_f64(dl, l) - p);
                    setl(el, l, g);
                    setl(el, m, 0.0);
                }
            }
        }
        if (lane < k) hd[lane] = dl;
    }
    __syncthreads();
    for (int i = tid; i < k; i += kNT) A[i * k + i] = hd[i];
    __syncthreads();
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
    // the previous lane's key by a DPP whole-wavefront shift (wave_shr:1; lane 0 keeps its
    // own and is a segment head regardless), not a cross-lane read through the LDS pipe
    const int prev = __builtin_amdgcn_update_dpp(key, key, 0x138, 0xf, 0xf, false);
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

// Sum of x over the lane's segment, rounded to T at the segment's last lane and returned
// in every lane of the segment (a float moves in one cross-lane read, a double in two).
template <typename T>
__device__ __forceinline__ T segment_sum(double x, const Segs &g) {
    return __shfl((T)segment_scan(x, g), g.end, 64);
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

// The same elimination by the four wavefronts of the block (k <= 64): wavefront w keeps
// rows [16 w, 16 w + 16) of the padded 64 x 64 matrix, lane c their entries in column c, in
// place (no rotation).  Step j: the wavefront holding row j puts it in LDS (two buffers
// used in turn, so one barrier per step orders each write after the last read of the same
// buffer), every lane reads its column's pivot-row entry and the pivot, and takes a_ij of
// its rows from lane j of its own wavefront (readlane).  Each step is 16 FMAs and 16
// cross-lane reads per lane instead of 63: with wide blocks the one-wavefront form is a
// chain of k (KP - 1) dependent steps.  Called by every thread of the block.
__device__ __forceinline__ void gj_block(int k, const double *A, double *G, int *bad, double *prow) {
    const int tid = threadIdx.x, w = tid >> 6, c = tid & 63;
    double a[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 16 * w + r;
        a[r] = (i < k && c < k) ? A[i * k + c] : (i == c ? 1.0 : 0.0);
    }
    bool nonpos = false;
    for (int jb = 0; jb < 4 && 16 * jb < k; ++jb) {
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int j = 16 * jb + jj;
            if (j < k) {
                double *buf = prow + (j & 1) * 64;
                if (w == jb) buf[c] = a[jj];
                __syncthreads();
                const double p = buf[j], pj = buf[c];
                nonpos |= !(p > 0.0);
                const double ip = 1.0 / (p > 0.0 ? p : 1.0);
                const bool piv = c == j;
                const double t = (piv ? 1.0 : pj) * ip;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const double aij = readlane_f64(a[r], j);
                    a[r] = (piv ? 0.0 : a[r]) - aij * t;
                }
                if (w == jb) a[jj] = t;   // the pivot row: a_jc / p, and 1 / p at c = j
            }
        }
    }
    if (c < k) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 16 * w + r;
            if (i < k) G[i * k + c] = a[r];
        }
    }
    if (tid == 0) *bad = nonpos;
}

// Inverse of the symmetric k x k matrix A (k <= 64, LDS) into G: Gauss-Jordan elimination
// on the diagonal pivots (gj_wave by the first wavefront up to k = 32, gj_block by the
// four beyond), then the result is
// symmetrised by the whole block.  Returns (the same in every thread) whether every
// pivot was positive (A positive definite) and |A|_F |A^-1|_F < 1e-4 / (k eps): then
// every eigenvalue lies above the drop threshold k eps max|l| (l_min >= 1 / |A^-1|_F,
// l_max <= |A|_F), so A^+ = A^-1.
__device__ __forceinline__ bool inv_gj(int k, const double *A, double *G, double *sh) {
    constexpr int U = kMaxK * kMaxK / kNT;   // elements per thread at most
    __shared__ int nonpos;
    __shared__ double prow[2 * 64];
    const int tid = threadIdx.x;
    const int kk = k * k;
    if (k > 32) {
        gj_block(k, A, G, &nonpos, prow);
    } else if (tid < 64) {
        if (k <= 16) gj_wave<16>(k, A, G, &nonpos);
        else gj_wave<32>(k, A, G, &nonpos);
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
// accepted; otherwise the eigendecomposition (sym_eig) decides.
__device__ __forceinline__ void pinv_sym_lds(int k, const double *A, double *V, double *G, double *sh, int *rank_sh) {
    const int tid = threadIdx.x;
    if (inv_gj(k, A, G, sh)) {
        if (tid == 0) *rank_sh = k;
        __syncthreads();
        return;
    }
    // V and G are free again: eigendecomposition of a copy of A
    for (int w = tid; w < k * k; w += kNT) G[w] = A[w];
    __syncthreads();
    sym_eig(k, G, V);
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
