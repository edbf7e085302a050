// Explicit reduced camera system in block-sparse rows (9 x 9 FP64 blocks), the
// paper's own representation of S (Sec. 3.2, "Optimized implementation": S_jk is
// nonzero iff cameras j and k observe a common point; Sec. 4.1 forms it as a
// row-major sparse matrix).
//
// Value layout of block row j (nb blocks, starting at block b0 = row_ptr[j]): the 81 nb
// values at val + 81 b0 are stored row-of-the-block-major, [r][t][c] = S_(j, col t)[r][c]
// at r (9 nb) + 9 t + c.  Each of the nine rows r of the block row is then one contiguous
// run of 9 nb values, multiplied entry by entry with the same gathered vector
// (v_(col t))_c, which the products load once for all nine.
//   S_jj = D(S)_j                                   (already formed by the build)
//   S_jk = - sum_{l observed by j and k} W_jl V_l^-1 W_kl^T,   W_jl = J_p,jl^T J_l,jl
// Assembly: one wavefront per block row j holds the row's blocks in LDS and adds the
// row's contributions, 64 at a time, in a fixed order.
#include "ba_internal.h"
#include "kernels.h"
#include "dev_la.h"

namespace ba {

typedef double dbl2b_t __attribute__((ext_vector_type(2)));

// W = J_p^T J_l (9 x 3) of the observation in tile-stream slot s (record layout of
// the S product: 12 x 16 B words per slot, 64 slots per tile)
__device__ __forceinline__ void w_of_slot(const double *__restrict__ J64, int64_t s, double W[27]) {
    const dbl2b_t *p = reinterpret_cast<const dbl2b_t *>(J64) + (s >> 6) * 12 * 64 + (s & 63);
    double v[24];
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const dbl2b_t d = p[q * 64];
        v[2 * q] = d.x;
        v[2 * q + 1] = d.y;
    }
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) W[r * 3 + c] = v[r] * v[18 + c] + v[9 + r] * v[21 + c];
}

// ---- pattern on the device: row j's columns are the cameras that share a landmark
// with camera j (j included).  One work-group per row marks them in an LDS bitmap of
// n_cams bits (every observation o of camera j, then every observation slot of o's
// landmark); the set bits, read in word order, are the row's columns in ascending order.
__device__ void row_bitmap(int j, const int64_t *__restrict__ cam_ptr, const int64_t *__restrict__ cam_obs,
                           const int32_t *__restrict__ obs_lm, const int32_t *__restrict__ lmk_store,
                           const int64_t *__restrict__ lmk_first_slot, const int32_t *__restrict__ lmk_count,
                           const int32_t *__restrict__ slot_cam, int nwords, uint32_t *bm) {
    for (int w = threadIdx.x; w < nwords; w += blockDim.x) bm[w] = 0u;
    __syncthreads();
    for (int64_t u = cam_ptr[j] + threadIdx.x; u < cam_ptr[j + 1]; u += blockDim.x) {
        const int s = lmk_store[obs_lm[cam_obs[u]]];
        const int64_t f = lmk_first_slot[s];
        const int c = lmk_count[s];
        for (int q = 0; q < c; ++q) {
            const int k = slot_cam[f + q];
            atomicOr(&bm[k >> 5], 1u << (k & 31));
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_bsr_rowcount(int nwords, const int64_t *__restrict__ cam_ptr,
                                                      const int64_t *__restrict__ cam_obs,
                                                      const int32_t *__restrict__ obs_lm,
                                                      const int32_t *__restrict__ lmk_store,
                                                      const int64_t *__restrict__ lmk_first_slot,
                                                      const int32_t *__restrict__ lmk_count,
                                                      const int32_t *__restrict__ slot_cam, int32_t *__restrict__ nnz) {
    extern __shared__ uint32_t bm[];
    __shared__ int part[256 / 64];
    const int j = blockIdx.x;
    row_bitmap(j, cam_ptr, cam_obs, obs_lm, lmk_store, lmk_first_slot, lmk_count, slot_cam, nwords, bm);
    int c = 0;
    for (int w = threadIdx.x; w < nwords; w += blockDim.x) c += __popc(bm[w]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) nnz[j] = part[0] + part[1] + part[2] + part[3];
}

// Writes row j's columns (ascending) at col[row_ptr[j] ...]: words are taken 256 at a
// time, each thread's set bits go after the set bits of the words before it.
__global__ __launch_bounds__(256) void k_bsr_rowfill(int nwords, const int64_t *__restrict__ cam_ptr,
                                                     const int64_t *__restrict__ cam_obs,
                                                     const int32_t *__restrict__ obs_lm,
                                                     const int32_t *__restrict__ lmk_store,
                                                     const int64_t *__restrict__ lmk_first_slot,
                                                     const int32_t *__restrict__ lmk_count,
                                                     const int32_t *__restrict__ slot_cam,
                                                     const int32_t *__restrict__ row_ptr, int32_t *__restrict__ col) {
    extern __shared__ uint32_t bm[];
    __shared__ int scan[256];
    const int j = blockIdx.x;
    row_bitmap(j, cam_ptr, cam_obs, obs_lm, lmk_store, lmk_first_slot, lmk_count, slot_cam, nwords, bm);
    int base = row_ptr[j];
    for (int w0 = 0; w0 < nwords; w0 += 256) {
        const int w = w0 + (int)threadIdx.x;
        const uint32_t bits = w < nwords ? bm[w] : 0u;
        scan[threadIdx.x] = __popc(bits);
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {   // inclusive scan (Hillis-Steele)
            const int add = (int)threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
            __syncthreads();
            scan[threadIdx.x] += add;
            __syncthreads();
        }
        int pos = base + scan[threadIdx.x] - __popc(bits);
        for (uint32_t b = bits; b; b &= b - 1) col[pos++] = w * 32 + __ffs(b) - 1;
        base += scan[255];
        __syncthreads();
    }
}

// One wavefront per (block row j, piece p of at most `piece` of its blocks): the piece's
// blocks in LDS (and the row's whole column list); camera j's observations 64 at a time,
// lane i taking observation o (of landmark l) and adding -W_o V_l^-1 W_q^T into the block
// of q's camera for every other observation q of l whose block lies in the piece, in slot
// order.  One wavefront issues all the LDS atomics of a block, so they resolve in program
// order and, within an instruction, in lane order: the sums are reproducible.  Rows wider
// than one piece (dense S) are assembled by several wavefronts, each re-reading the row's
// observations.  The diagonal block is D(S)_j.
__global__ __launch_bounds__(64) void k_bsr_assemble(const int64_t *__restrict__ cam_ptr,
                                                     const int64_t *__restrict__ cam_obs,
                                                     const int32_t *__restrict__ obs_lm,
                                                     const int32_t *__restrict__ lmk_store,
                                                     const int64_t *__restrict__ lmk_first_slot,
                                                     const int32_t *__restrict__ lmk_count,
                                                     const int32_t *__restrict__ slot_cam,
                                                     const int64_t *__restrict__ obs_slot,
                                                     const double *__restrict__ J64, const double *__restrict__ vinv,
                                                     const double *__restrict__ Dblk,
                                                     const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, double *__restrict__ val,
                                                     int piece) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    const int b0 = row_ptr[j], nb = row_ptr[j + 1] - b0;
    const int pb = blockIdx.y * piece;            // first block of this wavefront's piece
    if (pb >= nb) return;
    const int pn = min(piece, nb - pb);
    double *acc = reinterpret_cast<double *>(smem);
    int32_t *rc = reinterpret_cast<int32_t *>(acc + (size_t)piece * 81);
    for (int e = lane; e < pn * 81; e += 64) acc[e] = 0.0;
    for (int e = lane; e < nb; e += 64) rc[e] = col[b0 + e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int64_t u = cam_ptr[j] + lane; u < cam_ptr[j + 1]; u += 64) {
        const int64_t o = cam_obs[u];
        const int s = lmk_store[obs_lm[o]];
        const int64_t f = lmk_first_slot[s];
        const int c = lmk_count[s];
        double Wo[27], G[27];
        w_of_slot(J64, obs_slot[o], Wo);
        const double *vi = vinv + (int64_t)s * 6;
        const double v0 = vi[0], v1 = vi[1], v2 = vi[2], v3 = vi[3], v4 = vi[4], v5 = vi[5];
#pragma unroll
        for (int r = 0; r < 9; ++r) {   // G = W_o V^-1 (V^-1 symmetric, packed)
            const double x0 = Wo[r * 3], x1 = Wo[r * 3 + 1], x2 = Wo[r * 3 + 2];
            G[r * 3] = x0 * v0 + x1 * v1 + x2 * v2;
            G[r * 3 + 1] = x0 * v1 + x1 * v3 + x2 * v4;
            G[r * 3 + 2] = x0 * v2 + x1 * v4 + x2 * v5;
        }
        for (int q = 0; q < c; ++q) {
            const int k = slot_cam[f + q];
            if (k == j) continue;
            int lo = 0, hi = nb - 1;   // block of column k (present: k shares landmark l)
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (rc[mid] < k) lo = mid + 1;
                else hi = mid;
            }
            if (lo < pb || lo >= pb + pn) continue;   // another wavefront's piece
            double Wq[27];
            w_of_slot(J64, f + q, Wq);
            double *blk = acc + (size_t)(lo - pb) * 81;
#pragma unroll
            for (int r = 0; r < 9; ++r)
#pragma unroll
                for (int cc = 0; cc < 9; ++cc)
                    atomicAdd(&blk[r * 9 + cc],
                              -(G[r * 3] * Wq[cc * 3] + G[r * 3 + 1] * Wq[cc * 3 + 1] + G[r * 3 + 2] * Wq[cc * 3 + 2]));
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // diagonal block: D(S)_j, formed by the build from the same sums
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rc[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= pb && lo < pb + pn)
        for (int e = lane; e < 81; e += 64) acc[(size_t)(lo - pb) * 81 + e] = Dblk[(int64_t)j * 81 + e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // out in the row-of-the-block-major layout: run r holds 9 nb values
    const int64_t L = (int64_t)nb * 9;
    double *out = val + (int64_t)b0 * 81;
    for (int e = lane; e < pn * 81; e += 64) {
        const int t = e / 81, rc = e - t * 81, r = rc / 9, c = rc - r * 9;
        out[r * L + (int64_t)(pb + t) * 9 + c] = acc[e];
    }
}

// Loads of kBsrAhead positions e0 + 256 u of a block row (its nine runs of L values at S,
// columns cj): the nine values sv[u][r] = S[r L + e] and the gathered vector entry
// vg[u] = v[9 col(e / 9) + e mod 9]; with group, also gk[u] = group[col(e / 9)].
// Positions at or beyond L read nothing and give zeros.
constexpr int kBsrAhead = 4;

__device__ __forceinline__ void bsr_fetch(const double *__restrict__ S, const int32_t *__restrict__ cj,
                                          const double *__restrict__ v, int L, int e0, double (&sv)[kBsrAhead][9],
                                          double (&vg)[kBsrAhead], const int32_t *__restrict__ group = nullptr,
                                          int *gk = nullptr) {
    int k[kBsrAhead], c[kBsrAhead];
#pragma unroll
    for (int u = 0; u < kBsrAhead; ++u) {
        const int e = e0 + u * 256;
        const int t = e < L ? e / 9 : 0;
        c[u] = e - t * 9;
        k[u] = cj[t];
    }
#pragma unroll
    for (int u = 0; u < kBsrAhead; ++u) {
        const int e = e0 + u * 256;
#pragma unroll
        for (int r = 0; r < 9; ++r) sv[u][r] = e < L ? S[(int64_t)r * L + e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBsrAhead; ++u) {
        const bool ok = e0 + u * 256 < L;
        vg[u] = ok ? v[(int64_t)k[u] * 9 + c[u]] : 0.0;
        if (group) gk[u] = group[k[u]];
    }
}

// y_j = sum_t S_(j, col t) v_(col t).  One work-group of 256 threads per block row; thread
// i takes positions e = i, i + 256, ... of the row's 9 nb entries per block row r (block t
// = e / 9, column c = e % 9): it gathers (v_(col t))_c once and multiplies it with the nine
// entries S[r][e], which the work-group reads as nine coalesced runs.  Each output row r
// is added over the lanes of a wavefront, then over the four wavefronts in a fixed order.
// With gram, row j also leaves gram[2 j] = y_j . v_j and gram[2 j + 1] = v_j . gr_j (the
// Gram products Q^T P and P^T r of a one-column block, Q = S P).  When `done` is set and
// nonzero, the launch does nothing.
__global__ __launch_bounds__(256) void k_bsr_mv(int np, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col, const double *__restrict__ val,
                                                const double *__restrict__ v, double *__restrict__ y,
                                                const double *__restrict__ done, double *__restrict__ gram,
                                                const double *__restrict__ gr) {
    if (done && *done != 0.0) return;
    __shared__ double sh[4][9];
    const int j = blockIdx.x;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int b0 = row_ptr[j];
    const int L = (row_ptr[j + 1] - b0) * 9;
    const double *S = val + (int64_t)b0 * 81;
    const int32_t *cj = col + b0;
    double acc[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) acc[r] = 0.0;
    // kBsrAhead positions per trip (e0, e0 + 256, ...), all their loads issued before the
    // first multiply; each thread still adds its positions in ascending order
    for (int e0 = tid; e0 < L; e0 += kBsrAhead * 256) {
        double sv[kBsrAhead][9], vg[kBsrAhead];
        bsr_fetch(S, cj, v, L, e0, sv, vg);
#pragma unroll
        for (int u = 0; u < kBsrAhead; ++u)
#pragma unroll
            for (int r = 0; r < 9; ++r) acc[r] += sv[u][r] * vg[u];
    }
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const double t = wave_sum(acc[r]);
        if (lane == 0) sh[w][r] = t;
    }
    __syncthreads();
    if (tid >= 64) return;
    double yr = 0.0, qp = 0.0, pr = 0.0;
    if (tid < 9) {
        yr = (sh[0][tid] + sh[1][tid]) + (sh[2][tid] + sh[3][tid]);
        const int64_t i = (int64_t)j * 9 + tid;
        y[i] = yr;
        if (gram) {
            const double vi = v[i];
            qp = yr * vi;
            pr = vi * gr[i];
        }
    }
    if (!gram) return;   // the same for the whole launch
    qp = wave_sum(qp);
    pr = wave_sum(pr);
    if (tid == 0) {
        gram[2 * j] = qp;
        gram[2 * j + 1] = pr;
    }
}

// Y[p][row of j] = sum over blocks t of row j with group(col t) == p of S_(j, col t) z_(col t)
// (the multidirectional product of eq. (19)'s input).  One work-group of 256 threads per
// block row, positions as in k_bsr_mv.  The subsets are ranges of consecutive cameras and
// a row's columns ascend, so within one trip a wavefront's 64 consecutive positions fall
// into a few runs of equal subset: for each of the nine rows the products are added over
// each run by a segmented scan across the lanes (segment_scan), and the run's last lane
// adds the total into the wavefront's LDS row of that subset (distinct subsets per
// instruction, trips in program order).  The four wavefronts' rows are then added in a
// fixed order.
__global__ __launch_bounds__(256) void k_bsr_mm_grouped(int np, int N, int64_t n, const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const int32_t *__restrict__ group,
                                                        const double *__restrict__ z, double *__restrict__ Y,
                                                        const double *__restrict__ skip) {
    if (skip && *skip != 0.0) return;
    __shared__ double yl[4][kMaxBlock * 9];
    const int j = blockIdx.x;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int e = lane; e < N * 9; e += 64) yl[w][e] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int b0 = row_ptr[j];
    const int L = (row_ptr[j + 1] - b0) * 9;
    const double *S = val + (int64_t)b0 * 81;
    const int32_t *cj = col + b0;
    for (int e0 = tid; e0 - lane < L; e0 += kBsrAhead * 256) {   // whole wavefronts trip together
        double sv[kBsrAhead][9], zg[kBsrAhead];
        int gk[kBsrAhead];
        bsr_fetch(S, cj, z, L, e0, sv, zg, group, gk);
#pragma unroll
        for (int u = 0; u < kBsrAhead; ++u) {
            const int e = e0 + u * 256;
            if (e - lane >= L) break;   // wave-uniform: no position of this wavefront is left
            const bool ok = e < L;
            const Segs sg = key_segments(ok ? gk[u] : 64 + lane, lane);
            const bool last = ok && sg.end == lane;
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                const double t = segment_scan(sv[u][r] * zg[u], sg);
                if (last) yl[w][gk[u] * 9 + r] += t;
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < N * 9; e += 256) {
        const int p = e / 9, rr = e - p * 9;
        Y[(int64_t)p * n + (int64_t)j * 9 + rr] = (yl[0][e] + yl[1][e]) + (yl[2][e] + yl[3][e]);
    }
}

void launch_bsr_rowcount(int np, const BsrGather &g, int32_t *nnz, hipStream_t s) {
    const int nwords = (np + 31) / 32;
    hipLaunchKernelGGL(k_bsr_rowcount, dim3(np), dim3(256), (size_t)nwords * 4, s, nwords, g.cam_ptr, g.cam_obs,
                       g.obs_lm, g.lmk_store, g.lmk_first_slot, g.lmk_count, g.slot_cam, nnz);
}

void launch_bsr_rowfill(int np, const BsrGather &g, const int32_t *row_ptr, int32_t *col, hipStream_t s) {
    const int nwords = (np + 31) / 32;
    hipLaunchKernelGGL(k_bsr_rowfill, dim3(np), dim3(256), (size_t)nwords * 4, s, nwords, g.cam_ptr, g.cam_obs,
                       g.obs_lm, g.lmk_store, g.lmk_first_slot, g.lmk_count, g.slot_cam, row_ptr, col);
}

int bsr_assembly_piece(int max_row, size_t lds_bytes) {
    const size_t cols = (size_t)max_row * sizeof(int32_t);
    if (lds_bytes <= cols + 81 * sizeof(double)) return 0;
    return (int)std::min<size_t>((size_t)max_row, (lds_bytes - cols) / (81 * sizeof(double)));
}

void launch_bsr_assemble(int np, const BsrGather &g, const int64_t *obs_slot, const double *J64, const double *vinv,
                         const double *Dblk, const int32_t *row_ptr, const int32_t *col, int max_row, int piece,
                         double *val, hipStream_t s) {
    const size_t lds = (size_t)piece * 81 * sizeof(double) + (size_t)max_row * sizeof(int32_t);
    const unsigned pieces = (unsigned)((max_row + piece - 1) / piece);
    hipLaunchKernelGGL(k_bsr_assemble, dim3(np, pieces), dim3(64), lds, s, g.cam_ptr, g.cam_obs, g.obs_lm,
                       g.lmk_store, g.lmk_first_slot, g.lmk_count, g.slot_cam, obs_slot, J64, vinv, Dblk, row_ptr,
                       col, val, piece);
}

void launch_bsr_mv(int np, const int32_t *row_ptr, const int32_t *col, const double *val, const double *v, double *y,
                   const double *done, hipStream_t s, double *gram, const double *gram_r) {
    hipLaunchKernelGGL(k_bsr_mv, dim3(np), dim3(256), 0, s, np, row_ptr, col, val, v, y, done, gram, gram_r);
}

void launch_bsr_mm_grouped(int np, int N, const int32_t *row_ptr, const int32_t *col, const double *val,
                           const int32_t *group, const double *z, double *Y, hipStream_t s, const double *skip) {
    hipLaunchKernelGGL(k_bsr_mm_grouped, dim3(np), dim3(256), 0, s, np, N, (int64_t)np * 9, row_ptr, col, val, group,
                       z, Y, skip);
}

}  // namespace ba
