// Implicit Schur products of the reduced camera system (Sec. 3.1, eq. (14)):
//   S v = U_lambda v - W V_lambda^-1 W^T v
// computed from the per-observation Jacobian blocks without forming W or S:
//   e_o = J_p,o v_c                    (2)
//   g_l = sum_{o in l} J_l,o^T e_o     (3)   = (W^T v)_l
//   h_l = V_l^-1 g_l
//   y_c = sum_{o in c} J_p,o^T (e_o - J_l,o h_l) + lambda diag(U_c) v_c
// One wavefront owns one chunk of landmark tiles: landmark sums are reduced in
// LDS inside the tile, camera sums in a per-wavefront LDS accumulator indexed
// by chunk-local camera slot.  Each chunk writes one partial row per slot and a
// second kernel adds the partial rows of every camera in a fixed order, so the
// result does not depend on scheduling and no global atomics are used.
//
// The multidirectional product (Sec. 3.2, "Optimized implementation",
// eq. (19)) applies S to the N columns Z[:, p] = z restricted to the poses of
// subset p.  An observation of camera c in subset q contributes e_o to column q
// only; its landmark then carries one h_{l,p} per subset p among its observers,
// and every observation of l receives a contribution in each such column.
#include "ba_internal.h"
#include "kernels.h"
#include "dev_la.h"

namespace ba {

typedef double dbl2_t __attribute__((ext_vector_type(2)));
typedef float flt4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Per-observation stream record of one lane: 2 DP + 6 values (J_p rows 0, 1, then J_l
// rows 0, 1; DP = 9, or 6 for extrinsics only) as RecordShape<DP> 16 B words in FP64,
// FP32 or BF16.  Loads fetch the raw 16-byte words; unpacking (and the BF16
// conversion) is left to the point of use so that a prefetched record needs no wait.
template <int PREC, int DP>
struct Stream;
template <int DP>
struct Stream<0, DP> {
    typedef dbl2_t word_t;
    static constexpr int kWords = RecordShape<DP>::kW64;
    template <typename T>
    static __device__ __forceinline__ void unpack(const word_t (&w)[kWords], T (&v)[2 * DP + 6]) {
#pragma unroll
        for (int q = 0; q < kWords; ++q) {
            v[2 * q] = (T)w[q].x;
            v[2 * q + 1] = (T)w[q].y;
        }
    }
};
template <int DP>
struct Stream<1, DP> {
    typedef flt4_t word_t;
    static constexpr int kWords = RecordShape<DP>::kW32;
    template <typename T>
    static __device__ __forceinline__ void unpack(const word_t (&w)[kWords], T (&v)[2 * DP + 6]) {
#pragma unroll
        for (int q = 0; q < kWords; ++q) {
            const float x[4] = {w[q].x, w[q].y, w[q].z, w[q].w};
#pragma unroll
            for (int h = 0; h < 4; ++h)
                if (4 * q + h < 2 * DP + 6) v[4 * q + h] = (T)x[h];
        }
    }
};
template <int DP>
struct Stream<2, DP> {
    typedef u32x4_t word_t;
    static constexpr int kWords = RecordShape<DP>::kW16;
    template <typename T>
    static __device__ __forceinline__ void unpack(const word_t (&w)[kWords], T (&v)[2 * DP + 6]) {
#pragma unroll
        for (int q = 0; q < kWords; ++q) {
            const uint32_t u[4] = {w[q].x, w[q].y, w[q].z, w[q].w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                if (8 * q + 2 * h < 2 * DP + 6) v[8 * q + 2 * h] = (T)bf16_to_f32(u[h] & 0xFFFFu);
                if (8 * q + 2 * h + 1 < 2 * DP + 6) v[8 * q + 2 * h + 1] = (T)bf16_to_f32(u[h] >> 16);
            }
        }
    }
};

template <int PREC, int DP>
__device__ __forceinline__ void load_words(const void *J, int64_t tile, int lane,
                                           typename Stream<PREC, DP>::word_t (&w)[Stream<PREC, DP>::kWords]) {
    typedef typename Stream<PREC, DP>::word_t W;
    constexpr int K = Stream<PREC, DP>::kWords;
    const W *p = reinterpret_cast<const W *>(J) + tile * K * kTile + lane;
#pragma unroll
    for (int q = 0; q < K; ++q) w[q] = __builtin_nontemporal_load(p + q * kTile);
}

template <int PREC, int DP>
struct Loader {
    template <typename T>
    static __device__ __forceinline__ void load(const void *J, int64_t tile, int lane, T (&v)[2 * DP + 6]) {
        typename Stream<PREC, DP>::word_t w[Stream<PREC, DP>::kWords];
        load_words<PREC, DP>(J, tile, lane, w);
        Stream<PREC, DP>::template unpack<T>(w, v);
    }
};

// ---------------------------------------------------------------- one column

// The work-group of the chunk kernels is one wavefront.  A wavefront's LDS
// instructions are performed in issue order, so ordering them needs only a
// code-motion barrier with wavefront-scope fences, not s_barrier -- which would
// also wait for the global loads of the next tile that are already in flight.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Record, V_l^-1 and slot word of one tile for one lane.  FP64 and FP32 records
// are kept as the 24 values themselves (loading them is the unpacking); BF16
// records are kept as raw words and converted when the tile is processed, so
// that no conversion waits on a load in flight.
template <int PREC, typename T, int DP>
struct TileBuf {
    T v[2 * DP + 6];
    dbl2_t vi[3];
    uint32_t mt;
};
template <typename T, int DP>
struct TileBuf<2, T, DP> {
    u32x4_t w[RecordShape<DP>::kW16];
    dbl2_t vi[3];
    uint32_t mt;
};

template <int PREC, typename T, int DP>
__device__ __forceinline__ void fetch_record(const void *J, int t, int lane, TileBuf<PREC, T, DP> &b) {
    if constexpr (PREC == 0) {
        constexpr int K = RecordShape<DP>::kW64;
        const dbl2_t *p = reinterpret_cast<const dbl2_t *>(J) + (int64_t)t * K * kTile + lane;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const dbl2_t d = __builtin_nontemporal_load(p + q * kTile);
            b.v[2 * q] = d.x;
            b.v[2 * q + 1] = d.y;
        }
    } else if constexpr (PREC == 1) {
        constexpr int K = RecordShape<DP>::kW32;
        const flt4_t *p = reinterpret_cast<const flt4_t *>(J) + (int64_t)t * K * kTile + lane;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const flt4_t f = __builtin_nontemporal_load(p + q * kTile);
            const float x[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
            for (int h = 0; h < 4; ++h)
                if (4 * q + h < 2 * DP + 6) b.v[4 * q + h] = x[h];
        }
    } else {
        load_words<2, DP>(J, t, lane, b.w);
    }
}

// Requests the record and V^-1 of tile t (slot word m, already loaded) into b.
// Padding slots read V^-1 of the tile's first landmark (every tile holds at
// least one) and ignore it.
template <int PREC, typename T, int DP>
__device__ __forceinline__ void fetch_tile(const SchurArgs &a, int t, int lane, uint32_t m, TileBuf<PREC, T, DP> &b) {
    b.mt = m;
    fetch_record<PREC, T, DP>(a.J, t, lane, b);
    const int ll = m != kPad ? (int)((m >> 16) & 63u) : 0;
    const dbl2_t *p = reinterpret_cast<const dbl2_t *>(a.vinv + (int64_t)(a.tile_lmk_base[t] + ll) * 6);
#pragma unroll
    for (int q = 0; q < 3; ++q) b.vi[q] = p[q];
}

// Segment layout of a tile's lanes: a landmark's observations occupy consecutive lanes, so
// each lane's segment is the run of lanes with its landmark index (padding lanes form
// segments of their own); the scan itself is in dev_la.h.
__device__ __forceinline__ Segs tile_segments(uint32_t mt, int lane) {
    return key_segments(mt != kPad ? (int)((mt >> 16) & 63u) : 64 + lane, lane);
}

// e = J_p v, g_l = sum J_l^T e, h_l = V_l^-1 g_l, y_c += J_p^T (e - J_l h_l) (LDS).  Products
// are formed in T; the sums g_l and y_c accumulate in FP64 for every precision.  Besides
// being the more accurate choice, it is the faster one on gfx950: with FP32 LDS accumulators
// (ds_add_f32) the FP32 product took 370 us on the F-1936-shaped problem, with FP64 ones
// (ds_add_f64) 131 us.  Landmark sums: with SEG, segmented sums across the landmark's lanes
// in registers (no LDS, no wavefront sync; the reduced-precision products, which the LDS
// work bounds); without, FP64 LDS atomics into a per-landmark row (the FP64 product, which
// HBM bounds and which keeps three wavefronts per SIMD within its registers).  The camera
// sums go to LDS, whose atomics one wavefront issues in program order (lane order within
// an instruction).
template <typename T, int DP, bool SEG>
__device__ __forceinline__ void schur_tile(const T (&J)[2 * DP + 6], const dbl2_t (&vi)[3], uint32_t mt, int lane,
                                           const T *vloc, double *yloc, double *gloc) {
    constexpr int L0 = 2 * DP, L1 = 2 * DP + 3;   // J_l rows 0 and 1
    const bool valid = mt != kPad;
    const int slot = valid ? (int)(mt & 0xFFFFu) : 0;
    const int ll = valid ? (int)((mt >> 16) & 63u) : 0;
    T vc[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) vc[k] = vloc[slot * DP + k];
    T e0 = 0, e1 = 0;
#pragma unroll
    for (int k = 0; k < DP; ++k) {
        e0 += J[k] * vc[k];
        e1 += J[DP + k] * vc[k];
    }
    T gs[3];   // g_l, rounded to T where h = V^-1 g is formed
    if constexpr (SEG) {
        const Segs sg = tile_segments(mt, lane);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            gs[k] = segment_sum<T>(valid ? (double)(J[L0 + k] * e0 + J[L1 + k] * e1) : 0.0, sg);
    } else {
        gloc[lane * 3 + 0] = 0;
        gloc[lane * 3 + 1] = 0;
        gloc[lane * 3 + 2] = 0;
        wave_sync();
        if (valid) {
#pragma unroll
            for (int k = 0; k < 3; ++k) atomicAdd(&gloc[ll * 3 + k], (double)(J[L0 + k] * e0 + J[L1 + k] * e1));
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < 3; ++k) gs[k] = (T)gloc[ll * 3 + k];
    }
    if (valid) {
        const T w0 = (T)vi[0].x, w1 = (T)vi[0].y, w2 = (T)vi[1].x;
        const T w3 = (T)vi[1].y, w4 = (T)vi[2].x, w5 = (T)vi[2].y;
        const T g0 = gs[0], g1 = gs[1], g2 = gs[2];
        const T h0 = w0 * g0 + w1 * g1 + w2 * g2;
        const T h1 = w1 * g0 + w3 * g1 + w4 * g2;
        const T h2 = w2 * g0 + w4 * g1 + w5 * g2;
        const T f0 = e0 - (J[L0] * h0 + J[L0 + 1] * h1 + J[L0 + 2] * h2);
        const T f1 = e1 - (J[L1] * h0 + J[L1 + 1] * h1 + J[L1 + 2] * h2);
#pragma unroll
        for (int k = 0; k < DP; ++k) atomicAdd(&yloc[slot * DP + k], (double)(J[k] * f0 + J[DP + k] * f1));
    }
    if constexpr (!SEG) wave_sync();   // the landmark rows are reset by the next tile
}

template <int PREC, typename T, int DP>
__device__ __forceinline__ void process_tile(const TileBuf<PREC, T, DP> &b, int lane, const T *vloc, double *yloc,
                                             double *gloc) {
    if constexpr (PREC == 2) {
        T J[2 * DP + 6];
        Stream<2, DP>::template unpack<T>(b.w, J);
        schur_tile<T, DP, true>(J, b.vi, b.mt, lane, vloc, yloc, gloc);
    } else {
        schur_tile<T, DP, PREC != 0>(b.v, b.vi, b.mt, lane, vloc, yloc, gloc);
    }
}

// Software pipeline over the tiles of the chunk with two buffers: the record and
// V^-1 of tile t + 1 and the slot word of tile t + 2 are requested before tile t
// is processed, so a wavefront keeps up to two tiles of the stream in flight.
template <int PREC, typename T, int DP>
__global__ __launch_bounds__(64) void k_schur1(SchurArgs a, const double *__restrict__ v) {
    if (a.done && *a.done != 0.0) return;
    if (a.seg_skip && a.seg_skip[a.chunk_seg[blockIdx.x]]) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double *yloc = reinterpret_cast<double *>(smem);
    double *gloc = yloc + a.max_slots * DP;                                   // FP64: landmark rows
    T *vloc = reinterpret_cast<T *>(gloc + (PREC == 0 ? 3 * kTile : 0));
    const int chunk = blockIdx.x;
    const int lane = threadIdx.x;
    const int pb = a.chunk_part[chunk];
    const int ns = a.chunk_part[chunk + 1] - pb;
    const int t0 = a.chunk_tile[chunk], t1 = a.chunk_tile[chunk + 1];
    const uint32_t *meta = a.meta + lane;
    const int tl = t1 - 1;   // slot words past the chunk's end are read from its last tile
    TileBuf<PREC, T, DP> A, B;
    uint32_t mA, mB = 0;
    if (t0 < t1) {
        fetch_tile<PREC, T, DP>(a, t0, lane, meta[(int64_t)t0 * kTile], A);
        mB = meta[(int64_t)min(t0 + 1, tl) * kTile];
    }
    for (int i = lane; i < ns * DP; i += kTile) {
        vloc[i] = (T)v[(int64_t)a.part_cam[pb + i / DP] * DP + i % DP];
        yloc[i] = 0.0;
    }
    wave_sync();
    // steady state: tiles t, t + 1 and t + 2 exist, so both requests are unconditional
    // (a branch around a load leaves the compiler waiting for it at the join)
    int t = t0;
    for (; t + 2 < t1; t += 2) {
        fetch_tile<PREC, T, DP>(a, t + 1, lane, mB, B);
        mA = meta[(int64_t)(t + 2) * kTile];
        process_tile<PREC, T, DP>(A, lane, vloc, yloc, gloc);
        fetch_tile<PREC, T, DP>(a, t + 2, lane, mA, A);
        mB = meta[(int64_t)min(t + 3, tl) * kTile];
        process_tile<PREC, T, DP>(B, lane, vloc, yloc, gloc);
    }
    // the last one or two tiles
    if (t + 1 < t1) {
        fetch_tile<PREC, T, DP>(a, t + 1, lane, mB, B);
        process_tile<PREC, T, DP>(A, lane, vloc, yloc, gloc);
        process_tile<PREC, T, DP>(B, lane, vloc, yloc, gloc);
    } else if (t < t1) {
        process_tile<PREC, T, DP>(A, lane, vloc, yloc, gloc);
    }
    // row of slot k goes to its camera-major position
    for (int i = lane; i < ns * DP; i += kTile) {
        const int64_t row = a.part_dst[pb + i / DP];
        a.partial[row * DP + i % DP] = (double)yloc[i];
    }
}

// Sum of the DP-vectors rows[a..b) by the calling wavefront, R = 64 / DP rows at a
// time (7 for DP = 9, 10 for DP = 6): lane l < R DP adds component l % DP of rows
// a + l / DP + R i, eight rows per batch with all eight loads in flight (rows past b read
// row a and are dropped), row i into running sum i mod 4; then the 4 R sums of a
// component are added in a fixed order through sh (64 doubles of the wavefront).  Every
// lane returns its component's total (lanes past R DP return component 0's).
template <int DP>
__device__ __forceinline__ double wave_rows(const double *__restrict__ rows, int64_t a, int64_t b, double *sh) {
    constexpr int R = 64 / DP;
    const int lane = threadIdx.x & 63;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (lane < R * DP) {
        const int r0 = lane / DP, k = lane - r0 * DP;
        for (int64_t j = a + r0; j < b; j += 8 * R) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t jj = j + u * R;
                v[u] = rows[(jj < b ? jj : a) * DP + k];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (j + u * R < b) s[u & 3] += v[u];
        }
    }
    sh[lane] = (s[0] + s[1]) + (s[2] + s[3]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int k = lane < R * DP ? lane % DP : 0;
    double t = 0.0;
    for (int m = 0; m < R; ++m) t += sh[k + DP * m];
    return t;
}

// y_c = lambda diag(U_c) v_c + sum of the partial rows of camera c, which are
// contiguous (camera-major); one wavefront per camera (wave_rows).  With gram, block b
// also leaves gram[2 b] = sum of y_c . v_c and gram[2 b + 1] = sum of v_c . gr_c over its
// four cameras (the Gram products Q^T P and P^T r of a one-column block, Q = S P).
// The skip flag, the camera's row range and its entries of v, diag(U) and gr are
// requested together, before anything waits on one of them (a wavefront past the last
// camera reads the last camera's and drops them).
template <int DP>
__global__ __launch_bounds__(256) void k_reduce1(int np, const int32_t *__restrict__ ptr,
                                                 const double *__restrict__ partial,
                                                 const double *__restrict__ dU, const double *__restrict__ v,
                                                 double *__restrict__ y, const double *__restrict__ done,
                                                 const int32_t *__restrict__ cam_seg,
                                                 const int32_t *__restrict__ seg_skip, double *__restrict__ gram,
                                                 const double *__restrict__ gr, float *__restrict__ y32) {
    __shared__ double sh[4][64];
    __shared__ double gsum[2][4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + w;
    const int cl = c < np ? c : np - 1;
    const int64_t i = (int64_t)cl * DP + (lane < DP ? lane : 0);
    const double dn = done ? *done : 0.0;
    const int32_t ra = ptr[cl], rb = ptr[cl + 1];
    const double vi = v[i], du = dU[i];
    const double gi = gram ? gr[i] : 0.0;
    if (dn != 0.0) return;
    double qp = 0.0, pr = 0.0;
    if (c < np && !(seg_skip && seg_skip[cam_seg[c]])) {   // uniform per wavefront
        const double t = wave_rows<DP>(partial, ra, rb, sh[w]);
        if (lane < DP) {
            const double yi = du * vi + t;
            y[i] = yi;
            if (y32) y32[i] = (float)yi;
            if (gram) {
                qp = yi * vi;
                pr = vi * gi;
            }
        }
    }
    if (!gram) return;   // the same for the whole launch
    qp = wave_sum(qp);
    pr = wave_sum(pr);
    if (lane == 0) {
        gsum[0][w] = qp;
        gsum[1][w] = pr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        gram[2 * blockIdx.x] = (gsum[0][0] + gsum[0][1]) + (gsum[0][2] + gsum[0][3]);
        gram[2 * blockIdx.x + 1] = (gsum[1][0] + gsum[1][1]) + (gsum[1][2] + gsum[1][3]);
    }
}

void launch_schur_chunks(const SchurArgs &a, const double *v, hipStream_t s) {
    if (a.n_chunks > 0) {
        // FP64 camera rows (and, for the FP64 product, landmark rows), v in the product precision
        const size_t esz = a.precision == 0 ? sizeof(double) : sizeof(float);
        const size_t lds = (size_t)(a.max_slots * a.dp + (a.precision == 0 ? 3 * kTile : 0)) * sizeof(double) +
                           (size_t)a.max_slots * a.dp * esz;
        const dim3 g(a.n_chunks), b(kTile);
        if (a.dp == 6) {
            switch (a.precision) {
                case 0: hipLaunchKernelGGL((k_schur1<0, double, 6>), g, b, lds, s, a, v); break;
                case 1: hipLaunchKernelGGL((k_schur1<1, float, 6>), g, b, lds, s, a, v); break;
                default: hipLaunchKernelGGL((k_schur1<2, float, 6>), g, b, lds, s, a, v); break;
            }
        } else {
            switch (a.precision) {
                case 0: hipLaunchKernelGGL((k_schur1<0, double, 9>), g, b, lds, s, a, v); break;
                case 1: hipLaunchKernelGGL((k_schur1<1, float, 9>), g, b, lds, s, a, v); break;
                default: hipLaunchKernelGGL((k_schur1<2, float, 9>), g, b, lds, s, a, v); break;
            }
        }
    }
}

int schur_gram_blocks(int np) { return (np + 3) / 4; }

void launch_schur_reduce(const SchurArgs &a, const double *v, double *y, hipStream_t s) {
    const dim3 g((unsigned)schur_gram_blocks(a.np)), b(256);
    if (a.dp == 6)
        hipLaunchKernelGGL(k_reduce1<6>, g, b, 0, s, a.np, a.cam_part_ptr, a.partial, a.dU, v, y, a.done, a.cam_seg,
                           a.seg_skip, a.gram, a.gram_r, a.y32);
    else
        hipLaunchKernelGGL(k_reduce1<9>, g, b, 0, s, a.np, a.cam_part_ptr, a.partial, a.dU, v, y, a.done, a.cam_seg,
                           a.seg_skip, a.gram, a.gram_r, a.y32);
}

void launch_schur_matvec(const SchurArgs &a, const double *v, double *y, hipStream_t s) {
    launch_schur_chunks(a, v, s);
    launch_schur_reduce(a, v, y, s);
}

// ---------------------------------------------------------------- N columns

// Slot words of one lane of a tile for the multidirectional product: the pair word
// (own pair, first pair of the landmark, pair count; kPad on padding slots), the
// camera, the pair's landmark (0xFF past the tile's pairs) and the offset of the
// slot's output indices.
struct MultiSlot {
    uint32_t mm;
    int32_t cam;
    uint32_t pll;
    uint32_t ooff;
};

__device__ __forceinline__ MultiSlot fetch_mslot(const MultiArgs &a, int64_t sidx) {
    MultiSlot m;
    m.mm = a.mmeta[sidx];
    m.cam = a.slot_cam[sidx];
    m.pll = a.pair_ll[sidx];
    m.ooff = a.slot_ooff[sidx];
    return m;
}

// Record, z of the slot's camera, V^-1 of the lane's pair landmark and the slot words
// of one tile (see TileBuf).  Padding slots read camera 0's z and the tile's first
// landmark's V^-1 and ignore them.
template <int PREC, typename T, int DP>
struct MultiBuf {
    TileBuf<PREC, T, DP> r;   // record (r.vi and r.mt unused)
    double z[DP];             // z_c
    dbl2_t vi[3];
    MultiSlot m;
    uint32_t obase;           // tile_oidx of the tile
    int o0, o1;               // output rows of the slot's first two pairs (kept with the tile's loads)
};

// The reduced-precision products sum each pair across its lanes (a pair's observations
// occupy consecutive lanes: a landmark's slots are in camera order and the subsets are
// ranges of consecutive cameras), so every lane takes V^-1 of its own observation's
// landmark; the FP64 product forms h of pair p on lane p, from V^-1 of that pair's landmark.
template <int PREC, typename T, int DP>
__device__ __forceinline__ void fetch_mtile(const MultiArgs &a, const double *__restrict__ z, int t, int lane,
                                            const MultiSlot &m, MultiBuf<PREC, T, DP> &b) {
    b.m = m;
    fetch_record<PREC, T, DP>(a.J, t, lane, b.r);
    const bool valid = m.mm != kPad;
    const double *zc = z + (int64_t)(valid ? m.cam : 0) * DP;
#pragma unroll
    for (int k = 0; k < DP; ++k) b.z[k] = zc[k];
    int ll;
    if constexpr (PREC != 0) {
        const uint32_t mt = a.meta[(int64_t)t * kTile + lane];
        ll = mt != kPad ? (int)((mt >> 16) & 63u) : 0;
    } else {
        ll = m.pll != 0xFFu ? (int)m.pll : 0;
    }
    const dbl2_t *p = reinterpret_cast<const dbl2_t *>(a.vinv + (int64_t)(a.tile_lmk_base[t] + ll) * 6);
#pragma unroll
    for (int q = 0; q < 3; ++q) b.vi[q] = p[q];
    b.obase = a.tile_oidx[t];
    // The first two output rows travel with the tile: a load issued while the tile is
    // processed would wait for every load in flight, the next tile's included.  A padding
    // slot reads the tile's first entry (every tile holds an observation) and ignores it.
    const uint16_t *oi = a.oidx + b.obase + (valid ? m.ooff : 0u);
    const int cnt = valid ? (int)((m.mm >> 16) & 0xFFu) : 1;
    b.o0 = oi[0];
    b.o1 = oi[cnt > 1 ? 1 : 0];
}

// One tile: e = J_p z_c; g per (landmark, subset) pair = sum over the pair's
// observations of J_l^T e; h = V^-1 g; every observation of the landmark adds
// J_p^T (e [own pair] - J_l h_pair) to its (camera, pair subset) row.  With SEG (the
// reduced-precision products) g is a segmented sum across the pair's lanes in registers
// and the pair's last lane publishes h; without, g goes through FP64 LDS atomics and lane
// p forms h of pair p.
template <typename T, int DP, bool SEG>
__device__ __forceinline__ void multi_tile(const MultiArgs &a, const T (&J)[2 * DP + 6], const double (&zb)[DP],
                                           const dbl2_t (&vi)[3], const MultiSlot &m, uint32_t obase, int o0, int o1,
                                           int lane, double *yloc, double *gloc, double *hloc) {
    constexpr int L0 = 2 * DP, L1 = 2 * DP + 3;   // J_l rows 0 and 1
    const bool valid = m.mm != kPad;
    T e0 = 0, e1 = 0;
#pragma unroll
    for (int k = 0; k < DP; ++k) {
        e0 += J[k] * (T)zb[k];
        e1 += J[DP + k] * (T)zb[k];
    }
    const int own = (int)(m.mm & 0xFFu);
    const T w0 = (T)vi[0].x, w1 = (T)vi[0].y, w2 = (T)vi[1].x;
    const T w3 = (T)vi[1].y, w4 = (T)vi[2].x, w5 = (T)vi[2].y;
    if constexpr (SEG) {
        // segments: the pairs (own pair index), padding lanes one each
        const Segs sg = tile_segments(valid ? (uint32_t)own << 16 : kPad, lane);
        double gs[3];   // the pair's total, in its last lane (the only one that uses it)
#pragma unroll
        for (int k = 0; k < 3; ++k) gs[k] = segment_scan(valid ? (double)(J[L0 + k] * e0 + J[L1 + k] * e1) : 0.0, sg);
        if (valid && sg.end == lane) {
            const T g0 = (T)gs[0], g1 = (T)gs[1], g2 = (T)gs[2];
            hloc[own * 3 + 0] = (double)(w0 * g0 + w1 * g1 + w2 * g2);
            hloc[own * 3 + 1] = (double)(w1 * g0 + w3 * g1 + w4 * g2);
            hloc[own * 3 + 2] = (double)(w2 * g0 + w4 * g1 + w5 * g2);
        }
    } else {
        gloc[lane * 3 + 0] = 0;
        gloc[lane * 3 + 1] = 0;
        gloc[lane * 3 + 2] = 0;
        wave_sync();
        if (valid) {
#pragma unroll
            for (int k = 0; k < 3; ++k) atomicAdd(&gloc[own * 3 + k], (double)(J[L0 + k] * e0 + J[L1 + k] * e1));
        }
        wave_sync();
        if (m.pll != 0xFFu) {
            const T g0 = (T)gloc[lane * 3], g1 = (T)gloc[lane * 3 + 1], g2 = (T)gloc[lane * 3 + 2];
            hloc[lane * 3 + 0] = (double)(w0 * g0 + w1 * g1 + w2 * g2);
            hloc[lane * 3 + 1] = (double)(w1 * g0 + w3 * g1 + w4 * g2);
            hloc[lane * 3 + 2] = (double)(w2 * g0 + w4 * g1 + w5 * g2);
        }
    }
    wave_sync();
    if (valid) {
        const int base = (int)((m.mm >> 8) & 0xFFu), cnt = (int)((m.mm >> 16) & 0xFFu);
        auto add_pair = [&](int pj, int o) {
            const T h0 = (T)hloc[pj * 3], h1 = (T)hloc[pj * 3 + 1], h2 = (T)hloc[pj * 3 + 2];
            T f0 = -(J[L0] * h0 + J[L0 + 1] * h1 + J[L0 + 2] * h2);
            T f1 = -(J[L1] * h0 + J[L1 + 1] * h1 + J[L1 + 2] * h2);
            if (pj == own) {
                f0 += e0;
                f1 += e1;
            }
#pragma unroll
            for (int k = 0; k < DP; ++k) atomicAdd(&yloc[o * DP + k], (double)(J[k] * f0 + J[DP + k] * f1));
        };
        add_pair(base, o0);   // cnt >= 1 on a valid slot
        if (cnt > 1) add_pair(base + 1, o1);
        // landmarks spanning three subsets or more: the rest of the rows from memory
        const uint16_t *oi = a.oidx + obase + m.ooff;
        for (int j = 2; j < cnt; ++j) add_pair(base + j, oi[j]);
    }
    wave_sync();
}

template <int PREC, typename T, int DP>
__device__ __forceinline__ void process_mtile(const MultiArgs &a, const MultiBuf<PREC, T, DP> &b, int lane,
                                              double *yloc, double *gloc, double *hloc) {
    if constexpr (PREC == 2) {
        T J[2 * DP + 6];
        Stream<2, DP>::template unpack<T>(b.r.w, J);
        multi_tile<T, DP, true>(a, J, b.z, b.vi, b.m, b.obase, b.o0, b.o1, lane, yloc, gloc, hloc);
    } else {
        multi_tile<T, DP, PREC != 0>(a, b.r.v, b.z, b.vi, b.m, b.obase, b.o0, b.o1, lane, yloc, gloc, hloc);
    }
}

// One wavefront per chunk of tiles, software-pipelined as k_schur1: the record, z
// gather and V^-1 of tile t + 1 and the slot words of tile t + 2 are requested before
// tile t is processed.
template <int PREC, typename T, int DP>
__global__ __launch_bounds__(64) void k_schur_multi(MultiArgs a, const double *__restrict__ z) {
    if (a.skip && *a.skip != 0.0) return;
    if (a.seg_skip && a.seg_skip[a.chunk_seg[blockIdx.x]]) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double *yloc = reinterpret_cast<double *>(smem);   // FP64 sums for every precision (see schur_tile)
    double *gloc = yloc + a.max_out * DP;
    double *hloc = gloc + 3 * kTile;
    const int chunk = blockIdx.x;
    const int lane = threadIdx.x;
    const int pb = a.chunk_part[chunk];
    const int no = a.chunk_part[chunk + 1] - pb;
    const int t0 = a.chunk_tile[chunk], t1 = a.chunk_tile[chunk + 1];
    const int tl = t1 - 1;   // slot words past the chunk's end are read from its last tile
    MultiBuf<PREC, T, DP> A, B;
    MultiSlot mA, mB{};
    if (t0 < t1) {
        fetch_mtile<PREC, T, DP>(a, z, t0, lane, fetch_mslot(a, (int64_t)t0 * kTile + lane), A);
        mB = fetch_mslot(a, (int64_t)min(t0 + 1, tl) * kTile + lane);
    }
    for (int i = lane; i < no * DP; i += kTile) yloc[i] = 0.0;
    wave_sync();
    int t = t0;
    for (; t + 2 < t1; t += 2) {
        fetch_mtile<PREC, T, DP>(a, z, t + 1, lane, mB, B);
        mA = fetch_mslot(a, (int64_t)(t + 2) * kTile + lane);
        process_mtile<PREC, T, DP>(a, A, lane, yloc, gloc, hloc);
        fetch_mtile<PREC, T, DP>(a, z, t + 2, lane, mA, A);
        mB = fetch_mslot(a, (int64_t)min(t + 3, tl) * kTile + lane);
        process_mtile<PREC, T, DP>(a, B, lane, yloc, gloc, hloc);
    }
    if (t + 1 < t1) {
        fetch_mtile<PREC, T, DP>(a, z, t + 1, lane, mB, B);
        process_mtile<PREC, T, DP>(a, A, lane, yloc, gloc, hloc);
        process_mtile<PREC, T, DP>(a, B, lane, yloc, gloc, hloc);
    } else if (t < t1) {
        process_mtile<PREC, T, DP>(a, A, lane, yloc, gloc, hloc);
    }
    for (int i = lane; i < no * DP; i += kTile) {
        const int64_t row = a.part_dst[pb + i / DP];
        a.partial[row * DP + i % DP] = (double)yloc[i];
    }
}

// Y[p][c] = [group(c) == p] lambda diag(U_c) z_c + sum of the partial rows of (c, p),
// which are contiguous ((camera, subset)-major); one wavefront per (c, p) (wave_rows)
template <int DP>
__global__ __launch_bounds__(256) void k_reduce_multi(int np, int N, const int32_t *__restrict__ ptr,
                                                      const double *__restrict__ partial,
                                                      const double *__restrict__ dU,
                                                      const int32_t *__restrict__ group,
                                                      const double *__restrict__ z, double *__restrict__ Y,
                                                      const int32_t *__restrict__ cam_seg,
                                                      const int32_t *__restrict__ seg_skip,
                                                      const double *__restrict__ skip) {
    if (skip && *skip != 0.0) return;
    __shared__ double sh[4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t key = (int64_t)blockIdx.x * 4 + w;   // c * N + p
    if (key >= (int64_t)np * N) return;                 // uniform per wavefront
    const int c = (int)(key / N), p = (int)(key - (int64_t)c * N);
    if (seg_skip && seg_skip[cam_seg[c]]) return;
    const double t = wave_rows<DP>(partial, ptr[key], ptr[key + 1], sh[w]);
    if (lane < DP) {
        const int64_t rem = (int64_t)c * DP + lane;
        Y[(int64_t)p * np * DP + rem] = (group[c] == p ? dU[rem] * z[rem] : 0.0) + t;
    }
}

void launch_schur_multi(const MultiArgs &a, const double *z, double *Y, hipStream_t s) {
    if (a.n_chunks > 0) {
        const size_t lds = (size_t)(a.max_out * a.dp + 6 * kTile) * sizeof(double);
        const dim3 g(a.n_chunks), b(kTile);
        if (a.dp == 6) {
            switch (a.precision) {
                case 0: hipLaunchKernelGGL((k_schur_multi<0, double, 6>), g, b, lds, s, a, z); break;
                case 1: hipLaunchKernelGGL((k_schur_multi<1, float, 6>), g, b, lds, s, a, z); break;
                default: hipLaunchKernelGGL((k_schur_multi<2, float, 6>), g, b, lds, s, a, z); break;
            }
        } else {
            switch (a.precision) {
                case 0: hipLaunchKernelGGL((k_schur_multi<0, double, 9>), g, b, lds, s, a, z); break;
                case 1: hipLaunchKernelGGL((k_schur_multi<1, float, 9>), g, b, lds, s, a, z); break;
                default: hipLaunchKernelGGL((k_schur_multi<2, float, 9>), g, b, lds, s, a, z); break;
            }
        }
    }
    const int64_t keys = (int64_t)a.np * a.N;
    const dim3 g((unsigned)((keys + 3) / 4));
    if (a.dp == 6)
        hipLaunchKernelGGL(k_reduce_multi<6>, g, dim3(256), 0, s, a.np, a.N, a.cg_ptr, a.partial, a.dU, a.group, z, Y,
                           a.cam_seg, a.seg_skip, a.skip);
    else
        hipLaunchKernelGGL(k_reduce_multi<9>, g, dim3(256), 0, s, a.np, a.N, a.cg_ptr, a.partial, a.dU, a.group, z, Y,
                           a.cam_seg, a.seg_skip, a.skip);
}

// ---------------------------------------------------------------- eq. (16)

// dx_l = -V^-1 (b_l + W^T dx_p) for every landmark; the first observation of a
// landmark inside its tile writes the result.
template <int DP>
__global__ __launch_bounds__(64) void k_backsub(const double *__restrict__ J64, const uint32_t *__restrict__ meta,
                                                const int32_t *__restrict__ tile_lmk_base,
                                                const int32_t *__restrict__ chunk_tile,
                                                const int32_t *__restrict__ chunk_part,
                                                const int32_t *__restrict__ part_cam, int max_slots,
                                                const double *__restrict__ vinv, const double *__restrict__ bl,
                                                const int32_t *__restrict__ lmk_order,
                                                const double *__restrict__ dxp, double *__restrict__ dxl) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *vloc = reinterpret_cast<double *>(smem);
    double *gloc = vloc + max_slots * DP;
    const int chunk = blockIdx.x;
    const int lane = threadIdx.x;
    const int pb = chunk_part[chunk];
    const int ns = chunk_part[chunk + 1] - pb;
    for (int i = lane; i < ns * DP; i += kTile) vloc[i] = dxp[(int64_t)part_cam[pb + i / DP] * DP + i % DP];
    __syncthreads();
    for (int t = chunk_tile[chunk]; t < chunk_tile[chunk + 1]; ++t) {
        double J[2 * DP + 6];
        Loader<0, DP>::load(J64, t, lane, J);
        const uint32_t mt = meta[(int64_t)t * kTile + lane];
        const bool valid = mt != kPad;
        const int slot = valid ? (int)(mt & 0xFFFFu) : 0;
        const int ll = valid ? (int)((mt >> 16) & 63u) : 0;
        const uint32_t prev = lane > 0 ? meta[(int64_t)t * kTile + lane - 1] : kPad;
        const bool first = valid && (prev == kPad || ((prev >> 16) & 63u) != (uint32_t)ll);
        double e0 = 0, e1 = 0;
        for (int k = 0; k < DP; ++k) {
            e0 += J[k] * vloc[slot * DP + k];
            e1 += J[DP + k] * vloc[slot * DP + k];
        }
        gloc[lane * 3 + 0] = 0;
        gloc[lane * 3 + 1] = 0;
        gloc[lane * 3 + 2] = 0;
        __syncthreads();
        if (valid)
            for (int k = 0; k < 3; ++k) atomicAdd(&gloc[ll * 3 + k], J[2 * DP + k] * e0 + J[2 * DP + 3 + k] * e1);
        __syncthreads();
        if (first) {
            const int64_t ls = tile_lmk_base[t] + ll;
            const double *vi = vinv + ls * 6;
            const double g0 = gloc[ll * 3] + bl[ls * 3], g1 = gloc[ll * 3 + 1] + bl[ls * 3 + 1],
                         g2 = gloc[ll * 3 + 2] + bl[ls * 3 + 2];
            double *o = dxl + (int64_t)lmk_order[ls] * 3;
            o[0] = -(vi[0] * g0 + vi[1] * g1 + vi[2] * g2);
            o[1] = -(vi[1] * g0 + vi[3] * g1 + vi[4] * g2);
            o[2] = -(vi[2] * g0 + vi[4] * g1 + vi[5] * g2);
        }
        __syncthreads();
    }
}

void launch_back_substitute(const double *J64, const uint32_t *meta, const int32_t *tile_lmk_base,
                            const int32_t *chunk_tile, const int32_t *chunk_part, const int32_t *part_cam,
                            int n_chunks, int max_slots, const double *vinv, const double *bl,
                            const int32_t *lmk_order, const double *dxp, double *dxl, hipStream_t s, int dp) {
    if (n_chunks <= 0) return;
    size_t lds = (size_t)(max_slots * dp + 3 * kTile) * sizeof(double);
    if (dp == 6)
        hipLaunchKernelGGL(k_backsub<6>, dim3(n_chunks), dim3(kTile), lds, s, J64, meta, tile_lmk_base, chunk_tile,
                           chunk_part, part_cam, max_slots, vinv, bl, lmk_order, dxp, dxl);
    else
        hipLaunchKernelGGL(k_backsub<9>, dim3(n_chunks), dim3(kTile), lds, s, J64, meta, tile_lmk_base, chunk_tile,
                           chunk_part, part_cam, max_slots, vinv, bl, lmk_order, dxp, dxl);
}

// Chunk wavefronts of a kernel the device keeps resident at once (register-limited
// occupancy times compute units); 0 when it cannot be queried
static int resident_waves(const void *f) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, kTile, 0) != hipSuccess)
        return 0;
    return per * cus;
}

int schur1_resident_chunks(int dp) {
    return resident_waves(dp == 6 ? reinterpret_cast<const void *>(&k_schur1<0, double, 6>)
                                  : reinterpret_cast<const void *>(&k_schur1<0, double, 9>));
}

int schur_multi_resident_chunks(int dp) {
    return resident_waves(dp == 6 ? reinterpret_cast<const void *>(&k_schur_multi<0, double, 6>)
                                  : reinterpret_cast<const void *>(&k_schur_multi<0, double, 9>));
}

}  // namespace ba
