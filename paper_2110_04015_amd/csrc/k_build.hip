// System build kernels: the damped normal-equation blocks and the reduced
// camera system of Sec. 3.1, eq. (8)-(15), and the block-Jacobi preconditioner
// D(S) of Sec. 3.2 (before Algorithm 1), all in FP64.
#include "ba_internal.h"
#include "kernels.h"

namespace ba {

// ---------------------------------------------------------------- validation

__global__ void k_check_finite(const double *__restrict__ a, int64_t count, int32_t *status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < count; i += stride) bad |= !isfinite(a[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(status, kStatusNonfinite);
}

// ---------------------------------------------------------------- packing

// Record of one observation in the tile stream: J_p rows 0 and 1 (DP values each),
// then J_l rows 0 and 1 (3 each): RecordShape<DP>::kVals values, stored as FP64 pairs,
// FP32 quads or BF16 octets (the last word zero-padded).
template <int DP>
__device__ __forceinline__ void write_record(const double *v, int64_t tile, int lane, double *J64, float *J32,
                                             uint16_t *J16) {
    typedef RecordShape<DP> R;
    if (J64) {
        double2 *d2 = reinterpret_cast<double2 *>(J64);
        for (int q = 0; q < R::kW64; ++q) d2[(tile * R::kW64 + q) * kTile + lane] = make_double2(v[2 * q], v[2 * q + 1]);
    }
    if (J32) {
        float4 *f4 = reinterpret_cast<float4 *>(J32);
        for (int q = 0; q < R::kW32; ++q) {
            float w[4];
            for (int h = 0; h < 4; ++h) w[h] = 4 * q + h < R::kVals ? (float)v[4 * q + h] : 0.0f;
            f4[(tile * R::kW32 + q) * kTile + lane] = make_float4(w[0], w[1], w[2], w[3]);
        }
    }
    if (J16) {
        uint4 *u4 = reinterpret_cast<uint4 *>(J16);
        for (int q = 0; q < R::kW16; ++q) {
            uint32_t w[4];
            for (int h = 0; h < 4; ++h) {
                const int a = 8 * q + 2 * h;
                const uint32_t lo = a < R::kVals ? f32_to_bf16((float)v[a]) : 0u;
                const uint32_t hi = a + 1 < R::kVals ? f32_to_bf16((float)v[a + 1]) : 0u;
                w[h] = lo | (hi << 16);
            }
            u4[(tile * R::kW16 + q) * kTile + lane] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

// One thread per tile slot: gathers the observation's 2 x DP and 2 x 3 blocks and
// writes them in the component-pair-major tile layout (plus FP32 / BF16 copies).
template <int DP>
__global__ void k_pack(const int64_t *__restrict__ slot_obs, int64_t nslots, const double *__restrict__ Jp,
                       const double *__restrict__ Jl, double *__restrict__ J64, float *__restrict__ J32,
                       uint16_t *__restrict__ J16) {
    constexpr int NV = RecordShape<DP>::kVals;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    int64_t o = slot_obs[s];
    double v[NV];
    if (o >= 0) {
        for (int k = 0; k < 2 * DP; ++k) v[k] = Jp[o * 2 * DP + k];
        for (int k = 0; k < 6; ++k) v[2 * DP + k] = Jl[o * 6 + k];
    } else {
        for (int k = 0; k < NV; ++k) v[k] = 0.0;
    }
    write_record<DP>(v, s / kTile, (int)(s % kTile), J64, J32, J16);
}

// Lower-precision copies of an existing FP64 tile stream (one thread per slot).
template <int DP>
__global__ void k_convert(const double *__restrict__ J64, int64_t nslots, float *__restrict__ J32,
                          uint16_t *__restrict__ J16) {
    typedef RecordShape<DP> R;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    int64_t tile = s / kTile;
    int lane = (int)(s % kTile);
    const double2 *d2 = reinterpret_cast<const double2 *>(J64);
    double v[R::kVals];
    for (int q = 0; q < R::kW64; ++q) {
        double2 d = d2[(tile * R::kW64 + q) * kTile + lane];
        v[2 * q] = d.x;
        v[2 * q + 1] = d.y;
    }
    write_record<DP>(v, tile, lane, nullptr, J32, J16);
}

void launch_convert(const double *J64, int64_t nslots, float *J32, uint16_t *J16, hipStream_t s, int dp) {
    if (nslots <= 0) return;
    const dim3 g((unsigned)((nslots + 255) / 256));
    if (dp == 6) hipLaunchKernelGGL(k_convert<6>, g, dim3(256), 0, s, J64, nslots, J32, J16);
    else hipLaunchKernelGGL(k_convert<9>, g, dim3(256), 0, s, J64, nslots, J32, J16);
}

// ---------------------------------------------------------------- landmarks

// One thread per landmark (storage order): the undamped block J_l^T J_l of eq. (10)
// (symmetric, 6 entries: 00 01 02 11 12 22) and b_l = J_l^T r0 (eq. (12)).  Neither
// depends on lambda, so a new lambda re-uses them.
__global__ void k_landmarks_base(int nl, const int64_t *__restrict__ first_slot, const int32_t *__restrict__ count,
                                 const int64_t *__restrict__ slot_obs, const double *__restrict__ Jl,
                                 const double *__restrict__ r, double *__restrict__ Vraw, double *__restrict__ bl) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nl) return;
    double V[6] = {0, 0, 0, 0, 0, 0};
    double b[3] = {0, 0, 0};
    int64_t f = first_slot[s];
    int c = count[s];
    for (int q = 0; q < c; ++q) {
        int64_t o = slot_obs[f + q];
        const double *j = Jl + o * 6;
        double r0 = r[o * 2], r1 = r[o * 2 + 1];
        V[0] += j[0] * j[0] + j[3] * j[3];
        V[1] += j[0] * j[1] + j[3] * j[4];
        V[2] += j[0] * j[2] + j[3] * j[5];
        V[3] += j[1] * j[1] + j[4] * j[4];
        V[4] += j[1] * j[2] + j[4] * j[5];
        V[5] += j[2] * j[2] + j[5] * j[5];
        b[0] += j[0] * r0 + j[3] * r1;
        b[1] += j[1] * r0 + j[4] * r1;
        b[2] += j[2] * r0 + j[5] * r1;
    }
    for (int k = 0; k < 6; ++k) Vraw[(int64_t)s * 6 + k] = V[k];
    for (int k = 0; k < 3; ++k) bl[(int64_t)s * 3 + k] = b[k];
}

// One thread per landmark: V_lambda = V + lambda diag(V) (eq. (10) with Marquardt
// damping), V_lambda^-1 (symmetric, 6 entries) by its 3x3 Cholesky factor, and
// h0 = V_lambda^-1 b_l.
__global__ void k_landmarks_lambda(int nl, const double *__restrict__ Vraw, const double *__restrict__ bl,
                                   double lambda, double *__restrict__ vinv, double *__restrict__ h0,
                                   int32_t *status) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nl) return;
    double V[6], b[3];
    for (int k = 0; k < 6; ++k) V[k] = Vraw[(int64_t)s * 6 + k];
    for (int k = 0; k < 3; ++k) b[k] = bl[(int64_t)s * 3 + k];
    V[0] += lambda * V[0];
    V[3] += lambda * V[3];
    V[5] += lambda * V[5];
    // 3x3 Cholesky V = L L^T
    double l00 = V[0];
    bool ok = l00 > 0.0;
    l00 = sqrt(ok ? l00 : 1.0);
    double l10 = V[1] / l00, l20 = V[2] / l00;
    double l11 = V[3] - l10 * l10;
    ok = ok && l11 > 0.0;
    l11 = sqrt(ok ? l11 : 1.0);
    double l21 = (V[4] - l20 * l10) / l11;
    double l22 = V[5] - l20 * l20 - l21 * l21;
    ok = ok && l22 > 0.0;
    l22 = sqrt(ok ? l22 : 1.0);
    if (!ok) atomicOr(status, kStatusNotSpdLandmark);
    // L^-1 (lower), then V^-1 = L^-T L^-1
    double i00 = 1.0 / l00, i11 = 1.0 / l11, i22 = 1.0 / l22;
    double i10 = -l10 * i00 * i11;
    double i21 = -l21 * i11 * i22;
    double i20 = -(l20 * i00 + l21 * i10) * i22;
    double w[6];
    w[0] = i00 * i00 + i10 * i10 + i20 * i20;
    w[1] = i11 * i10 + i21 * i20;
    w[2] = i22 * i20;
    w[3] = i11 * i11 + i21 * i21;
    w[4] = i22 * i21;
    w[5] = i22 * i22;
    for (int k = 0; k < 6; ++k) vinv[(int64_t)s * 6 + k] = w[k];
    h0[(int64_t)s * 3 + 0] = w[0] * b[0] + w[1] * b[1] + w[2] * b[2];
    h0[(int64_t)s * 3 + 1] = w[1] * b[0] + w[3] * b[1] + w[4] * b[2];
    h0[(int64_t)s * 3 + 2] = w[2] * b[0] + w[4] * b[1] + w[5] * b[2];
}

// ---------------------------------------------------------------- cameras

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wavefront per camera: the undamped block U = J_p^T J_p (eq. (9), packed upper
// triangle) and b_p = J_p^T r0 (eq. (11)) over the camera's observations.  Neither
// depends on lambda.  DP x DP blocks (DP = 9, or 6 for extrinsics only).
template <int DP>
__global__ __launch_bounds__(64) void k_cameras_base(int np, const int64_t *__restrict__ cam_ptr,
                                                     const int64_t *__restrict__ cam_obs,
                                                     const double *__restrict__ Jp, const double *__restrict__ r,
                                                     double *__restrict__ Uraw, double *__restrict__ bp) {
    constexpr int T = DP * (DP + 1) / 2;   // packed upper triangle
    constexpr int NA = T + DP;
    int c = blockIdx.x;
    int lane = threadIdx.x;
    if (c >= np) return;
    int64_t a = cam_ptr[c], b = cam_ptr[c + 1];
    double acc[NA];
    for (int k = 0; k < NA; ++k) acc[k] = 0.0;
    for (int64_t q = a + lane; q < b; q += 64) {
        int64_t o = cam_obs[q];
        const double *j = Jp + o * 2 * DP;
        double r0 = r[o * 2], r1 = r[o * 2 + 1];
        int t = 0;
        for (int i = 0; i < DP; ++i)
            for (int k = i; k < DP; ++k) acc[t++] += j[i] * j[k] + j[DP + i] * j[DP + k];
        for (int i = 0; i < DP; ++i) acc[T + i] += j[i] * r0 + j[DP + i] * r1;
    }
    for (int k = 0; k < NA; ++k) {
        double v = wave_sum(acc[k]);
        if (lane == 0) {
            if (k < T) Uraw[(int64_t)c * T + k] = v;
            else bp[(int64_t)c * DP + (k - T)] = v;
        }
    }
}

// One wavefront per camera, for the current lambda: E = sum_o W_o V_lambda^-1 W_o^T and
// w = sum_o W_o h0 with W_o = J_p,o^T J_l,o read back from the packed tile stream (the
// observation's slot from obs_slot), then
//   D(S)_c = U + lambda diag(U) - E   (diagonal block of eq. (14))
//   b~_c   = b_p - w                  (eq. (15))
// the damping lambda diag(U) of the S product, and the Cholesky factor of D(S)_c.
template <int DP>
__global__ __launch_bounds__(64) void k_cameras_lambda(int np, const int64_t *__restrict__ cam_ptr,
                                                       const int64_t *__restrict__ cam_obs,
                                                       const int32_t *__restrict__ obs_lm,
                                                       const int32_t *__restrict__ lmk_store,
                                                       const int64_t *__restrict__ obs_slot,
                                                       const double *__restrict__ J64,
                                                       const double *__restrict__ Uraw, const double *__restrict__ bpv,
                                                       const double *__restrict__ vinv,
                                                       const double *__restrict__ h0, double lambda,
                                                       double *__restrict__ dU, double *__restrict__ Dblk,
                                                       double *__restrict__ Dchol, double *__restrict__ bt,
                                                       int32_t *status) {
    typedef RecordShape<DP> R;
    constexpr int T = DP * (DP + 1) / 2;
    constexpr int NA = T + DP;
    int c = blockIdx.x;
    int lane = threadIdx.x;
    if (c >= np) return;
    __shared__ double red[NA];
    int64_t a = cam_ptr[c], b = cam_ptr[c + 1];
    const double2 *d2 = reinterpret_cast<const double2 *>(J64);
    double acc[NA];
    for (int k = 0; k < NA; ++k) acc[k] = 0.0;
    for (int64_t q = a + lane; q < b; q += 64) {
        int64_t o = cam_obs[q];
        const int64_t sl = obs_slot[o];
        const int64_t tile = sl / kTile;
        const int sl_lane = (int)(sl % kTile);
        double v[2 * R::kW64];
        for (int w = 0; w < R::kW64; ++w) {
            const double2 d = d2[(tile * R::kW64 + w) * kTile + sl_lane];
            v[2 * w] = d.x;
            v[2 * w + 1] = d.y;
        }
        const double *jp = v, *jl = v + 2 * DP;
        int64_t ls = lmk_store[obs_lm[o]];
        const double *vi = vinv + ls * 6;
        const double *hh = h0 + ls * 3;
        double W[DP * 3];
        for (int i = 0; i < DP; ++i)
            for (int k = 0; k < 3; ++k) W[i * 3 + k] = jp[i] * jl[k] + jp[DP + i] * jl[3 + k];
        double VW[DP * 3];   // (V^-1 W^T)^T = W V^-1, rows i
        for (int i = 0; i < DP; ++i) {
            double w0 = W[i * 3], w1 = W[i * 3 + 1], w2 = W[i * 3 + 2];
            VW[i * 3 + 0] = w0 * vi[0] + w1 * vi[1] + w2 * vi[2];
            VW[i * 3 + 1] = w0 * vi[1] + w1 * vi[3] + w2 * vi[4];
            VW[i * 3 + 2] = w0 * vi[2] + w1 * vi[4] + w2 * vi[5];
        }
        int t = 0;
        for (int i = 0; i < DP; ++i)
            for (int k = i; k < DP; ++k)
                acc[t++] += VW[i * 3] * W[k * 3] + VW[i * 3 + 1] * W[k * 3 + 1] + VW[i * 3 + 2] * W[k * 3 + 2];
        for (int i = 0; i < DP; ++i) acc[T + i] += W[i * 3] * hh[0] + W[i * 3 + 1] * hh[1] + W[i * 3 + 2] * hh[2];
    }
    for (int k = 0; k < NA; ++k) {
        double v = wave_sum(acc[k]);
        if (lane == 0) red[k] = v;
    }
    __syncthreads();
    if (lane != 0) return;
    const double *U = Uraw + (int64_t)c * T;
    double D[DP * DP];
    int t = 0;
    for (int i = 0; i < DP; ++i) {
        for (int k = i; k < DP; ++k, ++t) {
            double u = U[t];
            if (k == i) u += lambda * U[t];
            double d = u - red[t];
            D[i * DP + k] = d;
            D[k * DP + i] = d;
        }
    }
    for (int i = 0; i < DP; ++i) {
        int diag = i * DP - (i * (i - 1)) / 2;   // index of (i, i) in the packed upper triangle
        dU[(int64_t)c * DP + i] = lambda * U[diag];
        bt[(int64_t)c * DP + i] = bpv[(int64_t)c * DP + i] - red[T + i];
    }
    for (int k = 0; k < DP * DP; ++k) Dblk[(int64_t)c * DP * DP + k] = D[k];
    // packed lower Cholesky factor, row i holds L[i][0..i]
    double L[T];
    bool ok = true;
    for (int j = 0; j < DP; ++j) {
        double d = D[j * DP + j];
        for (int p = 0; p < j; ++p) d -= L[j * (j + 1) / 2 + p] * L[j * (j + 1) / 2 + p];
        if (!(d > 0.0)) {
            ok = false;
            d = 1.0;
        }
        d = sqrt(d);
        L[j * (j + 1) / 2 + j] = d;
        for (int i = j + 1; i < DP; ++i) {
            double s = D[i * DP + j];
            for (int p = 0; p < j; ++p) s -= L[i * (i + 1) / 2 + p] * L[j * (j + 1) / 2 + p];
            L[i * (i + 1) / 2 + j] = s / d;
        }
    }
    if (!ok) atomicOr(status, kStatusNotSpdCamera);
    for (int k = 0; k < T; ++k) Dchol[(int64_t)c * T + k] = L[k];
}

// ---------------------------------------------------------------- launchers

void launch_check_finite(const double *a, int64_t count, int32_t *status, hipStream_t s) {
    if (count <= 0) return;
    int blocks = (int)std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_check_finite, dim3(blocks), dim3(256), 0, s, a, count, status);
}

void launch_pack(const int64_t *slot_obs, int64_t nslots, const double *Jp, const double *Jl, double *J64,
                 float *J32, uint16_t *J16, hipStream_t s, int dp) {
    const dim3 g((unsigned)((nslots + 255) / 256));
    if (dp == 6) hipLaunchKernelGGL(k_pack<6>, g, dim3(256), 0, s, slot_obs, nslots, Jp, Jl, J64, J32, J16);
    else hipLaunchKernelGGL(k_pack<9>, g, dim3(256), 0, s, slot_obs, nslots, Jp, Jl, J64, J32, J16);
}

void launch_landmarks_base(int nl, const int64_t *first_slot, const int32_t *count, const int64_t *slot_obs,
                           const double *Jl, const double *r, double *Vraw, double *bl, hipStream_t s) {
    hipLaunchKernelGGL(k_landmarks_base, dim3((nl + 255) / 256), dim3(256), 0, s, nl, first_slot, count, slot_obs, Jl,
                       r, Vraw, bl);
}

void launch_landmarks_lambda(int nl, const double *Vraw, const double *bl, double lambda, double *vinv, double *h0,
                             int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(k_landmarks_lambda, dim3((nl + 255) / 256), dim3(256), 0, s, nl, Vraw, bl, lambda, vinv, h0,
                       status);
}

void launch_cameras_base(int np, const int64_t *cam_ptr, const int64_t *cam_obs, const double *Jp, const double *r,
                         double *Uraw, double *bp, hipStream_t s, int dp) {
    if (dp == 6)
        hipLaunchKernelGGL(k_cameras_base<6>, dim3(np), dim3(64), 0, s, np, cam_ptr, cam_obs, Jp, r, Uraw, bp);
    else
        hipLaunchKernelGGL(k_cameras_base<9>, dim3(np), dim3(64), 0, s, np, cam_ptr, cam_obs, Jp, r, Uraw, bp);
}

void launch_cameras_lambda(int np, const int64_t *cam_ptr, const int64_t *cam_obs, const int32_t *obs_lm,
                           const int32_t *lmk_store, const int64_t *obs_slot, const double *J64, const double *Uraw,
                           const double *bp, const double *vinv, const double *h0, double lambda, double *dU,
                           double *Dblk, double *Dchol, double *bt, int32_t *status, hipStream_t s, int dp) {
    if (dp == 6)
        hipLaunchKernelGGL(k_cameras_lambda<6>, dim3(np), dim3(64), 0, s, np, cam_ptr, cam_obs, obs_lm, lmk_store,
                           obs_slot, J64, Uraw, bp, vinv, h0, lambda, dU, Dblk, Dchol, bt, status);
    else
        hipLaunchKernelGGL(k_cameras_lambda<9>, dim3(np), dim3(64), 0, s, np, cam_ptr, cam_obs, obs_lm, lmk_store,
                           obs_slot, J64, Uraw, bp, vinv, h0, lambda, dU, Dblk, Dchol, bt, status);
}

}  // namespace ba
