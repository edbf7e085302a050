// Kernels of the Levenberg-Marquardt outer loop (Sec. 4.1) for the nine-parameter
// camera (Sec. 3.1 with d_p = 9: rotation, translation, focal length, two radial
// distortion coefficients).
//
// Camera c is 15 doubles: R row-major (9), t (3), f, k1, k2.  Landmark l is X_l (3).
//   P = R X + t,  p = P_xy / P_z,  rho2 = |p|^2,  s = 1 + k1 rho2 + k2 rho2^2,  u = f s p,
//   r_o = u - u_obs[o];  F = sum_o |r_o|^2 (eq. (1)).
// The 9 step coordinates of a camera are a left rigid motion (w, dt), then df, dk1,
// dk2: R <- exp([w]x) R, t <- exp([w]x) t + dt.  With A = du/dP,
//   dr/dw = -A [P]x,  dr/dt = A,  dr/df = s p,  dr/dk1 = f rho2 p,  dr/dk2 = f rho2^2 p,
//   dr/dX = A R.
#include "ba_internal.h"
#include "kernels.h"
#include "dev_la.h"

namespace ba {

constexpr int kLmThreads = 256;

// One thread per observation.  Writes r (and, when Jp is set, the Jacobian blocks in
// the [m][2][9] / [m][2][3] layout of ba_problem_desc); the block's sum of |r_o|^2 goes
// to partials[blockIdx.x] (wavefront butterflies, then the wavefronts in order).
__global__ __launch_bounds__(kLmThreads) void k_project(int64_t m, const int32_t *__restrict__ obs_cam,
                                                        const int32_t *__restrict__ obs_lm,
                                                        const double *__restrict__ cams,
                                                        const double *__restrict__ X,
                                                        const double *__restrict__ u_obs, double *__restrict__ Jp,
                                                        double *__restrict__ Jl, double *__restrict__ r,
                                                        double *__restrict__ partials) {
    __shared__ double wsum[kLmThreads / 64];
    const int64_t o = (int64_t)blockIdx.x * kLmThreads + threadIdx.x;
    double sq = 0.0;
    if (o < m) {
        const double *cm = cams + (int64_t)obs_cam[o] * 15;
        const double *xl = X + (int64_t)obs_lm[o] * 3;
        double R[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) R[i] = cm[i];
        const double X0 = xl[0], X1 = xl[1], X2 = xl[2];
        const double Px = R[0] * X0 + R[1] * X1 + R[2] * X2 + cm[9];
        const double Py = R[3] * X0 + R[4] * X1 + R[5] * X2 + cm[10];
        const double Pz = R[6] * X0 + R[7] * X1 + R[8] * X2 + cm[11];
        const double f = cm[12], k1 = cm[13], k2 = cm[14];
        const double iz = 1.0 / Pz;
        const double px = Px * iz, py = Py * iz;
        const double rho2 = px * px + py * py;
        const double s = 1.0 + k1 * rho2 + k2 * rho2 * rho2;
        const double r0 = f * s * px - u_obs[2 * o];
        const double r1 = f * s * py - u_obs[2 * o + 1];
        sq = r0 * r0 + r1 * r1;
        if (r) {
            r[2 * o] = r0;
            r[2 * o + 1] = r1;
        }
        if (Jp) {
            // du/dp = f (s I + g p p^T), g = 2 k1 + 4 k2 rho2; dp/dP = [[iz, 0, -px iz], [0, iz, -py iz]]
            const double g = 2.0 * k1 + 4.0 * k2 * rho2;
            const double a00 = f * (s + g * px * px), a01 = f * g * px * py, a11 = f * (s + g * py * py);
            // A = du/dP (2 x 3)
            const double A[2][3] = {{a00 * iz, a01 * iz, -(a00 * px + a01 * py) * iz},
                                    {a01 * iz, a11 * iz, -(a01 * px + a11 * py) * iz}};
            double *jp = Jp + o * 18;
            double *jl = Jl + o * 6;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                // -A [P]x, [P]x = [[0, -Pz, Py], [Pz, 0, -Px], [-Py, Px, 0]]
                jp[i * 9 + 0] = -(A[i][1] * Pz - A[i][2] * Py);
                jp[i * 9 + 1] = -(-A[i][0] * Pz + A[i][2] * Px);
                jp[i * 9 + 2] = -(A[i][0] * Py - A[i][1] * Px);
                jp[i * 9 + 3] = A[i][0];
                jp[i * 9 + 4] = A[i][1];
                jp[i * 9 + 5] = A[i][2];
                const double pi = i == 0 ? px : py;
                jp[i * 9 + 6] = s * pi;
                jp[i * 9 + 7] = f * rho2 * pi;
                jp[i * 9 + 8] = f * rho2 * rho2 * pi;
#pragma unroll
                for (int c = 0; c < 3; ++c) jl[i * 3 + c] = A[i][0] * R[c] + A[i][1] * R[3 + c] + A[i][2] * R[6 + c];
            }
        }
    }
    sq = wave_sum(sq);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kLmThreads / 64; ++w) t += wsum[w];
        partials[blockIdx.x] = t;
    }
}

// out[0] = sum of nb partials (one wavefront, fixed order)
__global__ __launch_bounds__(64) void k_lm_cost_sum(const double *__restrict__ partials, int nb,
                                                     double *__restrict__ out) {
    const double t = wave_partials(partials, 1, nb);
    if (threadIdx.x == 0) out[0] = t;
}

// exp([w]x) (Rodrigues); Taylor terms below 1e-6 rad
__device__ __forceinline__ void rot_exp(double w0, double w1, double w2, double E[9]) {
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const double th = sqrt(th2);
    double a, b;
    if (th < 1e-6) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
    }
    // K = [w]x, K^2 = w w^T - th2 I
    E[0] = 1.0 + b * (w0 * w0 - th2);
    E[1] = -a * w2 + b * w0 * w1;
    E[2] = a * w1 + b * w0 * w2;
    E[3] = a * w2 + b * w1 * w0;
    E[4] = 1.0 + b * (w1 * w1 - th2);
    E[5] = -a * w0 + b * w1 * w2;
    E[6] = -a * w1 + b * w2 * w0;
    E[7] = a * w0 + b * w2 * w1;
    E[8] = 1.0 + b * (w2 * w2 - th2);
}

// The state moved by (dxp, dxl): thread i < np moves camera i, thread i < nl landmark i.
__global__ __launch_bounds__(kLmThreads) void k_apply_step(int np, int nl, const double *__restrict__ cams,
                                                           const double *__restrict__ X,
                                                           const double *__restrict__ dxp,
                                                           const double *__restrict__ dxl,
                                                           double *__restrict__ cams_out,
                                                           double *__restrict__ X_out) {
    const int64_t i = (int64_t)blockIdx.x * kLmThreads + threadIdx.x;
    if (i < np) {
        const double *c = cams + i * 15;
        const double *d = dxp + i * 9;
        double E[9];
        rot_exp(d[0], d[1], d[2], E);
        double *co = cams_out + i * 15;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int b = 0; b < 3; ++b)
                co[a * 3 + b] = E[a * 3] * c[b] + E[a * 3 + 1] * c[3 + b] + E[a * 3 + 2] * c[6 + b];
            co[9 + a] = E[a * 3] * c[9] + E[a * 3 + 1] * c[10] + E[a * 3 + 2] * c[11] + d[3 + a];
        }
        co[12] = c[12] + d[6];
        co[13] = c[13] + d[7];
        co[14] = c[14] + d[8];
    }
    if (i < nl) {
#pragma unroll
        for (int a = 0; a < 3; ++a) X_out[i * 3 + a] = X[i * 3 + a] + dxl[i * 3 + a];
    }
}

int project_blocks(int64_t m) { return (int)((m + kLmThreads - 1) / kLmThreads); }

void launch_project(int64_t m, const int32_t *obs_cam, const int32_t *obs_lm, const double *cams, const double *X,
                    const double *u_obs, double *Jp, double *Jl, double *r, double *partials, double *cost,
                    hipStream_t s) {
    const int nb = project_blocks(m);
    hipLaunchKernelGGL(k_project, dim3(nb), dim3(kLmThreads), 0, s, m, obs_cam, obs_lm, cams, X, u_obs, Jp, Jl, r,
                       partials);
    hipLaunchKernelGGL(k_lm_cost_sum, dim3(1), dim3(64), 0, s, partials, nb, cost);
}

void launch_apply_step(int np, int nl, const double *cams, const double *X, const double *dxp, const double *dxl,
                       double *cams_out, double *X_out, hipStream_t s) {
    const int64_t n = std::max<int64_t>(np, nl);
    hipLaunchKernelGGL(k_apply_step, dim3((unsigned)((n + kLmThreads - 1) / kLmThreads)), dim3(kLmThreads), 0, s,
                       np, nl, cams, X, dxp, dxl, cams_out, X_out);
}

}  // namespace ba
