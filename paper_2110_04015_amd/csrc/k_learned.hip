// Learned low-rank correction of the block-Jacobi preconditioner (an addition to
// the paper's block Jacobi D(S) of Sec. 3.2):
//     M^-1 = D(S)^-1 + U U^T,  U = [U_1; ...; U_np] (n x 8),  U_c = L_c^-T Uh_c,
// with D(S)_c = L_c L_c^T and Uh_c (9 x 8) the output of a 2-layer MLP
// (47 -> 128 tanh -> 72) applied to 47 scale-free features of camera c.
// M^-1 is symmetric positive definite for any weights.
//
// Parameters (FP32, 15,432): W1 [128][47], b1 [128], W2 [72][128], b2 [72].
// Inference runs in BF16 on the matrix cores (FP32 accumulation); training
// (forward with stored activations, backward, Adam) runs in FP32.
#include "ba_internal.h"
#include "kernels.h"

namespace ba {

constexpr int kFeat = 47, kHid = 128, kOut = 72, kRank = 8;
constexpr int kOffB1 = kHid * kFeat, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kOut * kHid;
constexpr int kParams = kOffB2 + kOut;   // 15432
constexpr int kNTL = 256;

// ---------------------------------------------------------------- features

// 36 correlations D_ij / sqrt(D_ii D_jj) (i < j, row-major), 9 log D_ii - mean log D,
// log(1 + covisibility degree), log(max(lambda, 1e-12)).
__global__ void k_features(int np, const double *__restrict__ Dblk, const int32_t *__restrict__ deg, double lambda,
                           float *__restrict__ F) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= np) return;
    const double *D = Dblk + (int64_t)c * 81;
    double d[9], ld[9], mean = 0.0;
    for (int i = 0; i < 9; ++i) {
        d[i] = D[i * 9 + i];
        ld[i] = log(d[i]);
        mean += ld[i];
    }
    mean /= 9.0;
    float *f = F + (int64_t)c * kFeat;
    int t = 0;
    for (int i = 0; i < 9; ++i)
        for (int j = i + 1; j < 9; ++j) f[t++] = (float)(D[i * 9 + j] / sqrt(d[i] * d[j]));
    for (int i = 0; i < 9; ++i) f[36 + i] = (float)(ld[i] - mean);
    f[45] = (float)log1p((double)deg[c]);
    f[46] = (float)log(lambda > 1e-12 ? lambda : 1e-12);
}

void launch_features(int np, const double *Dblk, const int32_t *deg, double lambda, float *F, hipStream_t s) {
    hipLaunchKernelGGL(k_features, dim3((np + 127) / 128), dim3(128), 0, s, np, Dblk, deg, lambda, F);
}

// ---------------------------------------------------------------- FP32 forward / backward

__global__ void k_mlp_hidden(const float *__restrict__ P, const float *__restrict__ F, int rows,
                             float *__restrict__ hid) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * kHid) return;
    const int row = (int)(idx / kHid), j = (int)(idx % kHid);
    float s = P[kOffB1 + j];
    const float *w = P + j * kFeat, *f = F + (int64_t)row * kFeat;
    for (int k = 0; k < kFeat; ++k) s += w[k] * f[k];
    hid[idx] = tanhf(s);
}

__global__ void k_mlp_out(const float *__restrict__ P, const float *__restrict__ hid, int rows, float *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * kOut) return;
    const int row = (int)(idx / kOut), o = (int)(idx % kOut);
    float s = P[kOffB2 + o];
    const float *w = P + kOffW2 + o * kHid, *h = hid + (int64_t)row * kHid;
    for (int j = 0; j < kHid; ++j) s += w[j] * h[j];
    out[idx] = s;
}

// g_pre = (g_out W2) * (1 - hid^2)
__global__ void k_mlp_bwd_hidden(const float *__restrict__ P, const float *__restrict__ g_out,
                                 const float *__restrict__ hid, int rows, float *__restrict__ g_pre) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * kHid) return;
    const int row = (int)(idx / kHid), j = (int)(idx % kHid);
    float s = 0.f;
    const float *g = g_out + (int64_t)row * kOut;
    for (int o = 0; o < kOut; ++o) s += g[o] * P[kOffW2 + o * kHid + j];
    const float h = hid[idx];
    g_pre[idx] = s * (1.f - h * h);
}

// one thread per parameter, rows summed in order
__global__ void k_mlp_grad_params(const float *__restrict__ F, const float *__restrict__ hid,
                                  const float *__restrict__ g_out, const float *__restrict__ g_pre, int rows,
                                  float *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    float s = 0.f;
    if (p < kOffB1) {
        const int j = p / kFeat, k = p % kFeat;
        for (int r = 0; r < rows; ++r) s += g_pre[(int64_t)r * kHid + j] * F[(int64_t)r * kFeat + k];
    } else if (p < kOffW2) {
        const int j = p - kOffB1;
        for (int r = 0; r < rows; ++r) s += g_pre[(int64_t)r * kHid + j];
    } else if (p < kOffB2) {
        const int o = (p - kOffW2) / kHid, j = (p - kOffW2) % kHid;
        for (int r = 0; r < rows; ++r) s += g_out[(int64_t)r * kOut + o] * hid[(int64_t)r * kHid + j];
    } else {
        const int o = p - kOffB2;
        for (int r = 0; r < rows; ++r) s += g_out[(int64_t)r * kOut + o];
    }
    grad[p] = s;
}

// ---------------------------------------------------------------- BF16 inference on the matrix cores

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16s(float f) { return (short)f32_to_bf16(f); }

// One wavefront per 16 rows.  v_mfma_f32_16x16x16_bf16 operand layout (wave64):
// A[i][k]: lane i + 16 (k / 4), element k % 4; B[k][j]: lane j + 16 (k / 4), element
// k % 4; D[i][j]: lane j + 16 (i / 4), element i % 4.
__global__ __launch_bounds__(64) void k_mlp_fwd_bf16(const float *__restrict__ P, const float *__restrict__ F,
                                                     int rows, float *__restrict__ out) {
    __shared__ short hs[16][kHid + 4];
    const int lane = threadIdx.x;
    const int i = lane & 15, q = lane >> 4;
    const int r0 = blockIdx.x * 16;
    // layer 1: [16 x 48] x [48 x 128], K padded 47 -> 48
    for (int jb = 0; jb < kHid / 16; ++jb) {
        f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
        for (int kb = 0; kb < 3; ++kb) {
            bf16x4_t a, b;
            for (int e = 0; e < 4; ++e) {
                const int k = kb * 16 + 4 * q + e;
                const int row = r0 + i;
                a[e] = bf16s(k < kFeat && row < rows ? F[(int64_t)row * kFeat + k] : 0.f);
                b[e] = bf16s(k < kFeat ? P[(jb * 16 + i) * kFeat + k] : 0.f);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        const float bias = P[kOffB1 + jb * 16 + i];
        for (int e = 0; e < 4; ++e) hs[4 * q + e][jb * 16 + i] = bf16s(tanhf(acc[e] + bias));
    }
    __syncthreads();
    // layer 2: [16 x 128] x [128 x 80], outputs padded 72 -> 80
    for (int ob = 0; ob < 5; ++ob) {
        f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
        const int o = ob * 16 + i;
        for (int kb = 0; kb < kHid / 16; ++kb) {
            bf16x4_t a, b;
            for (int e = 0; e < 4; ++e) {
                const int k = kb * 16 + 4 * q + e;
                a[e] = hs[i][k];
                b[e] = bf16s(o < kOut ? P[kOffW2 + o * kHid + k] : 0.f);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        if (o < kOut) {
            const float bias = P[kOffB2 + o];
            for (int e = 0; e < 4; ++e) {
                const int row = r0 + 4 * q + e;
                if (row < rows) out[(int64_t)row * kOut + o] = acc[e] + bias;
            }
        }
    }
}

void launch_mlp_forward(const float *P, const float *F, int rows, float *out, float *hid, int bf16, hipStream_t s) {
    if (bf16) {
        hipLaunchKernelGGL(k_mlp_fwd_bf16, dim3((rows + 15) / 16), dim3(64), 0, s, P, F, rows, out);
        return;
    }
    const int64_t nh = (int64_t)rows * kHid, no = (int64_t)rows * kOut;
    hipLaunchKernelGGL(k_mlp_hidden, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, s, P, F, rows, hid);
    hipLaunchKernelGGL(k_mlp_out, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, s, P, hid, rows, out);
}

// ---------------------------------------------------------------- U = L^-T Uh

__global__ void k_lowrank_U(int np, const double *__restrict__ Dchol, const float *__restrict__ out,
                            double *__restrict__ U) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= np) return;
    const double *L = Dchol + (int64_t)c * 45;   // packed lower, row i holds L[i][0..i]
    for (int a = 0; a < kRank; ++a) {
        double y[9];
        for (int i = 8; i >= 0; --i) {
            double s = (double)out[(int64_t)c * kOut + i * kRank + a];
            for (int p = i + 1; p < 9; ++p) s -= L[p * (p + 1) / 2 + i] * y[p];
            y[i] = s / L[i * (i + 1) / 2 + i];
        }
        for (int i = 0; i < 9; ++i) U[((int64_t)c * 9 + i) * kRank + a] = y[i];
    }
}

void launch_lowrank_U(int np, const double *Dchol, const float *out, double *U, hipStream_t s) {
    hipLaunchKernelGGL(k_lowrank_U, dim3((np + 127) / 128), dim3(128), 0, s, np, Dchol, out, U);
}

// y = L^-1 x (transpose 0) or L^-T x (transpose 1), block by block
__global__ void k_block_scale(int np, const double *__restrict__ Dchol, const double *__restrict__ x,
                              double *__restrict__ y, int transpose) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= np) return;
    const double *L = Dchol + (int64_t)c * 45;
    double v[9];
    for (int i = 0; i < 9; ++i) v[i] = x[(int64_t)c * 9 + i];
    if (!transpose) {
        for (int i = 0; i < 9; ++i) {
            double s = v[i];
            for (int p = 0; p < i; ++p) s -= L[i * (i + 1) / 2 + p] * v[p];
            v[i] = s / L[i * (i + 1) / 2 + i];
        }
    } else {
        for (int i = 8; i >= 0; --i) {
            double s = v[i];
            for (int p = i + 1; p < 9; ++p) s -= L[p * (p + 1) / 2 + i] * v[p];
            v[i] = s / L[i * (i + 1) / 2 + i];
        }
    }
    for (int i = 0; i < 9; ++i) y[(int64_t)c * 9 + i] = v[i];
}

void launch_block_scale(int np, const double *Dchol, const double *x, double *y, int transpose, hipStream_t s) {
    hipLaunchKernelGGL(k_block_scale, dim3((np + 127) / 128), dim3(128), 0, s, np, Dchol, x, y, transpose);
}

// ---------------------------------------------------------------- M^-1 r = D^-1 r + U (U^T r)

__device__ __forceinline__ double block_sum_l(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kNTL / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// partials[b][a] = sum over the block's rows of U[i][a] r[i]
__global__ __launch_bounds__(kNTL) void k_lr_proj(int64_t n, const double *__restrict__ U, const double *__restrict__ r,
                                                  double *__restrict__ partials, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    __shared__ double sh[kNTL];
    double acc[kRank];
    for (int a = 0; a < kRank; ++a) acc[a] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNTL + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNTL) {
        const double ri = r[i];
        for (int a = 0; a < kRank; ++a) acc[a] += U[i * kRank + a] * ri;
    }
    for (int a = 0; a < kRank; ++a) {
        const double s = block_sum_l(acc[a], sh);
        if (threadIdx.x == 0) partials[blockIdx.x * kRank + a] = s;
    }
}

// z += U t with t = sum of the projections (every block re-adds them in block order);
// partial sums of sum_i a2[i] z[i]
__global__ __launch_bounds__(kNTL) void k_lr_add_dot(int64_t n, const double *__restrict__ U,
                                                     const double *__restrict__ pproj, double *__restrict__ z,
                                                     const double *__restrict__ a2, double *__restrict__ partials,
                                                     const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    __shared__ double sh[kNTL];
    __shared__ double t[kRank];
    if (threadIdx.x < kRank) {
        double s = 0.0;
        for (int b = 0; b < kRedBlocks; ++b) s += pproj[b * kRank + threadIdx.x];
        t[threadIdx.x] = s;
    }
    __syncthreads();
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNTL + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNTL) {
        double s = 0.0;
        for (int a = 0; a < kRank; ++a) s += U[i * kRank + a] * t[a];
        const double zi = z[i] + s;
        z[i] = zi;
        if (a2) acc += a2[i] * zi;
    }
    if (partials) {
        acc = block_sum_l(acc, sh);
        if (threadIdx.x == 0) partials[blockIdx.x] = acc;
    }
}

void launch_lowrank_apply(int64_t n, const double *U, const double *r, double *z, const double *a2, double *pproj,
                          double *partials, const double *done, hipStream_t s) {
    hipLaunchKernelGGL(k_lr_proj, dim3(kRedBlocks), dim3(kNTL), 0, s, n, U, r, pproj, done);
    hipLaunchKernelGGL(k_lr_add_dot, dim3(kRedBlocks), dim3(kNTL), 0, s, n, U, pproj, z, a2, partials, done);
}

// ---------------------------------------------------------------- probe loss and its gradient

// loss = 1/(P n) sum_k |w_k - s_k - Uh (Uh^T s_k)|^2 over P <= 8 probes (columns k of the
// n x P row-major arrays W and Sw); Uh = out viewed as n x 8.
constexpr int kMaxProbes = 8;

__global__ __launch_bounds__(kNTL) void k_probe_T(int64_t n, int Pn, const float *__restrict__ Uh,
                                                  const double *__restrict__ Sw, double *__restrict__ partials) {
    __shared__ double sh[kNTL];
    double acc[kRank * kMaxProbes];
    for (int e = 0; e < kRank * kMaxProbes; ++e) acc[e] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNTL + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNTL) {
        for (int a = 0; a < kRank; ++a) {
            const double u = (double)Uh[i * kRank + a];
            for (int k = 0; k < kMaxProbes; ++k)
                if (k < Pn) acc[a * kMaxProbes + k] += u * Sw[i * Pn + k];
        }
    }
    for (int e = 0; e < kRank * kMaxProbes; ++e) {
        const double s = block_sum_l(acc[e], sh);
        if (threadIdx.x == 0) partials[blockIdx.x * kRank * kMaxProbes + e] = s;
    }
}

__global__ void k_sum_partials(const double *__restrict__ partials, int nd, double *__restrict__ out) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= nd) return;
    double s = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) s += partials[b * nd + d];
    out[d] = s;
}

// per-row residual E, partial sums of |E|^2 and of E^T Uh (P x 8)
__global__ __launch_bounds__(kNTL) void k_probe_E(int64_t n, int Pn, const float *__restrict__ Uh,
                                                  const double *__restrict__ W, const double *__restrict__ Sw,
                                                  const double *__restrict__ T, double *__restrict__ p_loss,
                                                  double *__restrict__ p_eu) {
    __shared__ double sh[kNTL];
    double l = 0.0;
    double eu[kRank * kMaxProbes];
    for (int e = 0; e < kRank * kMaxProbes; ++e) eu[e] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNTL + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNTL) {
        double u[kRank];
        for (int a = 0; a < kRank; ++a) u[a] = (double)Uh[i * kRank + a];
        for (int k = 0; k < kMaxProbes; ++k) {
            if (k >= Pn) break;
            double s = 0.0;
            for (int a = 0; a < kRank; ++a) s += u[a] * T[a * kMaxProbes + k];
            const double e = W[i * Pn + k] - Sw[i * Pn + k] - s;
            l += e * e;
            for (int a = 0; a < kRank; ++a) eu[k * kRank + a] += e * u[a];
        }
    }
    const double sl = block_sum_l(l, sh);
    if (threadIdx.x == 0) p_loss[blockIdx.x] = sl;
    for (int e = 0; e < kRank * kMaxProbes; ++e) {
        const double s = block_sum_l(eu[e], sh);
        if (threadIdx.x == 0) p_eu[blockIdx.x * kRank * kMaxProbes + e] = s;
    }
}

// g_out (= d loss / d Uh, n x 8): scale (E T^T + Sw (E^T Uh)), scale = -2 / (P n)
__global__ void k_probe_G(int64_t n, int Pn, const float *__restrict__ Uh, const double *__restrict__ W,
                          const double *__restrict__ Sw, const double *__restrict__ T, const double *__restrict__ EU,
                          double scale, float *__restrict__ g_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double u[kRank], g[kRank];
    for (int a = 0; a < kRank; ++a) {
        u[a] = (double)Uh[i * kRank + a];
        g[a] = 0.0;
    }
    for (int k = 0; k < Pn; ++k) {
        double s = 0.0;
        for (int a = 0; a < kRank; ++a) s += u[a] * T[a * kMaxProbes + k];
        const double e = W[i * Pn + k] - Sw[i * Pn + k] - s;
        const double sw = Sw[i * Pn + k];
        for (int a = 0; a < kRank; ++a) g[a] += e * T[a * kMaxProbes + k] + sw * EU[k * kRank + a];
    }
    for (int a = 0; a < kRank; ++a) g_out[i * kRank + a] = (float)(scale * g[a]);
}

void launch_probe_loss_grad(int64_t n, int Pn, const float *Uh, const double *W, const double *Sw, double *work,
                            float *g_out, hipStream_t s) {
    const int ne = kRank * kMaxProbes;
    double *pT = work, *T = pT + kRedBlocks * ne, *pl = T + ne, *peu = pl + kRedBlocks, *res = peu + kRedBlocks * ne;
    hipLaunchKernelGGL(k_probe_T, dim3(kRedBlocks), dim3(kNTL), 0, s, n, Pn, Uh, Sw, pT);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(ne), 0, s, pT, ne, T);
    hipLaunchKernelGGL(k_probe_E, dim3(kRedBlocks), dim3(kNTL), 0, s, n, Pn, Uh, W, Sw, T, pl, peu);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, pl, 1, res);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(ne), 0, s, peu, ne, res + 1);
    hipLaunchKernelGGL(k_probe_G, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, Pn, Uh, W, Sw, T, res + 1,
                       -2.0 / ((double)Pn * (double)n), g_out);
}

size_t probe_work_doubles() { return (size_t)(kRedBlocks * 2 + 2) * kRank * kMaxProbes + kRedBlocks + 1; }

void launch_mlp_backward(const float *P, const float *F, const float *hid, const float *g_out, float *g_pre, int rows,
                         float *grad, hipStream_t s) {
    const int64_t nh = (int64_t)rows * kHid;
    hipLaunchKernelGGL(k_mlp_bwd_hidden, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, s, P, g_out, hid, rows,
                       g_pre);
    hipLaunchKernelGGL(k_mlp_grad_params, dim3((kParams + 255) / 256), dim3(256), 0, s, F, hid, g_out, g_pre, rows,
                       grad);
}

// ---------------------------------------------------------------- Adam

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int np_, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np_) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

void launch_adam(float *P, const float *g, float *m, float *v, int t, float lr, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, P, g, m, v, kParams, lr, b1, b2, 1e-8f,
                       c1, c2);
}

}  // namespace ba
