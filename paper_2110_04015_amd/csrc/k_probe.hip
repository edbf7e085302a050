// Measurement helper: the HBM read rate this GPU sustains for the access pattern of the
// Schur chunk kernel (one wavefront per chunk of 16 tiles, each tile 12 coalesced 1 KiB
// loads per wavefront, non-temporal), with no arithmetic besides a running sum.  It is the
// practical ceiling against which the S-product kernel's bandwidth is read.
#include <hip/hip_runtime.h>

#include <chrono>
#include <string>

#include "ba_internal.h"
#include "kernels.h"

namespace {

typedef double dbl2p_t __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(64) void k_stream_read(const dbl2p_t *__restrict__ p, int64_t tiles,
                                                    double *__restrict__ out) {
    double s = 0.0;
    const int64_t t0 = (int64_t)blockIdx.x * 16;
    for (int64_t t = t0; t < t0 + 16 && t < tiles; ++t) {
        const dbl2p_t *q = p + t * 12 * 64 + threadIdx.x;
        dbl2p_t w[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = __builtin_nontemporal_load(q + k * 64);
#pragma unroll
        for (int k = 0; k < 12; ++k) s += w[k].x + w[k].y;
    }
    if (s == 1.0) out[0] = s;   // never true for the zero-filled buffer; keeps the loads
}

}  // namespace

extern "C" ba_status ba_stream_read_gbs(int64_t bytes, int32_t reps, double *gbs, void *stream) {
    using namespace ba;
    if (bytes < (int64_t)12 * 64 * 16 || reps < 1 || !gbs) return set_error(BA_ERR_INVALID_ARG, "bytes >= 12 KiB, reps >= 1");
    hipStream_t q = (hipStream_t)stream;
    const int64_t tiles = bytes / (12 * 64 * 16);
    const int64_t used = tiles * 12 * 64 * 16;
    void *buf = nullptr;
    double *out = nullptr;
    if (hipMalloc(&buf, (size_t)used) != hipSuccess) return set_error(BA_ERR_NOMEM, "probe buffer");
    if (hipMalloc((void **)&out, sizeof(double)) != hipSuccess) {
        (void)hipFree(buf);
        return set_error(BA_ERR_NOMEM, "probe buffer");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMemsetAsync(buf, 0, (size_t)used, q);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const unsigned chunks = (unsigned)((tiles + 15) / 16);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_stream_read, dim3(chunks), dim3(64), 0, q, (const dbl2p_t *)buf, tiles, out);
        e = hipEventRecord(e0, q);
    }
    for (int r = 0; r < reps && e == hipSuccess; ++r)
        hipLaunchKernelGGL(k_stream_read, dim3(chunks), dim3(64), 0, q, (const dbl2p_t *)buf, tiles, out);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, q);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    (void)hipFree(out);
    if (e != hipSuccess) return set_error(BA_ERR_HIP, std::string("ba_stream_read_gbs: ") + hipGetErrorString(e));
    *gbs = (double)used * reps / (ms * 1e-3) / 1e9;
    return BA_OK;
}
