// Allocation-free variant of the implicit Schur product (ba_schur_matvec_noalloc).
//
// The chunked product writes one partial camera row per (chunk, camera) before the
// camera reduction adds them; ba_schur_matvec keeps those rows in a buffer the
// library allocated at build.  This variant keeps them in a file-scope device array
// instead, so the call itself allocates nothing.  Each GPU holds its own copy of the
// array (at its own address) until the process ends; every call on one GPU shares
// it, so calls that overlap on one GPU race.  Every partial row is written by the
// chunk that owns it before the reduction reads it, so nothing needs clearing.
#include <mutex>

#include "ba_internal.h"
#include "kernels.h"

namespace {

constexpr size_t kScratchDoubles = size_t(4) << 20;   // 32 MiB of partial rows

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` on each device

// The device address of this device's copy of `scratch` (the host-side name is only
// a stand-in for it), looked up once per device with that device current.
ba_status scratch_for(int dev, double **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return ba::set_error(BA_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return BA_OK;
}

}  // namespace

extern "C" ba_status ba_schur_matvec_noalloc(ba_system *s, const double *v, double *y, int32_t precision) {
    if (!s || !v || !y) return ba::set_error(BA_ERR_INVALID_ARG, "NULL argument");
    if (precision < 0 || precision > 2)
        return ba::set_error(BA_ERR_INVALID_ARG, "precision must be 0 (FP64), 1 (FP32) or 2 (BF16)");
    if ((precision == 1 && !s->J32) || (precision == 2 && !s->J16))
        return ba::set_error(BA_ERR_UNSUPPORTED,
                             "the system holds no Jacobian copy in this precision (build it with store_fp32 or "
                             "store_bf16): the allocation-free product does not create one");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return ba::set_error(BA_ERR_HIP, "no current HIP device");
    if (dev != s->device)
        return ba::set_error(BA_ERR_INVALID_ARG, "the system's device must be the current device");
    const ba::SchurArgs base = ba::system_schur_args(s, precision);
    if (ba::system_uses_bsr(s, base)) {
        // the explicit S product keeps no partial rows
        ba::launch_bsr_mv(s->np, s->bsr_ptr, s->bsr_col, s->bsr_val, v, y, nullptr, s->stream, nullptr, nullptr);
    } else {
        const size_t need = (size_t)std::max<int64_t>(s->plan.n_part, 1) * (size_t)s->dp;
        if (need > kScratchDoubles)
            return ba::set_error(BA_ERR_WORKSPACE, "the product's partial rows (" + std::to_string(need) +
                                                       " doubles) exceed the allocation-free scratch (" +
                                                       std::to_string(kScratchDoubles) + " doubles)");
        double *ptr = nullptr;
        const ba_status st = scratch_for(dev, &ptr);
        if (st != BA_OK) return st;
        ba::SchurArgs a = base;
        a.partial = ptr;
        ba::launch_schur_matvec(a, v, y, s->stream);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return ba::set_error(BA_ERR_HIP, std::string("ba_schur_matvec_noalloc: ") + hipGetErrorString(e));
    return BA_OK;
}
