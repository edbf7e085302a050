// C ABI of the reduced-camera-system library: system build, Schur products,
// and the PCG (Algorithm 1) and MCG (Algorithm 2) drivers.  The host only
// orchestrates: every arithmetic step runs in the HIP kernels; per iteration
// the host reads back a handful of device scalars (the stop test and the
// tau-test branch) to choose the next launches.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ba_internal.h"
#include "kernels.h"

using namespace ba;

namespace {

thread_local std::string g_err;

constexpr int64_t kHistScratch = 4 << 20;   // doubles of split-K partials of the history products (32 MiB)

ba_status fail(ba_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(BA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
ba_status dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(BA_ERR_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    return BA_OK;
}

template <typename T>
ba_status upload(T **p, const std::vector<T> &v, hipStream_t s) {
    ba_status st = dalloc(p, v.size());
    if (st != BA_OK) return st;
    if (!v.empty()) HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return BA_OK;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

// Device memory of a system: from the caller's workspace when it brought one (a bump
// allocation, 256-byte aligned; BA_ERR_WORKSPACE when it is used up), else hipMalloc.  In
// the sizing pass (ws_counting) nothing is allocated: the offsets are only counted and a
// non-null stand-in address that nothing dereferences is returned.
template <typename T>
ba_status salloc(ba_system *s, T **p, size_t count) {
    if (!s->ws_base && !s->ws_counting) return dalloc(p, count);
    *p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    const size_t off = (s->ws_used + 255) & ~size_t(255);
    if (s->ws_counting) {
        s->ws_used = off + bytes;
        *p = reinterpret_cast<T *>((uintptr_t)4096 + off);
        return BA_OK;
    }
    if (off + bytes > s->ws_size)
        return fail(BA_ERR_WORKSPACE, "the caller's workspace is used up: " + std::to_string(off + bytes) +
                                          " bytes needed, " + std::to_string(s->ws_size) + " given");
    *p = reinterpret_cast<T *>(s->ws_base + off);
    s->ws_used = off + bytes;
    return BA_OK;
}

template <typename T>
void sfree(ba_system *s, T *&p) {
    if (!p) return;
    if (!s->ws_base && !s->ws_counting) (void)hipFree((void *)p);   // workspace memory is the caller's
    p = nullptr;
}

// salloc, then the host vector's contents (no copy in the sizing pass)
template <typename T>
ba_status supload(ba_system *s, T **p, const std::vector<T> &v) {
    ba_status st = salloc(s, p, v.size());
    if (st != BA_OK) return st;
    if (!s->ws_counting && !v.empty())
        HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s->stream));
    return BA_OK;
}

void free_multi(ba_system *s, DevMulti &m) {
    sfree(s, m.mmeta);
    sfree(s, m.slot_cam);
    sfree(s, m.pair_ll);
    sfree(s, m.tile_oidx);
    sfree(s, m.oidx);
    sfree(s, m.slot_ooff);
    sfree(s, m.chunk_tile);
    sfree(s, m.chunk_part);
    sfree(s, m.cg_ptr);
    sfree(s, m.cg_idx);
    sfree(s, m.part_dst);
    sfree(s, m.partial);
    sfree(s, m.group);
    sfree(s, m.chunk_seg);
    m = DevMulti();
}

void free_all(ba_system *s) {
    sfree(s, s->J64);
    sfree(s, s->J32);
    sfree(s, s->J16);
    sfree(s, s->slot_obs);
    sfree(s, s->cam_obs_ptr);
    sfree(s, s->cam_obs);
    sfree(s, s->lmk_store);
    sfree(s, s->obs_lm);
    sfree(s, s->h0);
    sfree(s, s->Vraw);
    sfree(s, s->Uraw);
    sfree(s, s->bp);
    sfree(s, s->obs_slot);
    sfree(s, s->bsr_slot_cam);
    sfree(s, s->meta);
    sfree(s, s->tile_lmk_base);
    sfree(s, s->chunk_tile);
    sfree(s, s->chunk_part);
    sfree(s, s->part_cam);
    sfree(s, s->cam_part_ptr);
    sfree(s, s->cam_part_idx);
    sfree(s, s->part_dst);
    sfree(s, s->partial);
    sfree(s, s->vinv);
    sfree(s, s->bl);
    sfree(s, s->dU);
    sfree(s, s->Dblk);
    sfree(s, s->Dchol);
    sfree(s, s->bt);
    sfree(s, s->lmk_order);
    sfree(s, s->lmk_first_slot);
    sfree(s, s->lmk_count);
    sfree(s, s->status);
    sfree(s, s->vec);
    sfree(s, s->red);
    sfree(s, s->hist);
    sfree(s, s->hist32);
    sfree(s, s->small);
    sfree(s, s->hscratch);
    sfree(s, s->tickets);
    sfree(s, s->refine_buf);
    sfree(s, s->Ulr);
    sfree(s, s->degree);
    sfree(s, s->lr_proj);
    sfree(s, s->seg_cam);
    sfree(s, s->seg_chunk);
    sfree(s, s->bsr_ptr);
    sfree(s, s->bsr_col);
    sfree(s, s->bsr_val);
    if (s->host_pinned) (void)hipHostFree(s->host_pinned);
    s->host_pinned = nullptr;
    s->host_pinned_dev = nullptr;
    free_multi(s, s->multi);
    for (hipEvent_t e : s->prof_events) (void)hipEventDestroy(e);
    s->prof_events.clear();
}

SchurArgs schur_args(ba_system *s, int precision) {
    SchurArgs a{};
    a.J = precision == 1 ? (const void *)s->J32 : precision == 2 ? (const void *)s->J16 : (const void *)s->J64;
    a.precision = precision;
    a.meta = s->meta;
    a.tile_lmk_base = s->tile_lmk_base;
    a.vinv = s->vinv;
    a.chunk_tile = s->chunk_tile;
    a.chunk_part = s->chunk_part;
    a.part_cam = s->part_cam;
    a.part_dst = s->part_dst;
    a.n_chunks = s->plan.n_chunks;
    // LDS rows per chunk: the most cameras any chunk holds (often well below the
    // max_slots limit, which leaves room for more resident wavefronts)
    a.max_slots = s->plan.max_used_slots;
    a.partial = s->partial;
    a.cam_part_ptr = s->cam_part_ptr;
    a.dU = s->dU;
    a.np = s->np;
    a.done = nullptr;
    a.dp = s->dp;
    return a;
}

// Flushes the recorded event pairs into the running total (waits for the stream).
void profile_flush(ba_system *s) {
    if (s->prof_used == 0) return;
    (void)hipStreamSynchronize(s->stream);
    for (size_t i = 0; i + 1 < s->prof_used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, s->prof_events[i], s->prof_events[i + 1]) == hipSuccess) {
            s->prof_ms += ms;
            s->prof_launches += 1;
        }
    }
    s->prof_used = 0;
}

// S v from the explicit block-sparse S (FP64 products of a system built with it)
inline bool use_bsr(const ba_system *s, const SchurArgs &a) {
    return s->bsr_val && a.precision == 0 && !a.seg_skip;
}

// partial pairs of the Gram products a product with gram set leaves (camera reduction of
// the implicit product: one per four cameras; explicit product: one per block row)
inline int gram_parts(const ba_system *s, const SchurArgs &a) {
    return use_bsr(s, a) ? bsr_gram_blocks(s->np) : schur_gram_blocks(s->np);
}
inline int gram_parts_max(const ba_system *s) { return std::max(bsr_gram_blocks(s->np), schur_gram_blocks(s->np)); }

// Room for one more start/stop pair of profiling events (created on demand, timing only:
// no system-scope fence, so no L2 writeback at each record); false when none can be made.
bool profile_room(ba_system *s) {
    if (s->prof_used + 2 <= s->prof_events.size()) return true;
    if (s->prof_events.size() >= 4096) profile_flush(s);
    while (s->prof_used + 2 > s->prof_events.size()) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return false;
        s->prof_events.push_back(e);
    }
    return true;
}

// y = S v; with profiling on, the dominant kernel (the chunk kernel of the implicit
// product, or the block-sparse product of an explicit S) is bracketed by events on the
// stream, on every prof_every-th call
void matvec(ba_system *s, const SchurArgs &a, const double *v, double *y) {
    const bool sample = s->profiling && (s->prof_calls++ % s->prof_every) == 0 && profile_room(s);
    if (use_bsr(s, a)) {
        if (sample) (void)hipEventRecord(s->prof_events[s->prof_used], s->stream);
        launch_bsr_mv(s->np, s->bsr_ptr, s->bsr_col, s->bsr_val, v, y, a.done, s->stream, a.gram, a.gram_r);
        if (sample) {
            (void)hipEventRecord(s->prof_events[s->prof_used + 1], s->stream);
            s->prof_used += 2;
        }
        return;
    }
    if (!sample) {
        launch_schur_matvec(a, v, y, s->stream);
        return;
    }
    (void)hipEventRecord(s->prof_events[s->prof_used], s->stream);
    launch_schur_chunks(a, v, s->stream);
    (void)hipEventRecord(s->prof_events[s->prof_used + 1], s->stream);
    s->prof_used += 2;
    launch_schur_reduce(a, v, y, s->stream);
}

ba_status ensure_precision(ba_system *s, int precision) {
    if (precision < 0 || precision > 2) return fail(BA_ERR_INVALID_ARG, "precision must be 0 (FP64), 1 (FP32) or 2 (BF16)");
    const int64_t nslots = s->plan.n_tiles * kTile;
    if (precision == 1 && !s->J32) {
        ba_status st = salloc(s, &s->J32, (size_t)nslots * 24);
        if (st != BA_OK) return st;
        if (!s->ws_counting) launch_convert(s->J64, nslots, s->J32, nullptr, s->stream, s->dp);
        HIPCHK(hipGetLastError());
    }
    if (precision == 2 && !s->J16) {
        ba_status st = salloc(s, &s->J16, (size_t)nslots * 24);
        if (st != BA_OK) return st;
        if (!s->ws_counting) launch_convert(s->J64, nslots, nullptr, s->J16, s->stream, s->dp);
        HIPCHK(hipGetLastError());
    }
    return BA_OK;
}

// The partition into N subsets and, with `plan`, the layout of the implicit
// multidirectional product (the explicit S's grouped product needs the partition only).
ba_status ensure_multi(ba_system *s, int N, bool plan = true) {
    if (s->multi.N == N && s->multi.group && (!plan || s->multi.partial)) return BA_OK;
    if (s->ws_base && s->multi.group)
        return fail(BA_ERR_WORKSPACE, "the caller's workspace holds the layout of N = " + std::to_string(s->multi.N) +
                                          " subsets (ba_build_opts.ws_groups), not of N = " + std::to_string(N));
    free_multi(s, s->multi);
    HostMultiPlan mp;
    std::string err;
    // subsets: Sec. 3.2's partition of the poses; in a batch, of each problem's poses
    std::vector<int32_t> grp((size_t)s->np);
    const std::vector<int32_t> &seg = s->plan.cam_seg;
    if (seg.empty()) {
        partition_groups(s->np, N, grp.data());
    } else {
        for (int c0 = 0; c0 < s->np;) {
            int c1 = c0;
            while (c1 < s->np && seg[(size_t)c1] == seg[(size_t)c0]) ++c1;
            if (c1 - c0 < N) return fail(BA_ERR_INVALID_ARG, "N exceeds the cameras of a problem of the batch");
            partition_groups(c1 - c0, N, grp.data() + c0);
            c0 = c1;
        }
    }
    ba_status st;
    if (!plan) {
        if ((st = supload(s, &s->multi.group, grp)) != BA_OK) return st;
        s->multi.N = N;
        HIPCHK(hipStreamSynchronize(s->stream));   // grp goes out of scope
        return BA_OK;
    }
    st = build_multi_plan(s->plan, N, 512, mp, err, grp.data());
    if (st != BA_OK) return fail(st, err);
    // LDS of the multidirectional kernel: max_out rows of 9 plus 2 x 64 x 3 values (FP64),
    // up to the device's work-group limit (160 KiB on gfx950: 2,232 rows)
    int dev = 0, lds_max = 65536;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t lds_need = (size_t)(mp.max_out * s->dp + 6 * kTile) * sizeof(double);
    if (lds_need > (size_t)lds_max)
        return fail(BA_ERR_UNSUPPORTED, "multidirectional product: a tile touches " + std::to_string(mp.max_out) +
                                            " (camera, subset) pairs; at most " +
                                            std::to_string(((size_t)lds_max / sizeof(double) - 6 * kTile) / s->dp) +
                                            " fit in LDS");
    DevMulti &m = s->multi;
    hipStream_t q = s->stream;
    if ((st = supload(s, &m.mmeta, mp.mmeta)) != BA_OK) return st;
    if ((st = supload(s, &m.slot_cam, mp.slot_cam)) != BA_OK) return st;
    if ((st = supload(s, &m.pair_ll, mp.pair_ll)) != BA_OK) return st;
    if ((st = supload(s, &m.tile_oidx, mp.tile_oidx)) != BA_OK) return st;
    if ((st = supload(s, &m.oidx, mp.oidx)) != BA_OK) return st;
    if ((st = supload(s, &m.slot_ooff, mp.slot_ooff)) != BA_OK) return st;
    if ((st = supload(s, &m.chunk_tile, mp.chunk_tile)) != BA_OK) return st;
    if ((st = supload(s, &m.chunk_part, mp.chunk_part)) != BA_OK) return st;
    if ((st = supload(s, &m.cg_ptr, mp.cg_ptr)) != BA_OK) return st;
    if ((st = supload(s, &m.cg_idx, mp.cg_idx)) != BA_OK) return st;
    if ((st = supload(s, &m.part_dst, mp.part_dst)) != BA_OK) return st;
    if ((st = supload(s, &m.group, grp)) != BA_OK) return st;
    if ((st = supload(s, &m.chunk_seg, mp.chunk_seg)) != BA_OK) return st;
    if ((st = salloc(s, &m.partial, (size_t)std::max<int64_t>(mp.n_part, 1) * s->dp)) != BA_OK) return st;
    m.N = N;
    m.n_chunks = mp.n_chunks;
    m.max_out = mp.max_out;
    m.n_part = mp.n_part;
    HIPCHK(hipStreamSynchronize(q));   // the host vectors above go out of scope
    return BA_OK;
}

MultiArgs multi_args(ba_system *s, int precision) {
    MultiArgs a{};
    a.J = precision == 1 ? (const void *)s->J32 : precision == 2 ? (const void *)s->J16 : (const void *)s->J64;
    a.precision = precision;
    a.meta = s->meta;
    a.mmeta = s->multi.mmeta;
    a.slot_cam = s->multi.slot_cam;
    a.pair_ll = s->multi.pair_ll;
    a.tile_oidx = s->multi.tile_oidx;
    a.oidx = s->multi.oidx;
    a.slot_ooff = s->multi.slot_ooff;
    a.tile_lmk_base = s->tile_lmk_base;
    a.vinv = s->vinv;
    a.chunk_tile = s->multi.chunk_tile;
    a.chunk_part = s->multi.chunk_part;
    a.n_chunks = s->multi.n_chunks;
    a.max_out = s->multi.max_out;
    a.partial = s->multi.partial;
    a.part_dst = s->multi.part_dst;
    a.cg_ptr = s->multi.cg_ptr;
    a.dU = s->dU;
    a.group = s->multi.group;
    a.np = s->np;
    a.N = s->multi.N;
    a.dp = s->dp;
    return a;
}

// Grows a buffer of the system to `count` elements: the new buffer is allocated before the
// old one is dropped, so a failure (a used-up workspace) leaves the system as it was.
template <typename T, typename C>
ba_status grow(ba_system *s, T *&buf, C &cap, size_t count) {
    if ((size_t)cap >= count) return BA_OK;
    T *nb = nullptr;
    ba_status st = salloc(s, &nb, count);
    if (st != BA_OK) return st;
    sfree(s, buf);
    buf = nb;
    cap = (C)count;
    return BA_OK;
}

ba_status ensure_vec(ba_system *s, size_t doubles) { return grow(s, s->vec, s->vec_cap, doubles); }

ba_status ensure_red(ba_system *s, size_t doubles) { return grow(s, s->red, s->red_cap, doubles); }

// per-iteration residual trace of PCG (device, max_iter doubles)
ba_status ensure_trace(ba_system *s, int64_t count) { return grow(s, s->trace_buf, s->trace_cap, (size_t)count); }

// arrival counters of the last-block reductions: zero on allocation, and every kernel
// that takes one leaves it zero
ba_status ensure_tickets(ba_system *s, int64_t count) {
    if (s->tickets_cap >= count) return BA_OK;
    ba_status st = grow(s, s->tickets, s->tickets_cap, (size_t)count);
    if (st != BA_OK) return st;
    if (!s->ws_counting) HIPCHK(hipMemsetAsync(s->tickets, 0, (size_t)count * sizeof(uint32_t), s->stream));
    return BA_OK;
}

ba_status ensure_pinned(ba_system *s) {
    if (s->ws_counting) return BA_OK;
    if (!s->host_pinned) {
        // SC_COUNT scalars and the tag of the kernel-written copy
        HIPCHK(hipHostMalloc((void **)&s->host_pinned, (SC_COUNT + 1) * sizeof(double), hipHostMallocMapped));
        s->host_pinned[SC_COUNT] = 0.0;
        HIPCHK(hipHostGetDevicePointer((void **)&s->host_pinned_dev, s->host_pinned, 0));
    }
    return BA_OK;
}

// Waits for the scalars a kernel wrote to host_pinned with the tag `tag` (written after
// the values, which the kernel released at system scope first): the host polls the tag,
// with no event between the kernels.  Only when the tag is late (10 ms) does it ask the
// stream, every 10 ms, whether it failed or drained without the tag (an error either
// way): a stream query can itself put work on the device's queue.
static ba_status scalars_wait_tag(ba_system *s, double tag, double *out) {
    volatile double *t = s->host_pinned + SC_COUNT;
    const auto t0 = std::chrono::steady_clock::now();
    auto next = t0 + std::chrono::milliseconds(10);
    for (int64_t spin = 1; *t != tag; ++spin) {
        if ((spin & 255) == 0 && std::chrono::steady_clock::now() >= next) {
            next += std::chrono::milliseconds(10);
            const hipError_t e = hipStreamQuery(s->stream);
            if (e != hipSuccess && e != hipErrorNotReady)
                return fail(BA_ERR_HIP, std::string("waiting for the MCG scalars: ") + hipGetErrorString(e));
            if (e == hipSuccess && *t != tag) return fail(BA_ERR_HIP, "the MCG scalars were not written");
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60))
                return fail(BA_ERR_HIP, "timed out waiting for the MCG scalars");
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    memcpy(out, s->host_pinned, SC_COUNT * sizeof(double));
    return BA_OK;
}

// Copies the device scalars to the host and waits for the stream.
ba_status read_scalars(ba_system *s, const double *sc, double *out) {
    HIPCHK(hipMemcpyAsync(s->host_pinned, sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    memcpy(out, s->host_pinned, SC_COUNT * sizeof(double));
    return BA_OK;
}

ba_status init_scalars(ba_system *s, double *sc) {
    double h[SC_COUNT];
    for (int i = 0; i < SC_COUNT; ++i) h[i] = 0.0;
    h[SC_RR0] = -1.0;
    memcpy(s->host_pinned, h, sizeof h);
    HIPCHK(hipMemcpyAsync(sc, s->host_pinned, SC_COUNT * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

// |-b~ - S x| / |b~| in FP64 (tmp: 2n doubles, red: partial sums)
ba_status true_rel_residual(ba_system *s, const double *x, double *tmp, double *red, double *sc, double *out) {
    const int64_t n = (int64_t)s->np * s->dp;
    matvec(s, schur_args(s, 0), x, tmp);
    launch_pcg_init(n, s->bt, tmp, tmp + n, red, s->stream);
    launch_finalize(red, 1, sc + SC_COUNT - 1, s->stream);
    launch_pcg_init(n, s->bt, nullptr, tmp + n, red, s->stream);
    launch_finalize(red, 1, sc + SC_COUNT - 2, s->stream);
    HIPCHK(hipGetLastError());
    double h[SC_COUNT];
    ba_status st = read_scalars(s, sc, h);
    if (st != BA_OK) return st;
    double num = h[SC_COUNT - 1], den = h[SC_COUNT - 2];
    *out = den > 0.0 ? std::sqrt(num / den) : std::sqrt(num);
    return BA_OK;
}

void fill_default_opts(ba_solve_opts *o) {
    memset(o, 0, sizeof(*o));
    o->eps = 1e-6;
    o->max_iter = 1000;
    o->precision = BA_PREC_FP64;
    o->precond = 0;
    o->max_history_cols = 0;
    o->inner_eps = 0.0;     // automatic: by the precision of the products
    o->max_outer = 20;
    o->history_fp32 = 1;   // mixed precision: the reorthogonalisation reads the FP32 history copy
    o->max_inner = 1000;
}

}  // namespace

namespace ba {
ba_status set_error(ba_status st, const std::string &msg) { return fail(st, msg); }
SchurArgs system_schur_args(ba_system *s, int precision) { return schur_args(s, precision); }
bool system_uses_bsr(const ba_system *s, const SchurArgs &a) { return use_bsr(s, a); }

ba_status prepare_mcg(ba_system *s, int N, int precision) {
    ba_status st = ensure_precision(s, precision);
    if (st != BA_OK || N <= 1) return st;
    if (N > s->np) return fail(BA_ERR_INVALID_ARG, "N must be in [1, n_cams]");
    const bool bsr = s->bsr_val && precision == 0 && N <= kMaxBlock;
    return ensure_multi(s, N, !bsr);
}
}  // namespace ba

extern "C" {

void ba_default_solve_opts(ba_solve_opts *opts) {
    if (opts) fill_default_opts(opts);
}

const char *ba_last_error(void) { return g_err.c_str(); }

const char *ba_status_string(int32_t st) {
    switch (st) {
        case BA_OK: return "ok";
        case BA_MAXITER: return "maximum number of iterations reached";
        case BA_ERR_INVALID_ARG: return "invalid argument";
        case BA_ERR_NONFINITE: return "non-finite input";
        case BA_ERR_NOT_SPD: return "matrix block not positive definite";
        case BA_ERR_BREAKDOWN: return "Krylov breakdown";
        case BA_ERR_WORKSPACE: return "workspace too small";
        case BA_ERR_HIP: return "HIP runtime error";
        case BA_ERR_NOMEM: return "out of memory";
        case BA_ERR_UNSUPPORTED: return "unsupported input";
        default: return "unknown status";
    }
}

ba_status ba_partition(int32_t n_cams, int32_t n_groups, int32_t *group) {
    if (!group || n_cams < 1 || n_groups < 1 || n_groups > n_cams)
        return fail(BA_ERR_INVALID_ARG, "ba_partition: need group != NULL and 1 <= N <= n_cams");
    partition_groups(n_cams, n_groups, group);
    return BA_OK;
}

void ba_free_system(ba_system *sys) {
    if (!sys) return;
    (void)hipStreamSynchronize(sys->stream);
    free_all(sys);
    delete sys;
}

static BsrGather bsr_gather(const ba_system *s) {
    BsrGather g;
    g.cam_ptr = s->cam_obs_ptr;
    g.cam_obs = s->cam_obs;
    g.obs_lm = s->obs_lm;
    g.lmk_store = s->lmk_store;
    g.lmk_first_slot = s->lmk_first_slot;
    g.lmk_count = s->lmk_count;
    g.slot_cam = s->bsr_slot_cam;
    return g;
}

// The values of a system that depend on lambda (s->lambda), from the lambda-free sums
// and the packed Jacobian stream: V_lambda^-1 and h0 = V_lambda^-1 b_l per landmark,
// D(S), its factor, the damping of the S product and b~ per camera (eq. (9)-(15)), and
// the explicit S when the system keeps one.  Waits for the stream.
static ba_status apply_lambda(ba_system *s) {
    hipStream_t q = s->stream;
    HIPCHK(hipMemsetAsync(s->status, 0, sizeof(int32_t), q));
    launch_landmarks_lambda(s->nl, s->Vraw, s->bl, s->lambda, s->vinv, s->h0, s->status, q);
    launch_cameras_lambda(s->np, s->cam_obs_ptr, s->cam_obs, s->obs_lm, s->lmk_store, s->obs_slot, s->J64, s->Uraw,
                          s->bp, s->vinv, s->h0, s->lambda, s->dU, s->Dblk, s->Dchol, s->bt, s->status, q, s->dp);
    if (s->bsr_val) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        if (e0) (void)hipEventRecord(e0, q);
        launch_bsr_assemble(s->np, bsr_gather(s), s->obs_slot, s->J64, s->vinv, s->Dblk, s->bsr_ptr, s->bsr_col,
                            s->bsr_max_row, s->bsr_piece, s->bsr_val, q);
        if (e1) (void)hipEventRecord(e1, q);
        if (hipStreamSynchronize(q) == hipSuccess && e0 && e1) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) s->bsr_build_ms = ms;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
    HIPCHK(hipGetLastError());
    int32_t hst = 0;
    HIPCHK(hipMemcpyAsync(&hst, s->status, 4, hipMemcpyDeviceToHost, q));
    HIPCHK(hipStreamSynchronize(q));
    if (hst & kStatusNotSpdLandmark) return fail(BA_ERR_NOT_SPD, "a landmark block V_lambda is not positive definite");
    if (hst & kStatusNotSpdCamera)
        return fail(BA_ERR_NOT_SPD, "a block of D(S) is not positive definite (unobserved camera?)");
    return BA_OK;
}

// Values of a system whose layout is set: checks J_p, J_l, r (device, observation
// order of the build) for NaN/Inf, packs the Jacobian stream, forms the lambda-free
// sums (J_l^T J_l, b_l, J_p^T J_p, b_p), then the values for s->lambda.  Waits for the
// stream.
static ba_status fill_values(ba_system *s, const double *J_p, const double *J_l, const double *r) {
    hipStream_t q = s->stream;
    const int64_t m = s->m;
    const int64_t nslots = s->plan.n_tiles * kTile;
    HIPCHK(hipMemsetAsync(s->status, 0, sizeof(int32_t), q));
    launch_check_finite(J_p, m * 2 * s->dp, s->status, q);
    launch_check_finite(J_l, m * 6, s->status, q);
    launch_check_finite(r, m * 2, s->status, q);
    int32_t hst = 0;
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&hst, s->status, 4, hipMemcpyDeviceToHost, q));
    HIPCHK(hipStreamSynchronize(q));
    if (hst & kStatusNonfinite) return fail(BA_ERR_NONFINITE, "NaN or Inf in J_p, J_l or r");
    launch_pack(s->slot_obs, nslots, J_p, J_l, s->J64, s->J32, s->J16, q, s->dp);
    launch_landmarks_base(s->nl, s->lmk_first_slot, s->lmk_count, s->slot_obs, J_l, r, s->Vraw, s->bl, q);
    launch_cameras_base(s->np, s->cam_obs_ptr, s->cam_obs, J_p, r, s->Uraw, s->bp, q, s->dp);
    HIPCHK(hipGetLastError());
    return apply_lambda(s);
}

static ba_status pcg_buffers(ba_system *s, int max_iter, bool trace);
static ba_status mcg_buffers(ba_system *s, int N, int64_t cap);

// The solver memory a system in a caller's workspace reserves at build, so that the solves
// the options name never allocate: PCG (with a residual trace), MCG with ws_groups subsets
// (0: none) and a history for ws_max_iter iterations (0: 1000), the multidirectional
// layout, and the refinement vectors when a reduced-precision copy is stored.
static ba_status reserve_solvers(ba_system *s, const ba_build_opts *o) {
    const int N = o ? o->ws_groups : 0;
    const int it = o && o->ws_max_iter > 0 ? o->ws_max_iter : 1000;
    const bool mixed = o && (o->store_fp32 || o->store_bf16);
    if (N < 0 || N > s->np || it < 1) return fail(BA_ERR_INVALID_ARG, "ws_groups must be in [0, n_cams] and ws_max_iter >= 0");
    ba_status st;
    if ((st = pcg_buffers(s, it, true)) != BA_OK) return st;
    if (N >= 1) {
        if (N > 1) {
            // the explicit S's grouped product needs the partition only, reduced-precision
            // products the implicit layout
            const bool bsr = s->bsr_val && N <= kMaxBlock;
            if ((st = ensure_multi(s, N, !bsr || mixed)) != BA_OK) return st;
        }
        if ((st = mcg_buffers(s, N, 1 + (int64_t)it * N)) != BA_OK) return st;
    }
    if (mixed) {
        const int64_t n = (int64_t)s->np * s->dp;
        if ((st = grow(s, s->refine_buf, s->refine_cap, (size_t)n * 5 + 8)) != BA_OK) return st;
        // the FP32 history copy of mixed-precision MCG (history_fp32, the default)
        if (N >= 1 && (st = grow(s, s->hist32, s->hist32_cap, (size_t)(s->hist_cap_cols * n))) != BA_OK) return st;
    }
    return BA_OK;
}

// ws (nullable): the caller's device workspace of ws_bytes; counting: the sizing pass, which
// plans the layout on the host and counts the device bytes without allocating or launching.
static ba_status build_system(const ba_problem_desc *d, const ba_build_opts *opts, void *stream,
                              const int32_t *cam_seg, ba_system **out, char *ws = nullptr, size_t ws_bytes = 0,
                              bool counting = false) {
    if (!out) return fail(BA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!d) return fail(BA_ERR_INVALID_ARG, "desc is NULL");
    if (d->d_p != 9 && d->d_p != 6) return fail(BA_ERR_INVALID_ARG, "d_p must be 9 or 6");
    if (d->d_p == 6 && cam_seg) return fail(BA_ERR_UNSUPPORTED, "batches take poses with d_p = 9");
    if (d->d_p == 6 && opts && opts->explicit_schur)
        return fail(BA_ERR_UNSUPPORTED, "the explicit S is formed for d_p = 9 only");
    if (d->n_cams < 1 || d->n_lms < 1 || d->n_obs < 1)
        return fail(BA_ERR_INVALID_ARG, "n_cams, n_lms and n_obs must be positive");
    if (!d->obs_cam || !d->obs_lm || !d->J_p || !d->J_l || !d->r)
        return fail(BA_ERR_INVALID_ARG, "a problem array is NULL");
    if (!std::isfinite(d->lambda)) return fail(BA_ERR_NONFINITE, "lambda is not finite");
    if (d->lambda < 0.0) return fail(BA_ERR_INVALID_ARG, "lambda must be >= 0");
    int max_slots = opts && opts->max_slots ? opts->max_slots : 128;
    // max_tiles 0: chunks sized so that the S product's chunks are all resident at once
    int max_tiles = opts && opts->max_tiles ? opts->max_tiles : 0;
    // the chunk kernel keeps 2 * max_slots camera rows of 9 doubles in LDS (<= 64 KiB)
    const int max_tiles_multi = opts ? opts->max_tiles_multi : 0;
    if (max_tiles_multi < 0 || max_tiles_multi > 4096)
        return fail(BA_ERR_INVALID_ARG, "max_tiles_multi must be in [0, 4096]");
    if (max_slots < kTile || max_slots > 440 || max_tiles < 0 || max_tiles > 4096)
        return fail(BA_ERR_INVALID_ARG, "max_slots must be in [64, 440] and max_tiles in [1, 4096]");

    ba_system *s = new ba_system();
    s->stream = (hipStream_t)stream;
    s->ws_base = ws;
    s->ws_size = ws_bytes;
    s->ws_counting = counting;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(BA_ERR_HIP, "no current HIP device");
    }
    s->np = d->n_cams;
    s->nl = d->n_lms;
    s->m = d->n_obs;
    s->lambda = d->lambda;
    s->dp = d->d_p;
    hipStream_t q = s->stream;
    auto bail = [&](ba_status st) {
        (void)hipStreamSynchronize(q);
        free_all(s);
        delete s;
        return st;
    };
    const int64_t m = d->n_obs;
    std::vector<int32_t> hcam((size_t)m), hlm((size_t)m);
    if (hipMemcpyAsync(hcam.data(), d->obs_cam, (size_t)m * 4, hipMemcpyDeviceToHost, q) != hipSuccess ||
        hipMemcpyAsync(hlm.data(), d->obs_lm, (size_t)m * 4, hipMemcpyDeviceToHost, q) != hipSuccess ||
        hipStreamSynchronize(q) != hipSuccess)
        return bail(fail(BA_ERR_HIP, "copying the observation indices to the host failed"));
    std::string err;
    ba_status st = build_plan(s->np, s->nl, m, hcam.data(), hlm.data(), max_slots, max_tiles, s->plan, err,
                              cam_seg, max_tiles == 0 ? schur1_resident_chunks(d->d_p) : 0, max_tiles_multi,
                              max_tiles == 0 && max_tiles_multi == 0 ? schur_multi_resident_chunks(d->d_p) : 0);
    if (st != BA_OK) return bail(fail(st, err));
    if (cam_seg) {
        if ((st = supload(s, &s->seg_cam, s->plan.cam_seg)) != BA_OK) return bail(st);
        if ((st = supload(s, &s->seg_chunk, s->plan.chunk_seg)) != BA_OK) return bail(st);
    }
    const HostPlan &P = s->plan;
    const int64_t nslots = P.n_tiles * kTile;

    if ((st = salloc(s, &s->status, 1)) != BA_OK) return bail(st);
    // layout on the device (kept for ba_update_system)
    if ((st = supload(s, &s->slot_obs, P.slot_obs)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->cam_obs_ptr, P.cam_obs_ptr)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->cam_obs, P.cam_obs)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->lmk_store, P.lmk_store)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->obs_lm, hlm)) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->h0, (size_t)s->nl * 3)) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->Vraw, (size_t)s->nl * 6)) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->Uraw, (size_t)s->np * (d->d_p * (d->d_p + 1) / 2))) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->bp, (size_t)s->np * d->d_p)) != BA_OK) return bail(st);
    {
        // tile slot of every observation (the lambda kernels read the packed stream by it)
        std::vector<int64_t> oslot((size_t)m, 0);
        for (int64_t sl = 0; sl < P.n_tiles * kTile; ++sl) {
            const int64_t o = P.slot_obs[(size_t)sl];
            if (o >= 0) oslot[(size_t)o] = sl;
        }
        if ((st = supload(s, &s->obs_slot, oslot)) != BA_OK) return bail(st);
        if (hipStreamSynchronize(q) != hipSuccess) return bail(fail(BA_ERR_HIP, "uploading the slot map failed"));
    }
    if ((st = supload(s, &s->meta, P.meta)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->tile_lmk_base, P.tile_lmk_base)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->chunk_tile, P.chunk_tile)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->chunk_part, P.chunk_part)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->part_cam, P.part_cam)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->cam_part_ptr, P.cam_part_ptr)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->cam_part_idx, P.cam_part_idx)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->part_dst, P.part_dst)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->lmk_order, P.lmk_order)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->lmk_first_slot, P.lmk_first_slot)) != BA_OK) return bail(st);
    if ((st = supload(s, &s->lmk_count, P.lmk_count)) != BA_OK) return bail(st);
    const int dp = s->dp;
    if ((st = salloc(s, &s->partial, (size_t)std::max<int64_t>(P.n_part, 1) * dp)) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->J64, (size_t)nslots * 24)) != BA_OK) return bail(st);
    if (opts && opts->store_fp32 && (st = salloc(s, &s->J32, (size_t)nslots * 24)) != BA_OK) return bail(st);
    if (opts && opts->store_bf16 && (st = salloc(s, &s->J16, (size_t)nslots * 24)) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->vinv, (size_t)s->nl * 6)) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->bl, (size_t)s->nl * 3)) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->dU, (size_t)s->np * dp)) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->Dblk, (size_t)s->np * dp * dp)) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->Dchol, (size_t)s->np * (dp * (dp + 1) / 2))) != BA_OK) return bail(st);
    if ((st = salloc(s, &s->bt, (size_t)s->np * dp)) != BA_OK) return bail(st);
    if (opts && opts->explicit_schur) {
        // explicit S in block-sparse rows, assembled from the same blocks (Sec. 3.2, 4.1): the
        // pattern and the contribution pairs depend on the observations only
        if (cam_seg) return bail(fail(BA_ERR_UNSUPPORTED, "batches use the implicit S products"));
        // camera of every observation slot (host, from the plan)
        std::vector<int32_t> scam((size_t)nslots, 0);
        for (int64_t sl = 0; sl < nslots; ++sl) {
            const int64_t o = P.slot_obs[(size_t)sl];
            if (o >= 0) scam[(size_t)sl] = P.obs_cam[(size_t)o];
        }
        if ((st = supload(s, &s->bsr_slot_cam, scam)) != BA_OK) return bail(st);
        // pattern on the device: block counts per row, then the rows' columns
        int32_t *d_nnz = nullptr;
        if ((st = salloc(s, &d_nnz, (size_t)s->np)) != BA_OK) return bail(st);
        std::vector<int32_t> nnz((size_t)s->np);
        if (counting) {
            // the same counts from the host plan: a row holds camera j and every camera
            // sharing a landmark with it
            covisibility_degree(P, nnz);
            for (int32_t &c : nnz) c += 1;
        } else {
            launch_bsr_rowcount(s->np, bsr_gather(s), d_nnz, q);
            const bool cnt_ok = hipGetLastError() == hipSuccess &&
                                hipMemcpyAsync(nnz.data(), d_nnz, (size_t)s->np * 4, hipMemcpyDeviceToHost, q) ==
                                    hipSuccess &&
                                hipStreamSynchronize(q) == hipSuccess;
            if (!cnt_ok) return bail(fail(BA_ERR_HIP, "explicit S: pattern count failed"));
        }
        sfree(s, d_nnz);
        std::vector<int32_t> rp((size_t)s->np + 1, 0);
        int max_row = 0;
        for (int j = 0; j < s->np; ++j) {
            if ((int64_t)rp[(size_t)j] + nnz[(size_t)j] > (int64_t)INT32_MAX)
                return bail(fail(BA_ERR_UNSUPPORTED, "explicit S: too many nonzero blocks"));
            rp[(size_t)j + 1] = rp[(size_t)j] + nnz[(size_t)j];
            max_row = std::max(max_row, (int)nnz[(size_t)j]);
        }
        int dev = 0, lds_max = 65536;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return bail(fail(BA_ERR_HIP, "device attribute query failed"));
        // rows wider than one wavefront's LDS are assembled in pieces
        const int piece = bsr_assembly_piece(max_row, (size_t)lds_max);
        if (piece < 1)
            return bail(fail(BA_ERR_UNSUPPORTED, "explicit S: a camera is covisible with " + std::to_string(max_row) +
                                                     " cameras, more than one work-group's LDS holds"));
        if ((size_t)((s->np + 31) / 32) * 4 > (size_t)lds_max)
            return bail(fail(BA_ERR_UNSUPPORTED, "explicit S: too many cameras for the pattern bitmap"));
        if ((st = supload(s, &s->bsr_ptr, rp)) != BA_OK) return bail(st);
        s->bsr_nnzb = (int64_t)rp[(size_t)s->np];
        s->bsr_max_row = max_row;
        s->bsr_piece = piece;
        if ((st = salloc(s, &s->bsr_col, (size_t)std::max<int64_t>(s->bsr_nnzb, 1))) != BA_OK) return bail(st);
        if (!counting) launch_bsr_rowfill(s->np, bsr_gather(s), s->bsr_ptr, s->bsr_col, q);
        if ((st = salloc(s, &s->bsr_val, (size_t)s->bsr_nnzb * 81)) != BA_OK) return bail(st);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(q) != hipSuccess)   // host vectors go out of scope
            return bail(fail(BA_ERR_HIP, "explicit S: pattern failed"));
    }
    if (!counting && (st = fill_values(s, d->J_p, d->J_l, d->r)) != BA_OK) return bail(st);
    if ((st = ensure_pinned(s)) != BA_OK) return bail(st);
    if ((ws || counting) && (st = reserve_solvers(s, opts)) != BA_OK) return bail(st);
    *out = s;
    return BA_OK;
}

ba_status ba_build_system(const ba_problem_desc *d, const ba_build_opts *opts, void *stream, ba_system **out) {
    return build_system(d, opts, stream, nullptr, out);
}

ba_status ba_build_workspace_bytes(const ba_problem_desc *d, const ba_build_opts *opts, size_t *bytes) {
    if (!bytes) return fail(BA_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = 0;
    ba_system *s = nullptr;
    const ba_status st = build_system(d, opts, nullptr, nullptr, &s, nullptr, 0, true);
    if (st != BA_OK) return st;
    *bytes = (s->ws_used + 255) & ~size_t(255);
    free_all(s);
    delete s;
    return BA_OK;
}

ba_status ba_build_system_ws(const ba_problem_desc *d, const ba_build_opts *opts, void *ws, size_t ws_bytes,
                             void *stream, ba_system **out) {
    if (out) *out = nullptr;
    if (!ws) return fail(BA_ERR_INVALID_ARG, "ws is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(BA_ERR_INVALID_ARG, "ws must be 256-byte aligned");
    return build_system(d, opts, stream, nullptr, out, static_cast<char *>(ws), ws_bytes, false);
}

ba_status ba_system_workspace_used(const ba_system *s, size_t *bytes) {
    if (!s || !bytes) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    *bytes = s->ws_base ? s->ws_used : 0;
    return BA_OK;
}

ba_status ba_update_system(ba_system *s, const double *J_p, const double *J_l, const double *r, double lambda) {
    if (!s || !J_p || !J_l || !r) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    if (s->seg_cam) return fail(BA_ERR_INVALID_ARG, "batch systems are not updated in place");
    if (!std::isfinite(lambda)) return fail(BA_ERR_NONFINITE, "lambda is not finite");
    if (lambda < 0.0) return fail(BA_ERR_INVALID_ARG, "lambda must be >= 0");
    const double prev = s->lambda;
    s->lambda = lambda;
    const ba_status st = fill_values(s, J_p, J_l, r);
    if (st == BA_ERR_NONFINITE) s->lambda = prev;   // rejected before any value changed
    return st;
}

ba_status ba_set_lambda(ba_system *s, double lambda) {
    if (!s) return fail(BA_ERR_INVALID_ARG, "sys is NULL");
    if (s->seg_cam) return fail(BA_ERR_INVALID_ARG, "batch systems are not updated in place");
    if (!std::isfinite(lambda)) return fail(BA_ERR_NONFINITE, "lambda is not finite");
    if (lambda < 0.0) return fail(BA_ERR_INVALID_ARG, "lambda must be >= 0");
    s->lambda = lambda;
    return apply_lambda(s);
}

ba_status ba_profile_enable(ba_system *s, int32_t on) {
    if (!s) return fail(BA_ERR_INVALID_ARG, "sys is NULL");
    if (on < 0) return fail(BA_ERR_INVALID_ARG, "on must be >= 0");
    profile_flush(s);
    s->profiling = on != 0;
    s->prof_every = on > 0 ? on : 1;
    s->prof_calls = 0;
    return BA_OK;
}

ba_status ba_profile_read(ba_system *s, double *ms_total, int64_t *launches, int32_t reset) {
    if (!s) return fail(BA_ERR_INVALID_ARG, "sys is NULL");
    profile_flush(s);
    if (ms_total) *ms_total = s->prof_ms;
    if (launches) *launches = s->prof_launches;
    if (reset) {
        s->prof_ms = 0.0;
        s->prof_launches = 0;
    }
    return BA_OK;
}

ba_status ba_system_info(const ba_system *s, int32_t *n_cams, int32_t *n_lms, int64_t *n_obs, int64_t *n_tiles,
                         int32_t *n_chunks, int64_t *matvec_bytes_fp64) {
    if (!s) return fail(BA_ERR_INVALID_ARG, "sys is NULL");
    if (n_cams) *n_cams = s->np;
    if (n_lms) *n_lms = s->nl;
    if (n_obs) *n_obs = s->m;
    if (n_tiles) *n_tiles = s->plan.n_tiles;
    if (n_chunks) *n_chunks = s->plan.n_chunks;
    // one read of the Jacobian blocks and a camera index per observation, V^-1 per
    // landmark, lambda diag(U), v and y per camera
    if (matvec_bytes_fp64)
        *matvec_bytes_fp64 = s->m * ((2 * s->dp + 6) * 8 + 4) + (int64_t)s->nl * 6 * 8 + (int64_t)s->np * s->dp * 8 * 3;
    return BA_OK;
}

ba_status ba_schur_matvec(ba_system *s, const double *v, double *y, int32_t precision) {
    if (!s || !v || !y) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    ba_status st = ensure_precision(s, precision);
    if (st != BA_OK) return st;
    matvec(s, schur_args(s, precision), v, y);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_schur_matvec_timed(ba_system *s, const double *v, double *y, int32_t precision, int32_t reps,
                                double *ms_per) {
    if (!s || !v || !y || !ms_per) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    if (reps < 1) return fail(BA_ERR_INVALID_ARG, "reps must be >= 1");
    ba_status st = ensure_precision(s, precision);
    if (st != BA_OK) return st;
    const SchurArgs a = schur_args(s, precision);
    matvec(s, a, v, y);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(BA_ERR_HIP, "hipEventCreate failed");
    }
    (void)hipEventRecord(e0, s->stream);
    for (int i = 0; i < reps; ++i) matvec(s, a, v, y);
    (void)hipEventRecord(e1, s->stream);
    const hipError_t err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(BA_ERR_HIP, std::string("timed S products: ") + hipGetErrorString(err));
    *ms_per = (double)ms / reps;
    return BA_OK;
}

ba_status ba_schur_matmat_grouped(ba_system *s, int32_t N, const double *z, double *Y, int32_t precision) {
    if (!s || !z || !Y) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    if (N < 1 || N > s->np) return fail(BA_ERR_INVALID_ARG, "N must be in [1, n_cams]");
    ba_status st = ensure_precision(s, precision);
    if (st != BA_OK) return st;
    const bool bsr = s->bsr_val && precision == 0 && N <= kMaxBlock;   // the grouped kernel keeps N x 9 sums in LDS
    if ((st = ensure_multi(s, N, !bsr)) != BA_OK) return st;
    if (bsr)
        launch_bsr_mm_grouped(s->np, N, s->bsr_ptr, s->bsr_col, s->bsr_val, s->multi.group, z, Y, s->stream);
    else
        launch_schur_multi(multi_args(s, precision), z, Y, s->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_precond_apply(ba_system *s, const double *r, double *z) {
    if (!s || !r || !z) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    launch_precond(s->np, s->Dchol, r, z, s->stream, s->dp);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_get_rhs(ba_system *s, double *bt) {
    if (!s || !bt) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    HIPCHK(hipMemcpyAsync(bt, s->bt, (size_t)s->np * s->dp * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_get_precond_blocks(ba_system *s, double *D) {
    if (!s || !D) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    HIPCHK(hipMemcpyAsync(D, s->Dblk, (size_t)s->np * s->dp * s->dp * sizeof(double), hipMemcpyDeviceToDevice,
                          s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_prepare_mcg(ba_system *s, int32_t N, int32_t precision) {
    if (!s) return fail(BA_ERR_INVALID_ARG, "sys is NULL");
    if (N < 1 || N > s->np) return fail(BA_ERR_INVALID_ARG, "N must be in [1, n_cams]");
    const ba_status st = prepare_mcg(s, N, precision);
    if (st != BA_OK) return st;
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_back_substitute(ba_system *s, const double *dxp, double *dxl) {
    if (!s || !dxp || !dxl) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    const HostPlan &P = s->plan;
    launch_back_substitute(s->J64, s->meta, s->tile_lmk_base, s->chunk_tile, s->chunk_part, s->part_cam,
                           P.n_chunks, P.max_used_slots, s->vinv, s->bl, s->lmk_order, dxp, dxl, s->stream, s->dp);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_pinv_sym(int32_t k, const double *A, double *Ap, int32_t *rank, void *stream) {
    if (!A || !Ap || k < 1 || k > 64) return fail(BA_ERR_INVALID_ARG, "ba_pinv_sym: need A, Ap and 1 <= k <= 64");
    hipStream_t q = (hipStream_t)stream;
    int32_t *drank = nullptr;
    ba_status st = dalloc(&drank, 1);
    if (st != BA_OK) return st;
    launch_pinv_sym(k, A, Ap, drank, q);
    hipError_t e = hipGetLastError();
    int32_t hr = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hr, drank, 4, hipMemcpyDeviceToHost, q);
    if (e == hipSuccess) e = hipStreamSynchronize(q);
    dfree(drank);
    if (e != hipSuccess) return fail(BA_ERR_HIP, std::string("ba_pinv_sym: ") + hipGetErrorString(e));
    if (rank) *rank = hr;
    return BA_OK;
}

// ------------------------------------------------------------------ solver buffers

// What Algorithm 1 needs: work vectors, reduction partials, the arrival counter and (for a
// trace) max_iter doubles of residual history.
static ba_status pcg_buffers(ba_system *s, int max_iter, bool trace) {
    const int64_t n = (int64_t)s->np * s->dp;
    ba_status st;
    if ((st = ensure_vec(s, (size_t)n * 6 + SC_COUNT)) != BA_OK) return st;
    // red: scratch partials (the true residual), |r|^2, Phi, the camera reduction's Gram
    // partials, then the fused iteration end's partials
    const size_t ngram = 2 * (size_t)gram_parts_max(s), nxz = 2 * (size_t)mcg_xrz_blocks(s->np, s->dp);
    if ((st = ensure_red(s, (size_t)kRedBlocks * 4 + ngram + nxz)) != BA_OK) return st;
    if ((st = ensure_tickets(s, 1)) != BA_OK) return st;
    if (trace && (st = ensure_trace(s, std::max(max_iter, 1))) != BA_OK) return st;
    return BA_OK;
}

// What Algorithm 2 with N subsets and a history of `cap` columns needs: the P and Q
// histories, the small dense storage (Delta^+ blocks, Phi, beta, gamma, alpha, block
// tables), work vectors, reduction partials, the arrival counter and the split-K scratch
// of the history products.
static ba_status mcg_buffers(ba_system *s, int N, int64_t cap) {
    const int64_t n = (int64_t)s->np * s->dp;
    if (cap < 1) return fail(BA_ERR_WORKSPACE, "history capacity must hold at least one column");
    ba_status st;
    if (s->hist_cap_cols < cap) {
        double *h = nullptr;
        if ((st = salloc(s, &h, (size_t)(2 * cap) * (size_t)n)) != BA_OK) return st;
        sfree(s, s->hist);
        s->hist = h;
        s->hist_cap_cols = cap;
    }
    const int64_t hc = s->hist_cap_cols;
    // small storage: Dp (64 * cap), Phi (cap * max(N, kPhiSeg)), beta (cap * hist_ldb(N)), gamma,
    // alpha (64 each), block tables
    const size_t small_need = (size_t)(64 * hc + hc * std::max(N, kPhiSeg) + hc * hist_ldb(N) + 128) +
                              (size_t)(3 * hc + 8);
    if ((st = grow(s, s->small, s->small_cap, small_need)) != BA_OK) return st;
    if ((st = ensure_vec(s, (size_t)n * 4 + SC_COUNT)) != BA_OK) return st;
    // red: the Gram partials of wide blocks and their sums, or the iteration-end kernel's
    // partials followed by the one-column Gram partials of the S product
    const size_t goff = 2 * (size_t)mcg_xrz_blocks(s->np, s->dp);
    if ((st = ensure_red(s, std::max<size_t>((size_t)(kRedBlocks + 1) * (64 * 64 + 64), goff + 2 * (size_t)gram_parts_max(s)))) !=
        BA_OK)
        return st;
    if ((st = ensure_tickets(s, 1)) != BA_OK) return st;   // the iteration-end kernel's
    // split-K scratch of the history products: four column slices of both matrices of the
    // widest block (at least one is required)
    return grow(s, s->hscratch, s->hscratch_cap, (size_t)std::max<int64_t>(kHistScratch, 4 * hist_scratch_min(n, N)));
}

// ------------------------------------------------------------------ Algorithm 1

// Algorithm 1 on S x = -bt (bt: device [n]).  report_true: also recompute the true
// residual of the system's own b~ into stats.
static ba_status pcg_core(ba_system *s, const double *bt, bool report_true, const double *x0, double *x,
                          const ba_solve_opts &opts, ba_solve_stats *stats) {
    const int prec = opts.precision;
    ba_status st = ensure_precision(s, prec);
    if (st != BA_OK) return st;
    const int64_t n = (int64_t)s->np * s->dp;
    hipStream_t q = s->stream;
    const bool want_trace = stats && stats->trace_res && stats->trace_cap > 0;
    if ((st = pcg_buffers(s, opts.max_iter, want_trace)) != BA_OK) return st;
    // red: scratch partials (pdq: the true residual), |r|^2 (prr), Phi (pphi), the camera reduction's
    // Gram partials (pg), then the fused iteration end's partials (pxz)
    const size_t ngram = 2 * (size_t)gram_parts_max(s);
    double *r = s->vec, *z = r + n, *P = z + n, *Q = P + n, *tmp = Q + n, *sc = tmp + 2 * n;
    double *pdq = s->red, *prr = pdq + kRedBlocks * 2, *pphi = prr + kRedBlocks, *pg = pphi + kRedBlocks;
    double *pxz = pg + ngram;
    auto t0 = std::chrono::steady_clock::now();
    if ((st = init_scalars(s, sc)) != BA_OK) return st;
    if (x0) {
        HIPCHK(hipMemcpyAsync(x, x0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, q));
        matvec(s, schur_args(s, prec), x, tmp);
        launch_pcg_init(n, bt, tmp, r, prr, q);
    } else {
        HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), q));
        launch_pcg_init(n, bt, nullptr, r, prr, q);
    }
    launch_pcg_rr(prr, sc, q);
    HIPCHK(hipGetLastError());
    double h[SC_COUNT];
    if ((st = read_scalars(s, sc, h)) != BA_OK) return st;
    const double rr0 = h[SC_RR0];
    double rr = rr0;
    int it = 0;
    ba_status result = BA_OK;
    if (rr0 > 0.0 && opts.max_iter > 0) {
        // Iterations are enqueued in batches; the stop test runs on the device and
        // turns the remaining kernels of the batch into no-ops, so the host waits
        // only once per batch.
        double *trace_dev = want_trace ? s->trace_buf : nullptr;
        const bool lowrank = opts.precond == 1;
        launch_precond(s->np, s->Dchol, r, P, q, s->dp);
        if (lowrank) launch_lowrank_apply(n, s->Ulr, r, P, nullptr, s->lr_proj, nullptr, nullptr, q);
        SchurArgs sa = schur_args(s, prec);
        sa.done = sc + SC_DONE;
        // Delta_i and gamma_i from the camera reduction of Q_i = S P_i (or from the
        // explicit-S product, which leaves the same partials)
        sa.gram = pg;
        sa.gram_r = r;
        int enqueued = 0, batch = 4;
        const size_t prof_mark = s->prof_used;
        const int64_t call_mark = s->prof_calls;
        double rr_prev = rr0;
        for (;;) {
            const int nb = std::min(batch, opts.max_iter - enqueued);
            for (int b = 0; b < nb; ++b) {
                matvec(s, sa, P, Q);                                         // Q_i = S P_i; Delta_i, gamma_i
                const double *dq = pg;
                const int ndq = gram_parts(s, sa);
                if (!lowrank) {
                    // alpha_i, x_{i+1}, r_{i+1}, the stop test, Z_{i+1}, Phi_i and beta_i
                    launch_pcg_xrz(s->np, dq, ndq, sc, x, r, P, Q, s->Dchol, z, pxz, s->tickets, opts.eps,
                                   opts.max_iter, trace_dev, q, s->dp);
                    launch_pcg_update_p(n, nullptr, sc, z, P, q);            // P_{i+1}
                } else {                                                     // M^-1 = D^-1 + U U^T
                    launch_pcg_update_xr(n, dq, ndq, sc, x, r, P, Q, prr, q);
                    launch_pcg_step_end(prr, sc, opts.eps, opts.max_iter, trace_dev, q);
                    launch_pcg_precond_phi(s->np, s->Dchol, r, Q, z, pphi, sc + SC_DONE, q, s->dp);
                    launch_lowrank_apply(n, s->Ulr, r, z, Q, s->lr_proj, pphi, sc + SC_DONE, q);
                    launch_pcg_update_p(n, pphi, sc, z, P, q);
                }                   // beta_i, P_{i+1}
            }
            enqueued += nb;
            if (hipGetLastError() != hipSuccess) return fail(BA_ERR_HIP, "PCG kernel launch failed");
            if ((st = read_scalars(s, sc, h)) != BA_OK) return st;
            if (h[SC_DONE] != 0.0 || enqueued >= opts.max_iter) break;
            // next batch: the iterations still needed at the observed rate of decrease
            const double rate = h[SC_RR] > 0.0 && rr_prev > 0.0 ? std::pow(h[SC_RR] / rr_prev, 1.0 / nb) : 1.0;
            const double goal = opts.eps * opts.eps * rr0;
            int need = 4;
            if (rate < 1.0 && h[SC_RR] > goal) need = (int)std::ceil(std::log(goal / h[SC_RR]) / std::log(rate));
            batch = std::max(1, std::min(need, 32));
            rr_prev = h[SC_RR];
        }
        it = (int)h[SC_ITER];
        // event pairs of launches after the stop test (no-ops) are not kernel work: keep the
        // pairs of the sampled launches among the first `it` (launch j of this loop has call
        // number call_mark + j and is sampled when that is a multiple of prof_every)
        if (s->profiling) {
            const int64_t k = s->prof_every;
            const auto sampled_below = [k](int64_t c) { return (c + k - 1) / k; };
            const size_t keep = 2 * (size_t)(sampled_below(call_mark + it) - sampled_below(call_mark));
            if (s->prof_used > prof_mark + keep) s->prof_used = prof_mark + keep;
        }
        rr = h[SC_RR];
        result = h[SC_DONE] != 0.0 ? (ba_status)(int)h[SC_STATUS] : BA_MAXITER;
        if (result == BA_ERR_BREAKDOWN) g_err = "PCG breakdown: P^T S P <= 0";
        if (want_trace && it > 0) {
            hipError_t e = hipMemcpy(stats->trace_res, trace_dev, sizeof(double) * (size_t)std::min(it, stats->trace_cap),
                                     hipMemcpyDeviceToHost);
            if (e != hipSuccess) return fail(BA_ERR_HIP, "trace copy failed");
        }
    }
    HIPCHK(hipStreamSynchronize(q));
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) {
        stats->iterations = it;
        stats->multi_steps = 0;
        stats->history_cols = it;
        stats->refinement_steps = 0;
        stats->status = result;
        stats->rel_res_recursive = rr0 > 0.0 ? std::sqrt(rr / rr0) : 0.0;
        stats->t_solve_ms = ms;
        double tr = stats->rel_res_recursive;
        if (report_true && (st = true_rel_residual(s, x, tmp, pdq, sc, &tr)) != BA_OK) return st;
        stats->rel_res_true = tr;
    }
    return result;
}

// ------------------------------------------------------------------ Algorithm 2

// Algorithm 2 on S x = -bt (arguments as pcg_core).
static ba_status mcg_core(ba_system *s, const double *bt, bool report_true, int N, double tau, const double *x0,
                          double *x, const ba_solve_opts &opts, ba_solve_stats *stats) {
    const int prec = opts.precision;
    ba_status st = ensure_precision(s, prec);
    if (st != BA_OK) return st;
    const bool use_bsr_multi = N > 1 && s->bsr_val && prec == 0 && N <= kMaxBlock;
    if (N > 1 && (st = ensure_multi(s, N, !use_bsr_multi)) != BA_OK) return st;
    const int64_t n = (int64_t)s->np * s->dp;
    hipStream_t q = s->stream;
    const int64_t cap = opts.max_history_cols > 0 ? opts.max_history_cols : 1 + (int64_t)opts.max_iter * N;
    if ((st = mcg_buffers(s, N, cap)) != BA_OK) return st;
    const int64_t hc = s->hist_cap_cols;
    double *Ph = s->hist, *Qh = s->hist + hc * n;
    // mixed precision: the reorthogonalisation reads (Phi and the history products) may
    // take an FP32 copy of the history: block 0 is copied, every later block's P and Q
    // columns are written in both precisions by the kernels that finish them
    const bool h32 = prec != 0 && opts.history_fp32 != 0;
    float *P32 = nullptr, *Q32 = nullptr;
    if (h32) {
        if ((st = grow(s, s->hist32, s->hist32_cap, (size_t)(hc * n))) != BA_OK) return st;
        P32 = reinterpret_cast<float *>(s->hist32);
        Q32 = P32 + hc * n;
    }
    const int phiw = std::max(N, kPhiSeg);
    const int ldb = hist_ldb(N);
    double *Dp = s->small, *Phi = Dp + 64 * hc, *beta = Phi + hc * phiw, *gamma = beta + hc * ldb, *alpha = gamma + 64;
    int32_t *blk_off = reinterpret_cast<int32_t *>(alpha + 64);
    int32_t *blk_k = blk_off + hc;
    int64_t *blk_dp = reinterpret_cast<int64_t *>(blk_k + hc + 2);
    const size_t goff = 2 * (size_t)mcg_xrz_blocks(s->np, s->dp);
    double *r = s->vec, *z = r + n, *tmp = z + n, *sc = tmp + 2 * n;
    double *red = s->red;
    const int gs = (s->np / N) * s->dp;   // rows of one subset (Sec. 3.2 partition)
    const SchurArgs sa = schur_args(s, prec);
    const MultiArgs ma = N > 1 && !use_bsr_multi ? multi_args(s, prec) : MultiArgs();

    auto t0 = std::chrono::steady_clock::now();
    if ((st = init_scalars(s, sc)) != BA_OK) return st;
    if (x0) {
        HIPCHK(hipMemcpyAsync(x, x0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, q));
        matvec(s, sa, x, tmp);
        launch_pcg_init(n, bt, tmp, r, red, q);
    } else {
        HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), q));
        launch_pcg_init(n, bt, nullptr, r, red, q);
    }
    launch_pcg_rr(red, sc, q);
    HIPCHK(hipGetLastError());
    double h[SC_COUNT];
    if ((st = read_scalars(s, sc, h)) != BA_OK) return st;
    const double rr0 = h[SC_RR0];
    double rr = rr0;
    int it = 0, multi_steps = 0;
    int64_t hcols = 0;
    ba_status result = BA_OK;
    if (rr0 > 0.0) {
        // P_0 = Z_0 = M^-1 r_0 ; Q_0 = S P_0
        const bool lowrank = opts.precond == 1;
        // one-column blocks take Delta and gamma from the camera reduction of Q = S P (or
        // the explicit-S product; partials at red + goff), and their Delta^+ and alpha from
        // the iteration-end kernel
        SchurArgs sag = sa;
        sag.gram = red + goff;
        sag.gram_r = r;
        // the learned term: U^T r partials, then w, in lr_proj (ensure_lowrank_storage)
        XrzLowrank lr;
        if (lowrank) {
            lr.U = s->Ulr;
            lr.part = s->lr_proj;
            lr.w = s->lr_proj + (int64_t)kLowRank * mcg_xrz_blocks(s->np, s->dp);
        }
        launch_precond(s->np, s->Dchol, r, Ph, q, s->dp);
        if (lowrank) launch_lowrank_apply(n, s->Ulr, r, Ph, nullptr, s->lr_proj, nullptr, nullptr, q);
        matvec(s, sag, Ph, Qh);
        if (h32) launch_hist_copy32(n, 0, 1, Ph, Qh, P32, Q32, q);
        std::vector<int32_t> hoff{0}, hk{1};
        std::vector<int64_t> hdp{0};
        int64_t dp_used = 1;
        hcols = 1;
        result = BA_MAXITER;
        for (it = 0; it < opts.max_iter;) {
            const int nb = (int)hoff.size();
            const int off = hoff.back(), k = hk.back();
            const int64_t dpo = hdp.back();
            // Delta_i = Q_i^T P_i, gamma_i = P_i^T r_i, alpha_i = Delta_i^+ gamma_i
            BlockEntry be;       // the current block's history table entry, written with its Delta^+
            be.off = blk_off;
            be.k = blk_k;
            be.dp = blk_dp;
            be.j = nb - 1;
            be.first = off;
            be.dpo = dpo;
            XrzGram g1;
            if (k == 1) {
                g1.part = red + goff;
                g1.nb = gram_parts(s, sag);
                g1.Dp = Dp + dpo;
                g1.blk = be;
            } else {
                launch_gram(n, k, Ph + (int64_t)off * n, Qh + (int64_t)off * n, r, red, q);
                launch_pinv_alpha(k, red, gram_blocks(k), Dp + dpo, gamma, alpha, sc, q, be);
            }
            // x_{i+1} = x_i + P_i alpha_i ; r_{i+1} = r_i - Q_i alpha_i ; Z = D^-1 r_{i+1}, and the
            // tau-test scalars before the single read-back of the iteration:
            // t_i = gamma_i^T alpha_i / (r_{i+1}^T D^-1 r_{i+1})
            // (the kernel also writes the scalars to the host, with a new tag; with the learned
            // term, rho = r^T M^-1 r and Z = D^-1 r + U (U^T r), the last by the next kernel)
            s->sc_tag += 1.0;
            launch_mcg_xrz(s->np, k, Ph + (int64_t)off * n, Qh + (int64_t)off * n, alpha, x, r, s->Dchol, z, red,
                           s->tickets, gamma, sc, s->host_pinned_dev, s->sc_tag, N, tau, opts.eps, q, s->dp, g1, lr);
            if (lowrank) launch_lr_zadd(n, s->Ulr, lr.w, z, q);
            // Everything up to the next iteration's Gram products that a one-column block
            // needs goes ahead of the read-back, so the device stays busy while the host
            // waits for it: Phi_{i,j} = Q_j^T Z_{i+1} per subset (valid for either outcome),
            // beta, the new block's P columns and the history sums of its Q columns, each
            // taking the block's width from the device's scalars (sc[SC_KN]), and S P_{i+1},
            // skipped on the device unless the block has one column.  A multidirectional
            // block's S Z and Q columns follow the read-back.
            double *Pn = Ph + hcols * n, *Qn = Qh + hcols * n;
            const bool ahead = N > 1 && hcols + N <= hc;   // room for a multidirectional block
            const bool room1 = hcols + 1 <= hc;
            const int kn_max = ahead ? N : room1 ? 1 : 0;
            float *Pn32 = h32 ? P32 + hcols * n : nullptr, *Qn32 = h32 ? Q32 + hcols * n : nullptr;
            if (h32) {
                launch_phi<float>(n, (int)hcols, Q32, z, N, gs, Phi, q);
            } else {
                launch_phi<double>(n, (int)hcols, Qh, z, N, gs, Phi, q);
            }
            // beta_{i,j} = Delta_j^+ Phi_{i,j}; P_{i+1} = Z - sum P_j beta
            launch_beta(nb, blk_off, blk_k, blk_dp, Dp, Phi, sc, kn_max, N, beta, q);
            if (h32)
                launch_update_pq<float>(n, (int)hcols, N, kn_max, P32, Q32, beta, z, gs, sc, Pn, s->hscratch,
                                        s->hscratch_cap, q, opts.history_mfma != 0, Pn32);
            else
                launch_update_pq<double>(n, (int)hcols, N, kn_max, Ph, Qh, beta, z, gs, sc, Pn, s->hscratch,
                                         s->hscratch_cap, q, opts.history_mfma != 0);
            bool spec_pair = false;   // the product's profiling events, dropped if it is skipped
            if (room1) {   // one-column block: Q_{i+1} = S P_{i+1}
                SchurArgs s1 = sag;
                s1.done = sc + SC_SKIPS;
                s1.y32 = Qn32;
                const size_t pu0 = s->prof_used;
                matvec(s, s1, Pn, Qn);
                spec_pair = s->prof_used != pu0;
            }
            HIPCHK(hipGetLastError());
            if ((st = scalars_wait_tag(s, s->sc_tag, h)) != BA_OK) return st;
            if (spec_pair && h[SC_KN] != 1.0) s->prof_used -= 2;   // a skipped launch is no kernel work
            if (h[SC_RANK] == 0.0) {
                result = BA_ERR_BREAKDOWN;
                g_err = "MCG breakdown: Delta_i is numerically zero";
                break;
            }
            ++it;
            rr = h[SC_RR];
            const int ti = it - 1;
            if (stats && ti < stats->trace_cap) {
                if (stats->trace_res) stats->trace_res[ti] = std::sqrt(rr / rr0);
                if (stats->trace_t) stats->trace_t[ti] = NAN;
                if (stats->trace_k) stats->trace_k[ti] = 0;
            }
            // the stop test and the tau-test are the device's (sc[SC_KN]: 0 once
            // |r| < eps |r_0|), so the host follows the blocks the device built
            const int kn = (int)h[SC_KN];
            if (kn == 0) {
                result = BA_OK;
                break;
            }
            const double t_i = h[SC_T];
            if (stats && ti < stats->trace_cap) {
                if (stats->trace_t) stats->trace_t[ti] = t_i;
                if (stats->trace_k) stats->trace_k[ti] = kn;
            }
            if (kn < 1 || kn > kn_max) {   // the device built nothing
                result = fail(BA_ERR_WORKSPACE, "MCG direction history is full (raise max_history_cols)");
                break;
            }
            const bool multi = kn > 1;
            if (multi) {   // Q_{i+1} = S Z - sum Q_j beta (eq. (19))
                if (use_bsr_multi) {
                    launch_bsr_mm_grouped(s->np, N, s->bsr_ptr, s->bsr_col, s->bsr_val, s->multi.group, z, Qn, q,
                                          nullptr);
                } else {
                    launch_schur_multi(ma, z, Qn, q);
                }
                launch_update_q(n, (int)hcols, N, sc, Qn, s->hscratch, s->hscratch_cap, q, Qn32);
            }
            hoff.push_back((int32_t)hcols);
            hk.push_back(kn);
            hdp.push_back(dp_used);
            dp_used += (int64_t)kn * kn;
            hcols += kn;
            multi_steps += multi;
        }
    }
    HIPCHK(hipStreamSynchronize(q));
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) {
        stats->iterations = it;
        stats->multi_steps = multi_steps;
        stats->history_cols = (int32_t)hcols;
        stats->refinement_steps = 0;
        stats->status = result;
        stats->rel_res_recursive = rr0 > 0.0 ? std::sqrt(rr / rr0) : 0.0;
        stats->t_solve_ms = ms;
        double tr = stats->rel_res_recursive;
        if (report_true && (st = true_rel_residual(s, x, tmp, red, sc, &tr)) != BA_OK) return st;
        stats->rel_res_true = tr;
    }
    return result;
}

// Mixed precision: FP64 iterative refinement around inner solves whose S products
// use the FP32 or BF16 Jacobian stream (all vectors and Krylov scalars stay FP64).
//   r = -b~ - S x (FP64 product);  stop when |r| < eps |b~|;
//   inner solve S d = r to inner_eps |r| (at most max_inner iterations);  x += d.
static ba_status refine(ba_system *s, bool use_mcg, int N, double tau, const double *x0, double *x,
                        const ba_solve_opts &opts, ba_solve_stats *stats) {
    const int64_t n = (int64_t)s->np * s->dp;
    hipStream_t q = s->stream;
    ba_status st = ensure_precision(s, opts.precision);
    if (st != BA_OK) return st;
    if ((st = grow(s, s->refine_buf, s->refine_cap, (size_t)n * 5 + 8)) != BA_OK) return st;
    double *r = s->refine_buf, *btp = r + n, *d = btp + n, *tmp = d + n, *xprev = tmp + n + 8;
    auto t0 = std::chrono::steady_clock::now();
    if (x0) HIPCHK(hipMemcpyAsync(x, x0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, q));
    else HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), q));
    ba_solve_opts in = opts;
    // Automatic inner tolerance: about the relative accuracy one inner solve on the
    // reduced-precision operator can deliver before restarting pays off.  Measured on
    // the F-1936-shaped problem to 1e-6 (iterations, refinement steps), with the final
    // step not oversolved (below): FP32 products, PCG 247 (2) at 1e-3 against 255 (3) at
    // 1e-2, 295 (3) at 3e-3 and 275 (2) at 3e-4; MCG N = 4 233 (2) at 1e-3 against 246 (3)
    // at 1e-2; BF16 storage, PCG 292 (6) at 1e-1 against 327 (5) at 3e-2 and 381 (4) at 1e-2.
    const double base_eps = opts.inner_eps > 0.0 ? opts.inner_eps : (opts.precision == BA_PREC_FP32 ? 1e-3 : 1e-1);
    in.max_iter = opts.max_inner;
    int total_it = 0, total_multi = 0, outer = 0;
    double rel = 0.0, prev = INFINITY;
    ba_status result = BA_MAXITER;
    const int trace_cap = stats ? stats->trace_cap : 0;
    for (;;) {
        // outer residual in FP64: r = -b~ - S x, btp = -r (so that S d = r reads S d = -btp)
        rel = 0.0;
        if ((st = ensure_red(s, (size_t)kRedBlocks * 4)) != BA_OK) return st;
        matvec(s, schur_args(s, 0), x, tmp);
        launch_residual_refine(n, s->bt, tmp, r, btp, s->red, q);
        double *sc2 = tmp + n;   // 8 scratch doubles after the four work vectors
        launch_finalize(s->red, 2, sc2, q);
        HIPCHK(hipGetLastError());
        double hh[2];
        HIPCHK(hipMemcpyAsync(hh, sc2, sizeof hh, hipMemcpyDeviceToHost, q));
        HIPCHK(hipStreamSynchronize(q));
        rel = hh[1] > 0.0 ? std::sqrt(hh[0] / hh[1]) : 0.0;
        if (rel < opts.eps || hh[0] == 0.0) {
            result = BA_OK;
            break;
        }
        if (outer > 0 && !(rel < prev)) {
            // the last correction did not reduce the FP64 residual (the inner solve on the
            // reduced-precision operator failed to contract, or diverged): keep the iterate
            // from before it
            HIPCHK(hipMemcpyAsync(x, xprev, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, q));
            rel = prev;
            break;
        }
        if (outer >= opts.max_outer || total_it >= opts.max_iter) break;
        prev = rel;
        ba_solve_stats is;
        memset(&is, 0, sizeof is);
        if (stats && stats->trace_res && total_it < trace_cap) {
            is.trace_cap = trace_cap - total_it;
            is.trace_res = stats->trace_res + total_it;
            is.trace_t = stats->trace_t ? stats->trace_t + total_it : nullptr;
            is.trace_k = stats->trace_k ? stats->trace_k + total_it : nullptr;
        }
        in.max_iter = std::min(opts.max_inner, opts.max_iter - total_it);
        // no oversolving: an inner solve need not take |r| below half of what the outer
        // target eps |b~| asks for (rel = |r| / |b~| >= eps here, so this stays <= 1/2)
        in.eps = std::max(base_eps, 0.5 * opts.eps / rel);
        ba_status ist = use_mcg ? mcg_core(s, btp, false, N, tau, nullptr, d, in, &is)
                                : pcg_core(s, btp, false, nullptr, d, in, &is);
        if (ist < 0 && ist != BA_ERR_BREAKDOWN) return ist;
        total_it += is.iterations;
        total_multi += is.multi_steps;
        ++outer;
        HIPCHK(hipMemcpyAsync(xprev, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, q));
        launch_axpy(n, 1.0, d, x, q);
        HIPCHK(hipGetLastError());
        if (is.iterations == 0) break;
    }
    HIPCHK(hipStreamSynchronize(q));
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) {
        stats->iterations = total_it;
        stats->multi_steps = total_multi;
        stats->history_cols = 0;
        stats->refinement_steps = outer;
        stats->status = result;
        stats->rel_res_recursive = rel;
        stats->rel_res_true = rel;
        stats->t_solve_ms = ms;
    }
    return result;
}

static ba_status check_opts(const ba_solve_opts *opts_in, ba_solve_opts *opts) {
    if (opts_in) *opts = *opts_in;
    else fill_default_opts(opts);
    if (opts->precond != 0 && opts->precond != 1) return fail(BA_ERR_INVALID_ARG, "precond must be 0 or 1");
    if (!(opts->eps >= 0.0) || opts->max_iter < 0) return fail(BA_ERR_INVALID_ARG, "eps >= 0 and max_iter >= 0 required");
    if (opts->precision < 0 || opts->precision > 2) return fail(BA_ERR_INVALID_ARG, "precision must be 0, 1 or 2");
    if (opts->precision != 0 && (!(opts->inner_eps >= 0.0) || opts->inner_eps >= 1.0 || opts->max_outer < 1 ||
                                 opts->max_inner < 1))
        return fail(BA_ERR_INVALID_ARG, "mixed precision needs 0 <= inner_eps < 1, max_outer >= 1, max_inner >= 1");
    return BA_OK;
}

ba_status ba_pcg_solve(ba_system *s, const double *x0, double *x, const ba_solve_opts *opts_in,
                       ba_solve_stats *stats) {
    if (!s || !x) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    ba_solve_opts opts;
    ba_status st = check_opts(opts_in, &opts);
    if (st != BA_OK) return st;
    if (opts.precond == 1 && !s->Ulr) return fail(BA_ERR_INVALID_ARG, "precond 1 needs a low-rank term (ba_set_lowrank_*)");
    if (opts.precision != 0) return refine(s, false, 0, 0.0, x0, x, opts, stats);
    return pcg_core(s, s->bt, true, x0, x, opts, stats);
}

ba_status ba_mcg_solve(ba_system *s, int32_t N, double tau, const double *x0, double *x,
                       const ba_solve_opts *opts_in, ba_solve_stats *stats) {
    if (!s || !x) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    if (N < 1 || N > s->np) return fail(BA_ERR_INVALID_ARG, "N must be in [1, n_cams]");
    if (N > 64) return fail(BA_ERR_UNSUPPORTED, "at most 64 subsets are supported");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(BA_ERR_INVALID_ARG, "tau must be finite and >= 0");
    ba_solve_opts opts;
    ba_status st = check_opts(opts_in, &opts);
    if (st != BA_OK) return st;
    if (opts.precond == 1 && !s->Ulr) return fail(BA_ERR_INVALID_ARG, "precond 1 needs a low-rank term (ba_set_lowrank_*)");
    if (opts.precision != 0) return refine(s, true, N, tau, x0, x, opts, stats);
    return mcg_core(s, s->bt, true, N, tau, x0, x, opts, stats);
}


// ------------------------------------------------------------------ learned preconditioner

// The learned correction's features and factors are defined on 9 x 9 pose blocks.
static ba_status lowrank_dp_check(const ba_system *s) {
    return s->dp == 9 ? BA_OK : fail(BA_ERR_UNSUPPORTED, "the learned low-rank preconditioner needs d_p = 9");
}

static ba_status ensure_lowrank_storage(ba_system *s) {
    ba_status st;
    if (!s->Ulr && (st = salloc(s, &s->Ulr, (size_t)s->np * 9 * 8)) != BA_OK) return st;
    // kRedBlocks rows of 8 for PCG's projections; MCG's iteration end keeps one row per
    // block and w after them
    const size_t proj = (size_t)std::max(kRedBlocks, mcg_xrz_blocks(s->np, s->dp) + 1) * kLowRank;
    if (!s->lr_proj && (st = salloc(s, &s->lr_proj, proj)) != BA_OK) return st;
    return BA_OK;
}

ba_status ba_lowrank_features(ba_system *s, float *F) {
    if (!s || !F) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    if (lowrank_dp_check(s) != BA_OK) return BA_ERR_UNSUPPORTED;
    if (!s->degree) {
        std::vector<int32_t> deg;
        covisibility_degree(s->plan, deg);
        ba_status st = supload(s, &s->degree, deg);
        if (st != BA_OK) return st;
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    launch_features(s->np, s->Dblk, s->degree, s->lambda, F, s->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_mlp_forward(const float *params, const float *F, int32_t rows, float *out, int32_t bf16, void *stream) {
    if (!params || !F || !out || rows < 1) return fail(BA_ERR_INVALID_ARG, "ba_mlp_forward: bad argument");
    hipStream_t q = (hipStream_t)stream;
    float *hid = nullptr;
    if (!bf16) {
        ba_status st = dalloc(&hid, (size_t)rows * 128);
        if (st != BA_OK) return st;
    }
    launch_mlp_forward(params, F, rows, out, hid, bf16 ? 1 : 0, q);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(q);
    dfree(hid);
    if (e != hipSuccess) return fail(BA_ERR_HIP, std::string("ba_mlp_forward: ") + hipGetErrorString(e));
    return BA_OK;
}

ba_status ba_set_lowrank_from_mlp(ba_system *s, const float *out) {
    if (!s || !out) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    if (lowrank_dp_check(s) != BA_OK) return BA_ERR_UNSUPPORTED;
    ba_status st = ensure_lowrank_storage(s);
    if (st != BA_OK) return st;
    launch_lowrank_U(s->np, s->Dchol, out, s->Ulr, s->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_set_lowrank_precond(ba_system *s, const double *U) {
    if (!s) return fail(BA_ERR_INVALID_ARG, "sys is NULL");
    if (U && lowrank_dp_check(s) != BA_OK) return BA_ERR_UNSUPPORTED;
    if (!U) {
        sfree(s, s->Ulr);
        return BA_OK;
    }
    ba_status st = ensure_lowrank_storage(s);
    if (st != BA_OK) return st;
    HIPCHK(hipMemcpyAsync(s->Ulr, U, (size_t)s->np * 9 * 8 * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_get_lowrank(ba_system *s, double *U) {
    if (!s || !U) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    if (!s->Ulr) return fail(BA_ERR_INVALID_ARG, "no low-rank term is set");
    HIPCHK(hipMemcpyAsync(U, s->Ulr, (size_t)s->np * 9 * 8 * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_block_scale(ba_system *s, const double *x, double *y, int32_t transpose) {
    if (!s || !x || !y) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    if (lowrank_dp_check(s) != BA_OK) return BA_ERR_UNSUPPORTED;
    launch_block_scale(s->np, s->Dchol, x, y, transpose ? 1 : 0, s->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return BA_OK;
}

ba_status ba_mlp_loss_grad(const float *params, const float *F, int32_t rows, const double *W, const double *Sw,
                           int32_t n_probes, float *grad, double *loss, void *stream) {
    if (!params || !F || !W || !Sw || !grad || rows < 1 || n_probes < 1 || n_probes > 8)
        return fail(BA_ERR_INVALID_ARG, "ba_mlp_loss_grad: bad argument (1 <= n_probes <= 8)");
    hipStream_t q = (hipStream_t)stream;
    const int64_t n = (int64_t)rows * 9;
    float *buf = nullptr;
    double *work = nullptr;
    ba_status st = dalloc(&buf, (size_t)rows * (128 * 2 + 72 * 2));
    if (st != BA_OK) return st;
    if ((st = dalloc(&work, probe_work_doubles())) != BA_OK) {
        dfree(buf);
        return st;
    }
    float *hid = buf, *gpre = hid + (size_t)rows * 128, *out = gpre + (size_t)rows * 128, *gout = out + (size_t)rows * 72;
    launch_mlp_forward(params, F, rows, out, hid, 0, q);
    launch_probe_loss_grad(n, n_probes, out, W, Sw, work, gout, q);
    launch_mlp_backward(params, F, hid, gout, gpre, rows, grad, q);
    double lsum = 0.0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        const int ne = 8 * 8;
        const double *res = work + (size_t)kRedBlocks * ne + ne + kRedBlocks + (size_t)kRedBlocks * ne;
        e = hipMemcpyAsync(&lsum, res, sizeof(double), hipMemcpyDeviceToHost, q);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(q);
    dfree(buf);
    dfree(work);
    if (e != hipSuccess) return fail(BA_ERR_HIP, std::string("ba_mlp_loss_grad: ") + hipGetErrorString(e));
    if (loss) *loss = lsum / ((double)n_probes * (double)n);
    return BA_OK;
}

ba_status ba_adam_step(float *params, const float *grad, float *m, float *v, int32_t t, float lr, void *stream) {
    if (!params || !grad || !m || !v || t < 1 || !(lr > 0.f)) return fail(BA_ERR_INVALID_ARG, "ba_adam_step: bad argument");
    hipStream_t q = (hipStream_t)stream;
    launch_adam(params, grad, m, v, t, lr, q);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(q));
    return BA_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
//
// A batch is one block-diagonal system over the concatenated problems (tiles and
// chunks never mix problems), solved by Algorithm 2 per problem with all state on
// the device: an iteration is a fixed launch sequence (no read-back), enqueued
// eagerly or captured into a graph window by window; the host looks at the
// per-problem stop flags once per window.

struct ba_batch {
    ba_system *sys = nullptr;
    int B = 0;
    std::vector<int32_t> cam0, np;
    // workspace for (N, cap)
    int N = 0;
    int64_t cap = 0;
    BatchProb *prob = nullptr;
    BatchDyn *dyn = nullptr;
    int32_t *skip_single = nullptr, *skip_multi = nullptr, *off = nullptr, *count = nullptr;
    double *alpha = nullptr, *gamma = nullptr, *gpart = nullptr, *upart = nullptr, *resid = nullptr;
    double *r = nullptr, *z = nullptr, *pstage = nullptr, *qstage = nullptr, *Y = nullptr;
    double *Ph = nullptr, *Qh = nullptr, *Dp = nullptr, *Phi = nullptr, *beta = nullptr;
    int32_t *blk_off = nullptr, *blk_k = nullptr;
    int64_t *blk_dp = nullptr;
    double *btp = nullptr, *d = nullptr, *tmp = nullptr, *xprev = nullptr;
    int32_t *mask = nullptr;        // [B] problems a restart or refinement step applies to
    int32_t *mask_skip = nullptr;   // [B] 1 - mask: the S products of such a step skip the others
    int32_t *max_it = nullptr;      // [B] iterations each problem's next inner solve may take
    // the window of iterations captured once and replayed; its kernels read every bound they
    // need from the device, so the graph only depends on the arguments in the key
    hipGraphExec_t gexec = nullptr;
    struct GraphKey {
        const double *x = nullptr;
        int precision = -1, window = 0, N = 0;
        double tau = 0.0, eps = 0.0;
        int64_t cap = 0;
        bool operator==(const GraphKey &o) const {
            return x == o.x && precision == o.precision && window == o.window && N == o.N && tau == o.tau &&
                   eps == o.eps && cap == o.cap;
        }
    } gkey;
    int32_t *host_i = nullptr;      // pinned
    double *host_d = nullptr;       // pinned [2B]
    // graph windows are captured on a stream of the batch (the caller's stream may be
    // the legacy default stream, which cannot be captured), ordered by events
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

namespace {

void free_batch_ws(ba_batch *b) {
    dfree(b->prob);
    dfree(b->dyn);
    dfree(b->skip_single);
    dfree(b->skip_multi);
    dfree(b->off);
    dfree(b->count);
    dfree(b->alpha);
    dfree(b->gamma);
    dfree(b->gpart);
    dfree(b->upart);
    dfree(b->resid);
    dfree(b->r);
    dfree(b->z);
    dfree(b->pstage);
    dfree(b->qstage);
    dfree(b->Y);
    dfree(b->Ph);
    dfree(b->Qh);
    dfree(b->Dp);
    dfree(b->Phi);
    dfree(b->beta);
    dfree(b->blk_off);
    dfree(b->blk_k);
    dfree(b->blk_dp);
    dfree(b->btp);
    dfree(b->d);
    dfree(b->tmp);
    dfree(b->xprev);
    dfree(b->mask);
    dfree(b->mask_skip);
    dfree(b->max_it);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->gkey = ba_batch::GraphKey();
    b->N = 0;
    b->cap = 0;
}

ba_status ensure_batch_ws(ba_batch *b, int N, int64_t cap) {
    if (b->N == N && b->cap >= cap && b->prob) return BA_OK;
    free_batch_ws(b);
    const int B = b->B;
    const int64_t ntot = (int64_t)b->sys->np * 9;
    std::vector<BatchProb> hp((size_t)B);
    int64_t hb = 0, cb = 0;
    for (int i = 0; i < B; ++i) {
        BatchProb &p = hp[(size_t)i];
        p.row0 = (int64_t)b->cam0[(size_t)i] * 9;
        p.n = b->np[(size_t)i] * 9;
        p.np = b->np[(size_t)i];
        p.cam0 = b->cam0[(size_t)i];
        p.gs = std::max(1, p.np / N);
        p.cap = (int32_t)cap;
        p.hbase = hb;
        p.colbase = cb;
        p.pad = 0;
        hb += cap * (int64_t)p.n;
        cb += cap;
    }
    hipStream_t q = b->sys->stream;
    ba_status st;
    if ((st = upload(&b->prob, hp, q)) != BA_OK) return st;
    if ((st = dalloc(&b->dyn, (size_t)B)) != BA_OK) return st;
    if ((st = dalloc(&b->skip_single, (size_t)B)) != BA_OK) return st;
    if ((st = dalloc(&b->skip_multi, (size_t)B)) != BA_OK) return st;
    if ((st = dalloc(&b->off, (size_t)B)) != BA_OK) return st;
    if ((st = dalloc(&b->count, 1)) != BA_OK) return st;
    if ((st = dalloc(&b->alpha, (size_t)B * kMaxBlock)) != BA_OK) return st;
    if ((st = dalloc(&b->gamma, (size_t)B * kMaxBlock)) != BA_OK) return st;
    if ((st = dalloc(&b->gpart, (size_t)B * kBatchGramBlocks * (size_t)(N * N + N))) != BA_OK) return st;
    if ((st = dalloc(&b->upart, (size_t)B * kBatchVecBlocks * 2)) != BA_OK) return st;
    if ((st = dalloc(&b->resid, (size_t)B * 2)) != BA_OK) return st;
    for (double **v : {&b->r, &b->z, &b->pstage, &b->qstage, &b->btp, &b->d, &b->tmp, &b->xprev})
        if ((st = dalloc(v, (size_t)ntot)) != BA_OK) return st;
    if ((st = dalloc(&b->Y, (size_t)ntot * N)) != BA_OK) return st;
    if ((st = dalloc(&b->Ph, (size_t)hb)) != BA_OK) return st;
    if ((st = dalloc(&b->Qh, (size_t)hb)) != BA_OK) return st;
    if ((st = dalloc(&b->Dp, (size_t)cb * N)) != BA_OK) return st;
    if ((st = dalloc(&b->Phi, (size_t)cb * N)) != BA_OK) return st;
    if ((st = dalloc(&b->beta, (size_t)cb * hist_ldb(N))) != BA_OK) return st;
    if ((st = dalloc(&b->blk_off, (size_t)cb)) != BA_OK) return st;
    if ((st = dalloc(&b->blk_k, (size_t)cb)) != BA_OK) return st;
    if ((st = dalloc(&b->blk_dp, (size_t)cb)) != BA_OK) return st;
    if ((st = dalloc(&b->mask, (size_t)B)) != BA_OK) return st;
    if ((st = dalloc(&b->mask_skip, (size_t)B)) != BA_OK) return st;
    if ((st = dalloc(&b->max_it, (size_t)B)) != BA_OK) return st;
    HIPCHK(hipStreamSynchronize(q));   // hp goes out of scope
    b->N = N;
    b->cap = cap;
    return BA_OK;
}

BatchLaunch batch_launch(ba_batch *b, double *x) {
    BatchLaunch L;
    L.B = b->B;
    L.N = b->N;
    for (int i = 0; i < b->B; ++i) {
        L.max_np = std::max(L.max_np, b->np[(size_t)i]);
        L.max_n = std::max<int64_t>(L.max_n, (int64_t)b->np[(size_t)i] * 9);
    }
    L.ntot = (int64_t)b->sys->np * 9;
    L.prob = b->prob;
    L.dyn = b->dyn;
    L.Dchol = b->sys->Dchol;
    L.x = x;
    L.r = b->r;
    L.z = b->z;
    L.pstage = b->pstage;
    L.qstage = b->qstage;
    L.Y = b->Y;
    L.Ph = b->Ph;
    L.Qh = b->Qh;
    L.Dp = b->Dp;
    L.Phi = b->Phi;
    L.beta = b->beta;
    L.alpha = b->alpha;
    L.gamma = b->gamma;
    L.gpart = b->gpart;
    L.upart = b->upart;
    L.blk_off = b->blk_off;
    L.blk_k = b->blk_k;
    L.blk_dp = b->blk_dp;
    L.skip_single = b->skip_single;
    L.skip_multi = b->skip_multi;
    return L;
}

// one iteration of Algorithm 2 for every running problem: the same launches whatever the
// iteration, the per-problem widths and bounds are read on the device
void batch_iteration(const BatchLaunch &L, const SchurArgs &sa, const MultiArgs &ma, double tau, double eps,
                     hipStream_t q) {
    launch_biter_head(L, tau, eps, q);
    if (L.N > 1) launch_schur_multi(ma, L.z, L.Y, q);
    launch_biter_tail(L, q);
    launch_schur_matvec(sa, L.pstage, L.qstage, q);
    launch_bqcopy_advance(L, q);
}

struct BatchRun {
    BatchLaunch L;
    SchurArgs sa;     // one-column product, skipping problems by their flags
    MultiArgs ma;
};

BatchRun batch_run(ba_batch *b, int precision, double *x) {
    ba_system *s = b->sys;
    BatchRun R;
    R.L = batch_launch(b, x);
    R.sa = schur_args(s, precision);
    R.sa.chunk_seg = s->seg_chunk;
    R.sa.cam_seg = s->seg_cam;
    R.sa.seg_skip = b->skip_single;
    R.ma = b->N > 1 ? multi_args(s, precision) : MultiArgs();
    if (b->N > 1) {
        R.ma.chunk_seg = s->multi.chunk_seg;
        R.ma.cam_seg = s->seg_cam;
        R.ma.seg_skip = b->skip_multi;
    }
    return R;
}

// (Re)starts Algorithm 2 on S x = -bt: every problem not flagged in `off` (only == NULL),
// or just the problems flagged in `only`, whose state is reset; each may take max_it[b]
// iterations (max_iter when max_it is NULL).  P_0 = D^-1 r_0 and Q_0 = S P_0.
ba_status batch_start(ba_batch *b, const BatchRun &R, const double *bt, const int32_t *off, const int32_t *only,
                      const int32_t *only_skip, int max_iter, const int32_t *max_it) {
    hipStream_t q = b->sys->stream;
    launch_bstart(R.L, bt, nullptr, off, q, only, max_iter, max_it);
    SchurArgs s0 = R.sa;
    if (only) s0.seg_skip = only_skip;   // the problems that keep running are left alone
    launch_schur_matvec(s0, R.L.pstage, R.L.qstage, q);
    launch_bqcopy_advance(R.L, q, only);
    HIPCHK(hipGetLastError());
    return BA_OK;
}

// `window` iterations for every running problem: replays of one captured graph (window >
// 0; captured on the batch's stream on first use for these arguments) or eager launches
ba_status batch_window(ba_batch *b, const BatchRun &R, int precision, double tau, double eps, int window) {
    hipStream_t q = b->sys->stream;
    if (window <= 0) {
        for (int k = 0; k < 8; ++k) batch_iteration(R.L, R.sa, R.ma, tau, eps, q);
        HIPCHK(hipGetLastError());
        return BA_OK;
    }
    ba_batch::GraphKey key;
    key.x = R.L.x;
    key.precision = precision;
    key.window = window;
    key.N = b->N;
    key.tau = tau;
    key.eps = eps;
    key.cap = b->cap;
    hipStream_t gs = b->gstream;
    if (!b->gexec || !(b->gkey == key)) {
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < window; ++k) batch_iteration(R.L, R.sa, R.ma, tau, eps, gs);
        hipError_t e = hipStreamEndCapture(gs, &g);
        if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->gexec = nullptr;
            return fail(BA_ERR_HIP, std::string("batch graph: ") + hipGetErrorString(e));
        }
        b->gkey = key;
    }
    HIPCHK(hipEventRecord(b->ev_in, q));
    HIPCHK(hipStreamWaitEvent(gs, b->ev_in, 0));
    HIPCHK(hipGraphLaunch(b->gexec, gs));
    HIPCHK(hipEventRecord(b->ev_out, gs));
    HIPCHK(hipStreamWaitEvent(q, b->ev_out, 0));
    return BA_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

ba_status batch_stats_from_device(ba_batch *b, std::vector<BatchDyn> &hd) {
    hd.resize((size_t)b->B);
    HIPCHK(hipMemcpyAsync(hd.data(), b->dyn, sizeof(BatchDyn) * (size_t)b->B, hipMemcpyDeviceToHost, b->sys->stream));
    HIPCHK(hipStreamSynchronize(b->sys->stream));
    return BA_OK;
}

// per-problem true relative residual |bt + S x| / |bt| in FP64; btp = bt + S x when given.
// With `only` (device mask, and only_skip its complement), just the flagged problems:
// the FP64 product skips the others and rel keeps their entries.
ba_status batch_true_residual(ba_batch *b, const double *x, double *btp, std::vector<double> &rel,
                              const int32_t *only = nullptr, const int32_t *only_skip = nullptr,
                              const std::vector<int32_t> *only_h = nullptr) {
    ba_system *s = b->sys;
    hipStream_t q = s->stream;
    BatchLaunch L = batch_launch(b, nullptr);
    SchurArgs a = schur_args(s, 0);
    if (only) {
        a.chunk_seg = s->seg_chunk;
        a.cam_seg = s->seg_cam;
        a.seg_skip = only_skip;
    }
    launch_schur_matvec(a, x, b->tmp, q);
    launch_bresidual(L, s->bt, b->tmp, btp, b->resid, q, only);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(b->host_d, b->resid, sizeof(double) * 2 * (size_t)b->B, hipMemcpyDeviceToHost, q));
    HIPCHK(hipStreamSynchronize(q));
    rel.resize((size_t)b->B, 0.0);
    for (int i = 0; i < b->B; ++i) {
        if (only_h && !(*only_h)[(size_t)i]) continue;
        const double a0 = b->host_d[2 * i], a1 = b->host_d[2 * i + 1];
        rel[(size_t)i] = a1 > 0.0 ? std::sqrt(a0 / a1) : 0.0;
    }
    return BA_OK;
}

// Uploads a per-problem mask and its complement (the S products' skip flags).
ba_status batch_set_mask(ba_batch *b, const std::vector<int32_t> &m, std::vector<int32_t> &skip_h) {
    hipStream_t q = b->sys->stream;
    skip_h.resize(m.size());
    for (size_t i = 0; i < m.size(); ++i) skip_h[i] = m[i] ? 0 : 1;
    HIPCHK(hipMemcpyAsync(b->mask, m.data(), sizeof(int32_t) * m.size(), hipMemcpyHostToDevice, q));
    HIPCHK(hipMemcpyAsync(b->mask_skip, skip_h.data(), sizeof(int32_t) * m.size(), hipMemcpyHostToDevice, q));
    return BA_OK;
}

}  // namespace

extern "C" {

ba_status ba_batch_build(const ba_problem_desc *all, int32_t n_problems, const int32_t *cams_per_problem,
                         const ba_build_opts *opts, void *stream, ba_batch **out) {
    if (!out) return fail(BA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!all || !cams_per_problem || n_problems < 1) return fail(BA_ERR_INVALID_ARG, "empty batch");
    std::vector<int32_t> seg((size_t)std::max(all->n_cams, 0));
    ba_batch *b = new ba_batch();
    b->B = n_problems;
    int64_t c0 = 0;
    for (int i = 0; i < n_problems; ++i) {
        const int c = cams_per_problem[i];
        if (c < 1 || c0 + c > all->n_cams) {
            delete b;
            return fail(BA_ERR_INVALID_ARG, "camera counts of the batch do not add up to n_cams");
        }
        b->cam0.push_back((int32_t)c0);
        b->np.push_back(c);
        for (int k = 0; k < c; ++k) seg[(size_t)(c0 + k)] = i;
        c0 += c;
    }
    if (c0 != all->n_cams) {
        delete b;
        return fail(BA_ERR_INVALID_ARG, "camera counts of the batch do not add up to n_cams");
    }
    ba_status st = build_system(all, opts, stream, seg.data(), &b->sys);
    if (st != BA_OK) {
        delete b;
        return st;
    }
    if (hipHostMalloc((void **)&b->host_i, sizeof(int32_t) * 4) != hipSuccess ||
        hipHostMalloc((void **)&b->host_d, sizeof(double) * 2 * (size_t)n_problems) != hipSuccess) {
        ba_batch_free(b);
        return fail(BA_ERR_NOMEM, "pinned host buffers");
    }
    if (hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        ba_batch_free(b);
        return fail(BA_ERR_HIP, "batch stream or events");
    }
    *out = b;
    return BA_OK;
}

void ba_batch_free(ba_batch *b) {
    if (!b) return;
    if (b->sys) (void)hipStreamSynchronize(b->sys->stream);
    free_batch_ws(b);
    if (b->host_i) (void)hipHostFree(b->host_i);
    if (b->host_d) (void)hipHostFree(b->host_d);
    if (b->gstream) {
        (void)hipStreamSynchronize(b->gstream);
        (void)hipStreamDestroy(b->gstream);
    }
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    ba_free_system(b->sys);
    delete b;
}

ba_system *ba_batch_system(ba_batch *b) { return b ? b->sys : nullptr; }

ba_status ba_explicit_schur_info(const ba_system *s, int64_t *nnz_blocks, int64_t *bytes, double *assembly_ms) {
    if (!s) return fail(BA_ERR_INVALID_ARG, "sys is NULL");
    if (!s->bsr_val) return fail(BA_ERR_INVALID_ARG, "the system was built without the explicit S");
    if (nnz_blocks) *nnz_blocks = s->bsr_nnzb;
    if (bytes) *bytes = s->bsr_nnzb * 81 * (int64_t)sizeof(double);
    if (assembly_ms) *assembly_ms = s->bsr_build_ms;
    return BA_OK;
}

ba_status ba_batch_mcg_solve(ba_batch *b, int32_t N, double tau, double *x, const ba_solve_opts *opts_in,
                             int32_t graph_window, ba_batch_stats *stats, double *elapsed_ms) {
    if (!b || !x) return fail(BA_ERR_INVALID_ARG, "NULL argument");
    ba_solve_opts opts;
    ba_status st = check_opts(opts_in, &opts);
    if (st != BA_OK) return st;
    if (opts.precond != 0) return fail(BA_ERR_UNSUPPORTED, "batches use the block-Jacobi preconditioner");
    int min_np = b->np[0];
    for (int i = 1; i < b->B; ++i) min_np = std::min(min_np, b->np[(size_t)i]);
    if (N < 1 || N > kMaxBlock || N > min_np) return fail(BA_ERR_INVALID_ARG, "N must be in [1, min(64, cameras of every problem)]");
    if (!(tau >= 0.0) || graph_window < 0) return fail(BA_ERR_INVALID_ARG, "tau >= 0 and graph_window >= 0 required");
    ba_system *s = b->sys;
    hipStream_t q = s->stream;
    if ((st = ensure_precision(s, opts.precision)) != BA_OK) return st;
    if (N > 1 && (st = ensure_multi(s, N)) != BA_OK) return st;
    const int inner_max = opts.precision == 0 ? opts.max_iter : std::min(opts.max_inner, opts.max_iter);
    const int64_t cap = opts.max_history_cols > 0 ? opts.max_history_cols : 1 + (int64_t)inner_max * N;
    if ((st = ensure_batch_ws(b, N, cap)) != BA_OK) return st;
    const int B = b->B;
    std::vector<double> done_ms((size_t)B, 0.0), rel((size_t)B, 0.0);
    std::vector<int32_t> iters((size_t)B, 0), multis((size_t)B, 0), outer((size_t)B, 0), status((size_t)B, BA_MAXITER);
    std::vector<int32_t> hcols((size_t)B, 0);
    std::vector<double> rrel((size_t)B, 0.0);
    std::vector<BatchDyn> hd((size_t)B);
    const int W = graph_window > 0 ? graph_window : 8;   // iterations between reads of the stop flags
    auto t0 = std::chrono::steady_clock::now();
    auto read_dyn = [&]() -> ba_status {
        HIPCHK(hipMemcpyAsync(hd.data(), b->dyn, sizeof(BatchDyn) * (size_t)B, hipMemcpyDeviceToHost, q));
        HIPCHK(hipStreamSynchronize(q));
        return BA_OK;
    };
    auto note_inner = [&](int i) {
        const BatchDyn &d = hd[(size_t)i];
        iters[(size_t)i] += d.iters;
        multis[(size_t)i] += d.multi_steps;
        hcols[(size_t)i] = d.hcols;
        rrel[(size_t)i] = d.rr0 > 0.0 ? std::sqrt(d.rr / d.rr0) : 0.0;
    };
    if (opts.precision == 0) {
        // one Algorithm 2 run per problem on S x = -b~; a problem's time is the end of the
        // window in which its stop flag was first seen
        BatchRun R = batch_run(b, 0, x);
        if ((st = batch_start(b, R, s->bt, nullptr, nullptr, nullptr, opts.max_iter, nullptr)) != BA_OK) return st;
        std::vector<int32_t> seen((size_t)B, 0);
        for (int it = 0;; it += W) {
            if ((st = read_dyn()) != BA_OK) return st;
            const double ms = ms_since(t0);
            int running = 0;
            for (int i = 0; i < B; ++i) {
                if (hd[(size_t)i].done && !seen[(size_t)i]) {
                    seen[(size_t)i] = 1;
                    done_ms[(size_t)i] = ms;
                }
                running += !hd[(size_t)i].done;
            }
            if (running == 0 || it >= opts.max_iter) break;
            if ((st = batch_window(b, R, 0, tau, opts.eps, graph_window)) != BA_OK) return st;
        }
        for (int i = 0; i < B; ++i) {
            note_inner(i);
            status[(size_t)i] = hd[(size_t)i].status;
        }
        if ((st = batch_true_residual(b, x, nullptr, rel)) != BA_OK) return st;
    } else {
        // FP64 iterative refinement around reduced-precision inner solves, each problem on
        // its own: when a problem's inner solve stops, its correction is added and its FP64
        // residual formed at once (the others keep iterating); it then either retires or
        // restarts its inner solve on the new residual
        // one tolerance for every problem of a window (the graph's kernels take it as an
        // argument): no per-problem raise of the last step, so FP32 keeps 1e-2 here
        const double ieps = opts.inner_eps > 0.0 ? opts.inner_eps : (opts.precision == BA_PREC_FP32 ? 1e-2 : 1e-1);
        HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * (size_t)s->np * 9, q));
        BatchRun R = batch_run(b, opts.precision, b->d);
        // host copies of the masks: one vector per upload in flight (pageable sources)
        std::vector<int32_t> live((size_t)B, 0), sel((size_t)B, 0), cap_h((size_t)B, inner_max);
        std::vector<int32_t> skip_sel, skip_rev, skip_again;
        std::vector<double> prev((size_t)B, INFINITY);
        // x = 0: btp = b~, every relative residual 1 (0 for a zero right-hand side)
        if ((st = batch_true_residual(b, x, b->btp, rel)) != BA_OK) return st;
        int running = 0;
        for (int i = 0; i < B; ++i) {
            if (rel[(size_t)i] < opts.eps) {
                status[(size_t)i] = BA_OK;
                done_ms[(size_t)i] = ms_since(t0);
            } else {
                live[(size_t)i] = 1;
                ++running;
            }
            prev[(size_t)i] = rel[(size_t)i];
        }
        auto restart = [&](const std::vector<int32_t> &m) -> ba_status {
            ba_status r2;
            if ((r2 = batch_set_mask(b, m, skip_again)) != BA_OK) return r2;
            HIPCHK(hipMemcpyAsync(b->max_it, cap_h.data(), sizeof(int32_t) * (size_t)B, hipMemcpyHostToDevice, q));
            return batch_start(b, R, b->btp, nullptr, b->mask, b->mask_skip, inner_max, b->max_it);
        };
        if (running > 0) {
            // the first start resets every problem (those already at eps stay stopped)
            std::vector<int32_t> offh((size_t)B);
            for (int i = 0; i < B; ++i) offh[(size_t)i] = !live[(size_t)i];
            HIPCHK(hipMemcpyAsync(b->off, offh.data(), sizeof(int32_t) * (size_t)B, hipMemcpyHostToDevice, q));
            HIPCHK(hipMemcpyAsync(b->max_it, cap_h.data(), sizeof(int32_t) * (size_t)B, hipMemcpyHostToDevice, q));
            if ((st = batch_start(b, R, b->btp, b->off, nullptr, nullptr, inner_max, b->max_it)) != BA_OK) return st;
            HIPCHK(hipStreamSynchronize(q));   // offh goes out of scope
        }
        std::vector<int32_t> reverted((size_t)B, 0), again_h((size_t)B, 0);
        while (running > 0) {
            if ((st = batch_window(b, R, opts.precision, tau, ieps, graph_window)) != BA_OK) return st;
            if ((st = read_dyn()) != BA_OK) return st;
            // the problems whose inner solve stopped in this window
            int nsel = 0;
            for (int i = 0; i < B; ++i) {
                sel[(size_t)i] = live[(size_t)i] && hd[(size_t)i].done;
                if (!sel[(size_t)i]) continue;
                note_inner(i);
                outer[(size_t)i] += 1;
                const int32_t ist = hd[(size_t)i].status;
                if (ist < 0 && ist != BA_ERR_BREAKDOWN) {   // an error ends this problem, x unchanged
                    status[(size_t)i] = ist;
                    live[(size_t)i] = 0;
                    sel[(size_t)i] = 0;
                    done_ms[(size_t)i] = ms_since(t0);
                    --running;
                    continue;
                }
                ++nsel;
            }
            if (nsel == 0) continue;
            // x += d on those problems (xprev keeps x), then their FP64 residuals
            if ((st = batch_set_mask(b, sel, skip_sel)) != BA_OK) return st;
            launch_bouter_step(R.L, b->mask, x, b->d, b->xprev, q);
            if ((st = batch_true_residual(b, x, b->btp, rel, b->mask, b->mask_skip, &sel)) != BA_OK) return st;
            const double ms = ms_since(t0);
            int nrev = 0, nre = 0;
            std::vector<int32_t> &again = again_h;
            std::fill(again.begin(), again.end(), 0);
            for (int i = 0; i < B; ++i) {
                reverted[(size_t)i] = 0;
                if (!sel[(size_t)i]) continue;
                bool retire = true;
                if (rel[(size_t)i] < opts.eps) {
                    status[(size_t)i] = BA_OK;
                } else if (!(rel[(size_t)i] < prev[(size_t)i])) {
                    // the correction did not reduce this problem's FP64 residual: keep its
                    // iterate from before it
                    reverted[(size_t)i] = 1;
                    ++nrev;
                    rel[(size_t)i] = prev[(size_t)i];
                    status[(size_t)i] = BA_MAXITER;
                } else if (outer[(size_t)i] >= opts.max_outer || iters[(size_t)i] >= opts.max_iter) {
                    status[(size_t)i] = BA_MAXITER;
                } else {
                    retire = false;
                    again[(size_t)i] = 1;
                    ++nre;
                    // the inner solve may take what is left of the problem's budget
                    cap_h[(size_t)i] = std::min(inner_max, opts.max_iter - iters[(size_t)i]);
                }
                prev[(size_t)i] = rel[(size_t)i];
                if (retire) {
                    live[(size_t)i] = 0;
                    done_ms[(size_t)i] = ms;
                    --running;
                }
            }
            if (nrev > 0) {
                if ((st = batch_set_mask(b, reverted, skip_rev)) != BA_OK) return st;
                launch_brevert(R.L, b->mask, x, b->xprev, q);
                HIPCHK(hipGetLastError());
            }
            if (nre > 0 && (st = restart(again)) != BA_OK) return st;
            HIPCHK(hipStreamSynchronize(q));   // the host masks are rewritten next window
        }
    }
    HIPCHK(hipStreamSynchronize(q));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (elapsed_ms) *elapsed_ms = ms;
    int worst = BA_OK;
    for (int i = 0; i < B; ++i) {
        if (stats) {
            ba_batch_stats &o = stats[i];
            o.iterations = iters[(size_t)i];
            o.multi_steps = multis[(size_t)i];
            o.history_cols = hcols[(size_t)i];
            o.refinement_steps = outer[(size_t)i];
            o.status = status[(size_t)i];
            o.reserved = 0;
            o.rel_res_recursive = rrel[(size_t)i];
            o.rel_res_true = rel[(size_t)i];
            o.done_ms = done_ms[(size_t)i] > 0.0 ? done_ms[(size_t)i] : ms;
        }
        if (status[(size_t)i] < 0) worst = std::min(worst, status[(size_t)i]);
        else if (status[(size_t)i] == BA_MAXITER && worst == BA_OK) worst = BA_MAXITER;
    }
    return (ba_status)worst;
}

}  // extern "C"
