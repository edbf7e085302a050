// Internal declarations of the reduced-camera-system library (gfx950).
//
// Layout of the Jacobian stream in HBM ("tiles"):
//   Observations are grouped by landmark; landmarks are packed into tiles of
//   64 observation slots (one slot per lane of a wavefront) without straddling
//   a tile boundary; unused slots are padding.  A tile stores its 24 Jacobian
//   scalars per observation component-pair-major: for pair q (0..11) and lane l
//   the two doubles J[2q], J[2q+1] sit at ((tile*12 + q)*64 + l)*2, so a
//   wavefront loads each pair with one fully coalesced 1 KiB access.
//   Components 0..17 are J_p (2x9 row-major), 18..23 are J_l (2x3 row-major).
//   Consecutive tiles form a "chunk", processed by one wavefront, whose
//   cameras are numbered by chunk-local slots; the wavefront accumulates its
//   camera contributions in LDS and writes one partial row per slot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ba.h"

namespace ba {

constexpr int kTile = 64;          // observation slots per tile (= wavefront width)
constexpr int kPairs = 12;         // 16-byte component pairs per observation
constexpr uint32_t kPad = 0xFFFFFFFFu;

// Per-slot metadata word: bits 0..15 chunk-local camera slot, bits 16..21 the
// landmark's index inside its tile.  Padding slots hold kPad.
__host__ __device__ inline uint32_t meta_pack(uint32_t slot, uint32_t ll) { return slot | (ll << 16); }

struct HostPlan {
    int np = 0, nl = 0;
    int64_t m = 0;
    int64_t n_tiles = 0;
    int n_chunks = 0;
    int64_t n_part = 0;
    int max_slots = 128, max_tiles = 16;
    int max_tiles_multi = 16;             // tiles per chunk of the multidirectional product
    int max_used_slots = 0;               // most cameras of one chunk (sizes the chunk kernels' LDS)
    std::vector<int32_t> lmk_order;       // storage index -> landmark id
    std::vector<int32_t> lmk_store;       // landmark id -> storage index
    std::vector<int64_t> slot_obs;        // tile slot -> observation index or -1
    std::vector<uint32_t> meta;           // tile slot -> meta word
    std::vector<int32_t> tile_lmk_base;   // tile -> storage index of its first landmark
    std::vector<int64_t> lmk_first_slot;  // storage index -> first tile slot
    std::vector<int32_t> lmk_count;       // storage index -> observations
    std::vector<int32_t> chunk_tile;      // [n_chunks + 1]
    std::vector<int32_t> chunk_part;      // [n_chunks + 1] first partial row
    std::vector<int32_t> part_cam;        // partial row -> camera
    std::vector<int32_t> cam_part_ptr;    // [np + 1]
    std::vector<int32_t> cam_part_idx;    // partial rows, camera-major, ascending
    std::vector<int32_t> part_dst;        // partial row -> its position in camera-major order
    std::vector<int64_t> cam_obs_ptr;     // [np + 1]
    std::vector<int64_t> cam_obs;         // observation indices, camera-major
    std::vector<int32_t> obs_cam;         // host copy of the camera of each observation
    // batches: problem of every camera (nondecreasing), of every tile and of every chunk;
    // tiles and chunks never mix problems.  Empty for a single problem.
    std::vector<int32_t> cam_seg, tile_seg, chunk_seg;
};

// Plan of the multidirectional product for one partition (N subsets).
struct HostMultiPlan {
    int N = 0;
    int n_chunks = 0;
    int64_t n_part = 0;
    int max_out = 0;                      // largest out-pair count of a chunk
    std::vector<uint32_t> mmeta;          // tile slot -> own pair | first pair << 8 | pairs << 16
    std::vector<int32_t> slot_cam;        // tile slot -> camera (0 for padding)
    std::vector<uint8_t> pair_ll;         // tile * 64 + pair -> landmark index in tile
    std::vector<uint32_t> tile_oidx;      // [n_tiles + 1] first entry of the tile in oidx
    std::vector<uint16_t> oidx;           // (slot, j-th pair of its landmark) -> chunk out-pair
    std::vector<uint16_t> slot_ooff;      // tile slot -> offset of its entries in the tile's oidx
    std::vector<int32_t> chunk_tile;      // [n_chunks + 1]
    std::vector<int32_t> chunk_part;      // [n_chunks + 1]
    std::vector<int32_t> cg_ptr;          // [np * N + 1] partial rows of (camera, subset)
    std::vector<int32_t> cg_idx;
    std::vector<int32_t> part_dst;        // out-pair row -> position in (camera, subset)-major order
    std::vector<int32_t> chunk_seg;       // batches: problem of every chunk
};

struct DevMulti {
    int N = 0, n_chunks = 0, max_out = 0;
    int64_t n_part = 0;
    uint32_t *mmeta = nullptr;
    int32_t *slot_cam = nullptr;
    uint8_t *pair_ll = nullptr;
    uint32_t *tile_oidx = nullptr;
    uint16_t *oidx = nullptr;
    uint16_t *slot_ooff = nullptr;
    int32_t *chunk_tile = nullptr, *chunk_part = nullptr;
    int32_t *cg_ptr = nullptr, *cg_idx = nullptr, *part_dst = nullptr;
    double *partial = nullptr;
    int32_t *group = nullptr;             // camera -> subset
    int32_t *chunk_seg = nullptr;         // batches: chunk -> problem
};

// Plan construction (host, plan.cpp).  Returns BA_OK or an error with message.
// cam_seg (nullable, host, [np], nondecreasing): problem of every camera of a batch.
// max_tiles = 0: the S product's chunks take ceil(n_tiles / target_chunks) tiles each
// (16 when target_chunks is 0), so that all of them are resident at once.  The
// multidirectional product's chunks take max_tiles_multi tiles (0: max_tiles when it is
// set, else ceil(n_tiles / target_multi), else 16).
ba_status build_plan(int np, int nl, int64_t m, const int32_t *cam, const int32_t *lm,
                     int max_slots, int max_tiles, HostPlan &plan, std::string &err,
                     const int32_t *cam_seg = nullptr, int target_chunks = 0, int max_tiles_multi = 0,
                     int target_multi = 0);
// group (nullable, host, [np]): subset of every camera; default partition_groups(np, N)
ba_status build_multi_plan(const HostPlan &plan, int N, int max_out, HostMultiPlan &mp,
                           std::string &err, const int32_t *group = nullptr);
void partition_groups(int np, int N, int32_t *group);
void covisibility_degree(const HostPlan &plan, std::vector<int32_t> &deg);

// Records msg as the text of ba_last_error() and returns st.
ba_status set_error(ba_status st, const std::string &msg);
// Lays out what Algorithm 2 with N subsets needs on the system (the reduced-precision
// Jacobian copy, the partition, the multidirectional product's layout), ahead of the solves.
ba_status prepare_mcg(ba_system *s, int N, int precision);

struct SchurArgs;
// Arguments of the system's chunked S product in a precision (partial rows in the
// system's own buffer), and whether its FP64 products read the explicit S instead.
SchurArgs system_schur_args(ba_system *s, int precision);
bool system_uses_bsr(const ba_system *s, const SchurArgs &a);

}  // namespace ba

// The system handle.
struct ba_system {
    hipStream_t stream = nullptr;
    int device = 0;                 // HIP device current at the build
    int np = 0, nl = 0;
    int dp = 9;                     // pose dimension d_p (9, or 6 for extrinsics only)
    int64_t m = 0;
    double lambda = 0.0;
    ba::HostPlan plan;
    // device arrays
    double *J64 = nullptr;          // n_tiles * 64 * 24
    float *J32 = nullptr;           // optional FP32 copy
    uint16_t *J16 = nullptr;        // optional BF16 copy (scaled)
    uint32_t *meta = nullptr;
    int32_t *tile_lmk_base = nullptr;
    int32_t *chunk_tile = nullptr, *chunk_part = nullptr, *part_cam = nullptr;
    int32_t *cam_part_ptr = nullptr, *cam_part_idx = nullptr, *part_dst = nullptr;
    double *partial = nullptr;      // n_part * 9, camera-major
    double *vinv = nullptr;         // nl * 6 (storage order): V_lambda^-1, symmetric
    double *bl = nullptr;           // nl * 3 (storage order)
    double *dU = nullptr;           // np * 9: lambda * diag(J_p^T J_p)
    double *Dblk = nullptr;         // np * 81: D(S)
    double *Dchol = nullptr;        // np * 45: packed lower Cholesky factor of D(S)
    double *bt = nullptr;           // n: b~
    int32_t *lmk_order = nullptr;   // storage index -> landmark id
    int64_t *lmk_first_slot = nullptr;
    int32_t *lmk_count = nullptr;
    int32_t *status = nullptr;      // device status word
    // layout arrays of the build, kept for new values of the same observations
    int64_t *slot_obs = nullptr;    // tile slot -> observation (or -1)
    int64_t *cam_obs_ptr = nullptr; // camera -> range of cam_obs
    int64_t *cam_obs = nullptr;     // observations camera by camera
    int32_t *lmk_store = nullptr;   // observation -> storage index of its landmark
    int32_t *obs_lm = nullptr;      // copy of the observations' landmarks
    double *h0 = nullptr;           // nl * 3: V^-1 b_l (storage order)
    double *Vraw = nullptr;         // nl * 6: undamped J_l^T J_l (storage order)
    double *Uraw = nullptr;         // np * dp (dp + 1) / 2: undamped J_p^T J_p, packed upper triangle
    double *bp = nullptr;           // np * dp: b_p = J_p^T r0
    int64_t *obs_slot = nullptr;    // tile slot of every observation
    int32_t *bsr_slot_cam = nullptr;// explicit S: camera of every observation slot
    int bsr_max_row = 0;
    int bsr_piece = 0;              // explicit S: blocks of a row per assembly wavefront
    // solver scratch (allocated on demand)
    double *vec = nullptr;          // work vectors
    size_t vec_cap = 0;
    double *red = nullptr;          // reduction partials
    size_t red_cap = 0;
    double *hist = nullptr;         // MCG history (P then Q)
    int64_t hist_cap_cols = 0;
    double *hist32 = nullptr;       // FP32 copy of the history (P then Q, floats), mixed path
    int64_t hist32_cap = 0;         // doubles
    double *small = nullptr;        // MCG small dense storage
    uint32_t *tickets = nullptr;    // arrival counters of last-block reductions (zero between launches)
    int64_t tickets_cap = 0;
    double *hscratch = nullptr;     // split-K partials of the history products
    int64_t hscratch_cap = 0;       // doubles
    double *refine_buf = nullptr;   // mixed precision: outer residual, inner right-hand side, update
    size_t refine_cap = 0;
    double *trace_buf = nullptr;    // PCG residual trace
    int64_t trace_cap = 0;
    // caller-owned workspace (ba_build_system_ws): device memory comes from it
    char *ws_base = nullptr;
    size_t ws_size = 0, ws_used = 0;
    bool ws_counting = false;       // sizing pass (ba_build_workspace_bytes): count, allocate nothing
    double *Ulr = nullptr;          // learned low-rank preconditioner term, n x 8 (row-major), or null
    int32_t *degree = nullptr;      // covisibility degree per camera (learned features)
    double *lr_proj = nullptr;      // kRedBlocks x 8 projections U^T r
    size_t small_cap = 0;
    double *host_pinned = nullptr;  // pinned host scalars
    double *host_pinned_dev = nullptr;  // the same memory as kernels address it
    double sc_tag = 0.0;            // tag of the last scalars a kernel wrote to host_pinned[SC_COUNT]
    ba::DevMulti multi;
    // batches: problem of every camera and of every chunk of the S product (device)
    int32_t *seg_cam = nullptr, *seg_chunk = nullptr;
    // explicit S in block-sparse rows (optional)
    int32_t *bsr_ptr = nullptr, *bsr_col = nullptr;
    double *bsr_val = nullptr;
    int64_t bsr_nnzb = 0;
    double bsr_build_ms = 0.0;
    // optional event timing of the chunked Schur-product kernel
    bool profiling = false;
    int32_t prof_every = 1;         // time every prof_every-th product launch
    int64_t prof_calls = 0;
    std::vector<hipEvent_t> prof_events;  // start/stop pairs
    size_t prof_used = 0;                 // events recorded since the last flush
    double prof_ms = 0.0;
    int64_t prof_launches = 0;
};
