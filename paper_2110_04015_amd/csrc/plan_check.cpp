// Host-only validation of the HBM layout plan: rebuilds the plans from host
// index arrays and checks every invariant the kernels index by (slot and pair
// bounds, chunk capacities, landmark contiguity, reduction CSRs).  Used by the
// CPU test suite; needs no GPU.
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "ba_internal.h"

using namespace ba;

namespace {
thread_local std::string g_check_err;

bool bad(const char *what, int64_t a = 0, int64_t b = 0) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s (%lld, %lld)", what, (long long)a, (long long)b);
    g_check_err = buf;
    return false;
}

bool check_plan(const HostPlan &P, const int32_t *cam, const int32_t *lm) {
    const int64_t T = P.n_tiles;
    if ((int64_t)P.slot_obs.size() != T * kTile || (int64_t)P.meta.size() != T * kTile) return bad("slot arrays");
    std::vector<int> seen((size_t)P.m, 0);
    for (int64_t s = 0; s < T * kTile; ++s) {
        int64_t o = P.slot_obs[(size_t)s];
        if (o < -1 || o >= P.m) return bad("slot_obs range", s, o);
        if ((o < 0) != (P.meta[(size_t)s] == kPad)) return bad("padding mismatch", s, o);
        if (o >= 0 && seen[(size_t)o]++) return bad("observation placed twice", o);
    }
    for (int64_t o = 0; o < P.m; ++o)
        if (!seen[(size_t)o]) return bad("observation not placed", o);
    // every tile starts with a landmark (the kernels read V^-1 of the tile's first
    // landmark for padding slots)
    for (int64_t t = 0; t < T; ++t) {
        const int b = P.tile_lmk_base[(size_t)t];
        if (b < 0 || b >= P.nl || P.meta[(size_t)(t * kTile)] == kPad) return bad("tile without a landmark", t, b);
    }
    // landmarks: contiguous, inside one tile, consistent local index
    for (int s = 0; s < P.nl; ++s) {
        int64_t f = P.lmk_first_slot[(size_t)s];
        int c = P.lmk_count[(size_t)s];
        if (c < 1 || c > kTile) return bad("landmark count", s, c);
        int64_t t = f / kTile;
        if ((f + c - 1) / kTile != t) return bad("landmark straddles a tile", s, f);
        int l = P.lmk_order[(size_t)s];
        uint32_t ll = P.meta[(size_t)f] >> 16;
        if (ll >= (uint32_t)kTile) return bad("landmark index in tile", s, ll);
        if (P.tile_lmk_base[(size_t)t] + (int)ll != s) return bad("tile_lmk_base + ll != storage index", s, ll);
        for (int q = 0; q < c; ++q) {
            int64_t o = P.slot_obs[(size_t)(f + q)];
            if (o < 0 || lm[o] != l) return bad("slot holds another landmark", s, q);
            if ((P.meta[(size_t)(f + q)] >> 16) != ll) return bad("ll differs inside a landmark", s, q);
        }
    }
    // chunks
    if ((int)P.chunk_tile.size() != P.n_chunks + 1 || P.chunk_tile[0] != 0 || P.chunk_tile[(size_t)P.n_chunks] != T)
        return bad("chunk tile ranges");
    int max_used = 0;
    for (int ch = 0; ch < P.n_chunks; ++ch) {
        int t0 = P.chunk_tile[(size_t)ch], t1 = P.chunk_tile[(size_t)ch + 1];
        if (t1 <= t0 || t1 - t0 > P.max_tiles) return bad("chunk tile count", ch, t1 - t0);
        int pb = P.chunk_part[(size_t)ch], ns = P.chunk_part[(size_t)ch + 1] - pb;
        if (ns < 1 || ns > P.max_slots) return bad("chunk slot count", ch, ns);
        if (ns > max_used) max_used = ns;
        std::vector<int> used((size_t)ns, 0);
        for (int64_t s = (int64_t)t0 * kTile; s < (int64_t)t1 * kTile; ++s) {
            if (P.meta[(size_t)s] == kPad) continue;
            int slot = (int)(P.meta[(size_t)s] & 0xFFFFu);
            if (slot >= ns) return bad("slot beyond chunk", ch, slot);
            if (P.part_cam[(size_t)(pb + slot)] != cam[P.slot_obs[(size_t)s]]) return bad("slot camera", ch, slot);
            used[(size_t)slot] = 1;
        }
        for (int k = 0; k < ns; ++k)
            if (!used[(size_t)k]) return bad("unused slot", ch, k);
    }
    // camera CSR over partial rows
    if ((int64_t)P.cam_part_idx.size() != P.n_part || P.cam_part_ptr[(size_t)P.np] != P.n_part)
        return bad("partial CSR size");
    for (int c = 0; c < P.np; ++c) {
        for (int j = P.cam_part_ptr[(size_t)c]; j < P.cam_part_ptr[(size_t)c + 1]; ++j) {
            int row = P.cam_part_idx[(size_t)j];
            if (row < 0 || row >= P.n_part || P.part_cam[(size_t)row] != c) return bad("partial CSR row", c, row);
            if (j > P.cam_part_ptr[(size_t)c] && row <= P.cam_part_idx[(size_t)j - 1]) return bad("CSR order", c, j);
            if (P.part_dst[(size_t)row] != j) return bad("partial destination", row, j);
        }
    }
    return true;
}

bool check_multi(const HostPlan &P, const HostMultiPlan &M, const int32_t *cam) {
    const int N = M.N;
    std::vector<int32_t> group((size_t)P.np);
    partition_groups(P.np, N, group.data());
    const int64_t T = P.n_tiles;
    if ((int)M.chunk_tile.size() != M.n_chunks + 1 || M.chunk_tile[(size_t)M.n_chunks] != T)
        return bad("multi chunk ranges");
    std::vector<int64_t> part_key((size_t)M.n_part, -1);
    for (int ch = 0; ch < M.n_chunks; ++ch) {
        int pb = M.chunk_part[(size_t)ch], no = M.chunk_part[(size_t)ch + 1] - pb;
        if (no < 1 || no > M.max_out) return bad("multi chunk out count", ch, no);
        for (int t = M.chunk_tile[(size_t)ch]; t < M.chunk_tile[(size_t)ch + 1]; ++t) {
            // the product loads a tile's first output-row entry with the tile, for every
            // lane, padding lanes included: every tile's list holds at least one entry
            if (M.tile_oidx[(size_t)t + 1] <= M.tile_oidx[(size_t)t] || M.tile_oidx[(size_t)t] >= M.oidx.size())
                return bad("empty tile output list", t);
            // pairs of the tile
            std::vector<int> pair_grp(kTile, -1);
            for (int q = 0; q < kTile; ++q) {
                size_t s = (size_t)((int64_t)t * kTile + q);
                if (P.slot_obs[s] < 0) {
                    if (M.mmeta[s] != kPad) return bad("multi padding", t, q);
                    continue;
                }
                int c = cam[P.slot_obs[s]];
                if (M.slot_cam[s] != c) return bad("slot_cam", t, q);
                uint32_t mm = M.mmeta[s];
                int own = mm & 0xFF, base = (mm >> 8) & 0xFF, cnt = (mm >> 16) & 0xFF;
                if (own < base || own >= base + cnt || base + cnt > kTile) return bad("pair range", t, q);
                uint8_t pll = M.pair_ll[(size_t)((int64_t)t * kTile + own)];
                if (pll != (P.meta[s] >> 16)) return bad("pair landmark", t, own);
                if (pair_grp[(size_t)own] >= 0 && pair_grp[(size_t)own] != group[(size_t)c]) return bad("pair group", t, own);
                // a pair's slots are consecutive (the reduced-precision products sum a pair
                // across its lanes): a pair seen before continues the previous slot's pair
                if (pair_grp[(size_t)own] >= 0 && (q == 0 || P.slot_obs[s - 1] < 0 || (M.mmeta[s - 1] & 0xFF) != (uint32_t)own))
                    return bad("pair slots not consecutive", t, q);
                pair_grp[(size_t)own] = group[(size_t)c];
            }
            for (int q = 0; q < kTile; ++q) {
                size_t s = (size_t)((int64_t)t * kTile + q);
                if (P.slot_obs[s] < 0) continue;
                uint32_t mm = M.mmeta[s];
                int base = (mm >> 8) & 0xFF, cnt = (mm >> 16) & 0xFF;
                int c = cam[P.slot_obs[s]];
                for (int j = 0; j < cnt; ++j) {
                    int g = pair_grp[(size_t)(base + j)];
                    if (g < 0) return bad("pair without group", t, base + j);
                    int64_t e = (int64_t)M.tile_oidx[(size_t)t] + M.slot_ooff[s] + j;
                    if (e >= (int64_t)M.tile_oidx[(size_t)t + 1]) return bad("oidx beyond tile", t, q);
                    int o = M.oidx[(size_t)e];
                    if (o >= no) return bad("out-pair beyond chunk", ch, o);
                    int64_t key = (int64_t)c * N + g;
                    int64_t &pk = part_key[(size_t)(pb + o)];
                    if (pk >= 0 && pk != key) return bad("out-pair label", pb + o, key);
                    pk = key;
                }
            }
        }
    }
    for (int64_t i = 0; i < M.n_part; ++i)
        if (part_key[(size_t)i] < 0) return bad("unused out-pair", i);
    for (int64_t k = 0; k < (int64_t)P.np * N; ++k)
        for (int j = M.cg_ptr[(size_t)k]; j < M.cg_ptr[(size_t)k + 1]; ++j)
            if (part_key[(size_t)M.cg_idx[(size_t)j]] != k || M.part_dst[(size_t)M.cg_idx[(size_t)j]] != j)
                return bad("(camera, subset) CSR", k, j);
    return true;
}
}  // namespace

extern "C" {

// Host-only: plan the layout for host index arrays, check its invariants (and
// those of the plan of the multidirectional product for each N in Ns), and
// report sizes: stats[0] tiles, [1] chunks, [2] partial rows, [3] largest chunk
// slot count, then per N: [4 + 3j] multi chunks, [5 + 3j] out-pairs, [6 + 3j]
// largest chunk out count.  Returns BA_OK, the planner's error, or
// BA_ERR_INVALID_ARG with ba_last_error() naming the broken invariant.
ba_status ba_plan_validate(int32_t n_cams, int32_t n_lms, int64_t n_obs, const int32_t *cam, const int32_t *lm,
                           int32_t max_slots, int32_t max_tiles, const int32_t *Ns, int32_t n_Ns, int64_t *stats) {
    HostPlan P;
    std::string err;
    ba_status st = build_plan(n_cams, n_lms, n_obs, cam, lm, max_slots ? max_slots : 128,
                              max_tiles ? max_tiles : 16, P, err);
    if (st != BA_OK) {
        g_check_err = err;
        return st;
    }
    if (!check_plan(P, cam, lm)) return BA_ERR_INVALID_ARG;
    int max_used = 0;
    for (int ch = 0; ch < P.n_chunks; ++ch) max_used = std::max(max_used, P.chunk_part[ch + 1] - P.chunk_part[ch]);
    if (stats) {
        stats[0] = P.n_tiles;
        stats[1] = P.n_chunks;
        stats[2] = P.n_part;
        stats[3] = max_used;
    }
    for (int j = 0; j < n_Ns; ++j) {
        HostMultiPlan M;
        st = build_multi_plan(P, Ns[j], 512, M, err);
        if (st != BA_OK) {
            g_check_err = err;
            return st;
        }
        if (!check_multi(P, M, cam)) return BA_ERR_INVALID_ARG;
        if (stats) {
            stats[4 + 3 * j] = M.n_chunks;
            stats[5 + 3 * j] = M.n_part;
            stats[6 + 3 * j] = M.max_out;
        }
    }
    return BA_OK;
}

const char *ba_plan_validate_error(void) { return g_check_err.c_str(); }

}  // extern "C"
