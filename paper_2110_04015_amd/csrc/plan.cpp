// Host-side planning of the HBM layout: landmark order, 64-slot tiles, chunks,
// and the deterministic camera reductions.  Integer work only; every floating
// point step runs in the HIP kernels.
#include <algorithm>
#include <cstdio>
#include <cstring>

#include "ba_internal.h"

namespace ba {

// Subset s = floor(np / N) holds poses [s*p, s*(p+1)) for p < N-1; the last
// subset holds the rest (Sec. 3.2, "Optimized implementation").
void partition_groups(int np, int N, int32_t *group) {
    int s = np / N;
    for (int c = 0; c < np; ++c) {
        int g = c / s;
        group[c] = g < N - 1 ? g : N - 1;
    }
}

static void counting_csr(const int32_t *key, int64_t m, int nk, std::vector<int64_t> &ptr,
                         std::vector<int64_t> &idx) {
    ptr.assign((size_t)nk + 1, 0);
    idx.resize((size_t)m);
    for (int64_t o = 0; o < m; ++o) ptr[(size_t)key[o] + 1]++;
    for (int k = 0; k < nk; ++k) ptr[k + 1] += ptr[k];
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t o = 0; o < m; ++o) idx[(size_t)fill[(size_t)key[o]]++] = o;
}

ba_status build_plan(int np, int nl, int64_t m, const int32_t *cam, const int32_t *lm,
                     int max_slots, int max_tiles, HostPlan &P, std::string &err, const int32_t *cam_seg,
                     int target_chunks, int max_tiles_multi, int target_multi) {
    char buf[256];
    P = HostPlan();
    P.np = np;
    P.nl = nl;
    P.m = m;
    P.max_slots = max_slots;
    P.max_tiles = max_tiles > 0 ? max_tiles : 16;
    P.max_tiles_multi = max_tiles_multi > 0 ? max_tiles_multi : max_tiles > 0 ? max_tiles : 16;
    for (int64_t o = 0; o < m; ++o) {
        if (cam[o] < 0 || cam[o] >= np || lm[o] < 0 || lm[o] >= nl) {
            snprintf(buf, sizeof buf, "observation %lld has camera %d / landmark %d out of range",
                     (long long)o, cam[o], lm[o]);
            err = buf;
            return BA_ERR_INVALID_ARG;
        }
    }
    P.obs_cam.assign(cam, cam + m);
    std::vector<int64_t> lptr, lobs;
    counting_csr(lm, m, nl, lptr, lobs);

    // per landmark: observations sorted by camera, duplicate check, min camera
    std::vector<int32_t> minc((size_t)nl, 0);
    for (int l = 0; l < nl; ++l) {
        int64_t a = lptr[l], b = lptr[l + 1];
        int64_t c = b - a;
        if (c > kTile) {
            snprintf(buf, sizeof buf, "landmark %d has %lld observations; at most %d are supported", l,
                     (long long)c, kTile);
            err = buf;
            return BA_ERR_UNSUPPORTED;
        }
        std::sort(lobs.begin() + a, lobs.begin() + b,
                  [&](int64_t x, int64_t y) { return cam[x] < cam[y] || (cam[x] == cam[y] && x < y); });
        for (int64_t q = a + 1; q < b; ++q) {
            if (cam[lobs[q]] == cam[lobs[q - 1]]) {
                snprintf(buf, sizeof buf, "camera %d observes landmark %d twice", cam[lobs[q]], l);
                err = buf;
                return BA_ERR_INVALID_ARG;
            }
        }
        if (c == 0) {
            snprintf(buf, sizeof buf, "landmark %d has no observation: V_lambda is singular", l);
            err = buf;
            return BA_ERR_NOT_SPD;
        }
        minc[l] = cam[lobs[a]];
        if (cam_seg && cam_seg[cam[lobs[b - 1]]] != cam_seg[minc[l]]) {
            snprintf(buf, sizeof buf, "landmark %d is observed by cameras of two problems of the batch", l);
            err = buf;
            return BA_ERR_INVALID_ARG;
        }
    }
    if (cam_seg) {
        for (int c = 1; c < np; ++c)
            if (cam_seg[c] < cam_seg[c - 1]) {
                err = "the problems of a batch must hold consecutive cameras";
                return BA_ERR_INVALID_ARG;
            }
        P.cam_seg.assign(cam_seg, cam_seg + np);
    }
    auto seg_of_lmk = [&](int l) { return cam_seg ? cam_seg[minc[(size_t)l]] : 0; };
    // landmark storage order: by smallest observing camera (stable counting sort), so
    // that consecutive landmarks share cameras on banded problems
    {
        std::vector<int64_t> cnt((size_t)np + 2, 0);
        for (int l = 0; l < nl; ++l) cnt[(size_t)minc[l] + 1]++;
        for (int k = 0; k <= np; ++k) cnt[k + 1] += cnt[k];
        P.lmk_order.resize((size_t)nl);
        for (int l = 0; l < nl; ++l) P.lmk_order[(size_t)cnt[(size_t)minc[l]]++] = l;
    }
    // tiles: landmarks never straddle a tile boundary.  Tiles are filled from a
    // window of the next kWindow landmarks of the sorted order: a landmark that
    // does not fit the current tile waits while later ones fill the gap, and the
    // oldest waiting landmark always opens the next tile.  The storage order of
    // the landmarks becomes their placement order.
    {
        constexpr int kWindow = 48;
        std::vector<int32_t> sorted = P.lmk_order;
        std::vector<int32_t> pending;
        pending.reserve(kWindow);
        P.lmk_order.clear();
        P.lmk_order.reserve((size_t)nl);
        P.lmk_first_slot.resize((size_t)nl);
        P.lmk_count.resize((size_t)nl);
        P.slot_obs.clear();
        P.meta.clear();
        P.tile_lmk_base.clear();
        size_t next = 0;
        int64_t t = 0;
        while (next < (size_t)nl || !pending.empty()) {
            while (pending.size() < (size_t)kWindow && next < (size_t)nl) pending.push_back(sorted[next++]);
            P.tile_lmk_base.push_back((int32_t)P.lmk_order.size());
            P.slot_obs.resize((size_t)(t + 1) * kTile, -1);
            P.meta.resize((size_t)(t + 1) * kTile, kPad);
            // a tile holds landmarks of one problem: that of the oldest waiting landmark
            const int tseg = seg_of_lmk(pending[0]);
            P.tile_seg.push_back(tseg);
            int used = 0, ll = 0;
            size_t keep = 0;
            for (size_t i = 0; i < pending.size(); ++i) {
                int l = pending[i];
                int c = (int)(lptr[l + 1] - lptr[l]);
                if (used + c > kTile || seg_of_lmk(l) != tseg) {
                    pending[keep++] = l;
                    continue;
                }
                int s_new = (int)P.lmk_order.size();
                P.lmk_order.push_back(l);
                P.lmk_first_slot[(size_t)s_new] = t * kTile + used;
                P.lmk_count[(size_t)s_new] = c;
                for (int q = 0; q < c; ++q) {
                    P.slot_obs[(size_t)(t * kTile + used + q)] = lobs[(size_t)(lptr[l] + q)];
                    P.meta[(size_t)(t * kTile + used + q)] = meta_pack(0, (uint32_t)ll);
                }
                used += c;
                ++ll;
            }
            pending.resize(keep);
            ++t;
        }
        P.lmk_store.resize((size_t)nl);
        for (int s = 0; s < nl; ++s) P.lmk_store[(size_t)P.lmk_order[s]] = s;
    }
    const int64_t tiles = (int64_t)P.tile_lmk_base.size();
    P.n_tiles = tiles;
    auto per_chunk = [&](int target) {
        return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (tiles + target - 1) / target));
    };
    if (max_tiles <= 0 && target_chunks > 0) P.max_tiles = per_chunk(target_chunks);
    if (max_tiles <= 0 && max_tiles_multi <= 0 && target_multi > 0) P.max_tiles_multi = per_chunk(target_multi);
    max_tiles = P.max_tiles;
    // chunks of consecutive tiles with at most max_slots distinct cameras
    {
        std::vector<int32_t> stamp((size_t)np, -1), slot_of((size_t)np, 0);
        std::vector<int64_t> tstamp((size_t)np, -1);
        P.chunk_tile.clear();
        P.chunk_part.clear();
        P.chunk_seg.clear();
        P.part_cam.clear();
        int chunk = -1, slots = 0, ntiles_in = 0;
        for (int64_t t = 0; t < tiles; ++t) {
            int fresh = 0;   // cameras of tile t not yet in the current chunk
            for (int q = 0; q < kTile; ++q) {
                int64_t o = P.slot_obs[(size_t)(t * kTile + q)];
                if (o < 0) continue;
                int c = cam[o];
                if (stamp[(size_t)c] != chunk && tstamp[(size_t)c] != t) {
                    tstamp[(size_t)c] = t;
                    ++fresh;
                }
            }
            if (chunk < 0 || slots + fresh > max_slots || ntiles_in >= max_tiles ||
                P.tile_seg[(size_t)t] != P.chunk_seg.back()) {
                ++chunk;
                slots = 0;
                ntiles_in = 0;
                P.chunk_tile.push_back((int32_t)t);
                P.chunk_part.push_back((int32_t)P.part_cam.size());
                P.chunk_seg.push_back(P.tile_seg[(size_t)t]);
            }
            for (int q = 0; q < kTile; ++q) {
                size_t sidx = (size_t)(t * kTile + q);
                int64_t o = P.slot_obs[sidx];
                if (o < 0) continue;
                int c = cam[o];
                if (stamp[(size_t)c] != chunk) {
                    stamp[(size_t)c] = chunk;
                    slot_of[(size_t)c] = slots++;
                    P.part_cam.push_back(c);
                }
                P.meta[sidx] = meta_pack((uint32_t)slot_of[(size_t)c], P.meta[sidx] >> 16);
            }
            ++ntiles_in;
        }
        P.n_chunks = chunk + 1;
        P.chunk_tile.push_back((int32_t)tiles);
        P.chunk_part.push_back((int32_t)P.part_cam.size());
        P.n_part = (int64_t)P.part_cam.size();
        P.max_used_slots = 1;
        for (int ch = 0; ch < P.n_chunks; ++ch)
            P.max_used_slots = std::max(P.max_used_slots, P.chunk_part[(size_t)ch + 1] - P.chunk_part[(size_t)ch]);
    }
    // camera-major CSR over partial rows (ascending row order = fixed summation order)
    {
        std::vector<int64_t> ptr, idx;
        counting_csr(P.part_cam.data(), P.n_part, np, ptr, idx);
        P.cam_part_ptr.resize((size_t)np + 1);
        for (int c = 0; c <= np; ++c) P.cam_part_ptr[c] = (int32_t)ptr[c];
        P.cam_part_idx.resize((size_t)P.n_part);
        for (int64_t i = 0; i < P.n_part; ++i) P.cam_part_idx[(size_t)i] = (int32_t)idx[(size_t)i];
        // a chunk writes its partial row straight into the camera-major position
        P.part_dst.resize((size_t)P.n_part);
        for (int64_t j = 0; j < P.n_part; ++j) P.part_dst[(size_t)P.cam_part_idx[(size_t)j]] = (int32_t)j;
    }
    counting_csr(cam, m, np, P.cam_obs_ptr, P.cam_obs);
    return BA_OK;
}

// Number of other cameras that share at least one landmark with each camera
// (the covisibility degree, an input feature of the learned preconditioner).
void covisibility_degree(const HostPlan &P, std::vector<int32_t> &deg) {
    const int np = P.np;
    deg.assign((size_t)np, 0);
    // landmark -> its observing cameras, from the tile layout (landmarks are contiguous)
    std::vector<int64_t> lptr((size_t)P.nl + 1, 0);
    for (int s = 0; s < P.nl; ++s) lptr[(size_t)s + 1] = lptr[(size_t)s] + P.lmk_count[(size_t)s];
    std::vector<int32_t> lcam((size_t)lptr[(size_t)P.nl]);
    for (int s = 0; s < P.nl; ++s)
        for (int q = 0; q < P.lmk_count[(size_t)s]; ++q)
            lcam[(size_t)(lptr[(size_t)s] + q)] = P.obs_cam[(size_t)P.slot_obs[(size_t)(P.lmk_first_slot[(size_t)s] + q)]];
    std::vector<int32_t> stamp((size_t)np, -1);
    // camera -> landmarks via the observation CSR
    std::vector<int32_t> obs_store((size_t)P.m);
    for (int s = 0; s < P.nl; ++s)
        for (int q = 0; q < P.lmk_count[(size_t)s]; ++q)
            obs_store[(size_t)P.slot_obs[(size_t)(P.lmk_first_slot[(size_t)s] + q)]] = s;
    for (int c = 0; c < np; ++c) {
        int cnt = 0;
        stamp[(size_t)c] = c;
        for (int64_t q = P.cam_obs_ptr[(size_t)c]; q < P.cam_obs_ptr[(size_t)c + 1]; ++q) {
            const int s = obs_store[(size_t)P.cam_obs[(size_t)q]];
            for (int64_t e = lptr[(size_t)s]; e < lptr[(size_t)s + 1]; ++e) {
                const int c2 = lcam[(size_t)e];
                if (stamp[(size_t)c2] != c) {
                    stamp[(size_t)c2] = c;
                    ++cnt;
                }
            }
        }
        deg[(size_t)c] = cnt;
    }
}

ba_status build_multi_plan(const HostPlan &P, int N, int max_out, HostMultiPlan &M,
                           std::string &err, const int32_t *group_in) {
    M = HostMultiPlan();
    M.N = N;
    const int np = P.np;
    std::vector<int32_t> group((size_t)np);
    if (group_in) group.assign(group_in, group_in + np);
    else partition_groups(np, N, group.data());
    const int64_t T = P.n_tiles;
    M.mmeta.assign((size_t)T * kTile, kPad);
    M.slot_cam.assign((size_t)T * kTile, 0);
    M.pair_ll.assign((size_t)T * kTile, 0xFF);
    M.slot_ooff.assign((size_t)T * kTile, 0);
    M.tile_oidx.assign((size_t)T + 1, 0);
    // per tile: landmark pairs (landmark, subset) in order of first appearance
    std::vector<int32_t> pair_grp((size_t)T * kTile, -1);
    for (int64_t t = 0; t < T; ++t) {
        int npairs = 0;
        int q = 0;
        while (q < kTile) {
            size_t s0 = (size_t)(t * kTile + q);
            if (P.slot_obs[s0] < 0) break;
            uint32_t ll = P.meta[s0] >> 16;
            int q1 = q;
            while (q1 < kTile && P.slot_obs[(size_t)(t * kTile + q1)] >= 0 &&
                   (P.meta[(size_t)(t * kTile + q1)] >> 16) == ll)
                ++q1;
            int base = npairs;
            for (int a = q; a < q1; ++a) {
                int c = P.obs_cam[(size_t)P.slot_obs[(size_t)(t * kTile + a)]];
                int g = group[(size_t)c];
                int found = -1;
                for (int pj = base; pj < npairs; ++pj)
                    if (pair_grp[(size_t)(t * kTile + pj)] == g) found = pj;
                if (found < 0) {
                    found = npairs++;
                    pair_grp[(size_t)(t * kTile + found)] = g;
                    M.pair_ll[(size_t)(t * kTile + found)] = (uint8_t)ll;
                }
                M.slot_cam[(size_t)(t * kTile + a)] = c;
                M.mmeta[(size_t)(t * kTile + a)] = (uint32_t)found | ((uint32_t)base << 8);
            }
            int cnt = npairs - base;
            for (int a = q; a < q1; ++a) M.mmeta[(size_t)(t * kTile + a)] |= (uint32_t)cnt << 16;
            q = q1;
        }
    }
    // chunks over out-pairs (camera, subset)
    std::vector<int32_t> stamp((size_t)np * N, -1), local((size_t)np * N, 0);
    std::vector<int64_t> part_key;                    // partial row -> camera * N + subset
    int chunk = -1, outs = 0, ntiles_in = 0;
    M.max_out = 0;
    for (int64_t t = 0; t < T; ++t) {
        // distinct out-pairs needed by this tile alone
        std::vector<int64_t> need;
        for (int q = 0; q < kTile; ++q) {
            size_t s = (size_t)(t * kTile + q);
            if (P.slot_obs[s] < 0) continue;
            uint32_t mm = M.mmeta[s];
            int base = (mm >> 8) & 0xFF, cnt = (mm >> 16) & 0xFF;
            int c = M.slot_cam[s];
            for (int j = 0; j < cnt; ++j) need.push_back((int64_t)c * N + pair_grp[(size_t)(t * kTile + base + j)]);
        }
        std::sort(need.begin(), need.end());
        need.erase(std::unique(need.begin(), need.end()), need.end());
        int fresh = 0;
        if (chunk >= 0)
            for (int64_t k : need) fresh += stamp[(size_t)k] != chunk;
        if ((int)need.size() > max_out) max_out = (int)need.size();
        if (chunk < 0 || outs + fresh > max_out || ntiles_in >= P.max_tiles_multi ||
            P.tile_seg[(size_t)t] != M.chunk_seg.back()) {
            ++chunk;
            outs = 0;
            ntiles_in = 0;
            M.chunk_tile.push_back((int32_t)t);
            M.chunk_part.push_back((int32_t)part_key.size());
            M.chunk_seg.push_back(P.tile_seg[(size_t)t]);
        }
        for (int64_t k : need) {
            if (stamp[(size_t)k] != chunk) {
                stamp[(size_t)k] = chunk;
                local[(size_t)k] = outs++;
                part_key.push_back(k);
            }
        }
        if (outs > M.max_out) M.max_out = outs;
        M.tile_oidx[(size_t)t] = (uint32_t)M.oidx.size();
        int off = 0;
        for (int q = 0; q < kTile; ++q) {
            size_t s = (size_t)(t * kTile + q);
            if (P.slot_obs[s] < 0) continue;
            uint32_t mm = M.mmeta[s];
            int base = (mm >> 8) & 0xFF, cnt = (mm >> 16) & 0xFF;
            int c = M.slot_cam[s];
            M.slot_ooff[s] = (uint16_t)off;
            for (int j = 0; j < cnt; ++j) {
                int64_t k = (int64_t)c * N + pair_grp[(size_t)(t * kTile + base + j)];
                M.oidx.push_back((uint16_t)local[(size_t)k]);
            }
            off += cnt;
        }
        ++ntiles_in;
    }
    M.tile_oidx[(size_t)T] = (uint32_t)M.oidx.size();
    M.n_chunks = chunk + 1;
    M.chunk_tile.push_back((int32_t)T);
    M.chunk_part.push_back((int32_t)part_key.size());
    M.n_part = (int64_t)part_key.size();
    if (M.max_out > 65535) {
        err = "multidirectional product: too many (camera, subset) pairs in one tile";
        return BA_ERR_UNSUPPORTED;
    }
    // (camera, subset)-major CSR over partial rows
    const int64_t K = (int64_t)np * N;
    M.cg_ptr.assign((size_t)K + 1, 0);
    for (int64_t k : part_key) M.cg_ptr[(size_t)k + 1]++;
    for (int64_t k = 0; k < K; ++k) M.cg_ptr[(size_t)k + 1] += M.cg_ptr[(size_t)k];
    M.cg_idx.resize(part_key.size());
    std::vector<int32_t> fill(M.cg_ptr.begin(), M.cg_ptr.end() - 1);
    for (size_t i = 0; i < part_key.size(); ++i) M.cg_idx[(size_t)fill[(size_t)part_key[i]]++] = (int32_t)i;
    M.part_dst.resize(part_key.size());
    for (size_t j = 0; j < part_key.size(); ++j) M.part_dst[(size_t)M.cg_idx[j]] = (int32_t)j;
    return BA_OK;
}

}  // namespace ba
