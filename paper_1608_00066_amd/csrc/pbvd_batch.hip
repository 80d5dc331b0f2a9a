// Batched decoding (pbvd_batch_* of include/pbvd.h): the work-list builder
// that packs the parallel blocks of many frames into waves, and the batch
// object that uploads it once and launches, per decode, one tile kernel per
// register-kernel code and one persistent state-parallel kernel per
// constraint length (all its codes in one launch), these launch units on
// forked streams so that they overlap on the device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdlib.h>

#include <algorithm>
#include <new>
#include <utility>
#include <vector>

#include "pbvd.h"
#include "pbvd_aux.hpp"
#include "pbvd_host.hpp"
#include "pbvd_registry.hpp"

namespace pbvd_host {

pbvd_status make_code_set(const pbvd_code *codes, int32_t n, CodeSet *out, int auto_lb) {
    if (!codes) return fail(PBVD_EINVAL, "codes must not be NULL");
    if (n < 1 || n > kMaxCodes) return fail(PBVD_EINVAL, "n_codes must be in [1, %d]", kMaxCodes);
    CodeSet cs;
    for (int i = 0; i < n; ++i) {
        int idx = -1;
        pbvd_status st = check_code(codes[i], &idx);
        if (st != PBVD_OK) return st;
        if (codes[i].D % 8 != 0)
            return fail(PBVD_EINVAL, "code %d: batched decoding needs D %% 8 == 0 (got %d)", i, codes[i].D);
        cs.codes[i] = codes[i];
        for (int r = codes[i].R; r < 4; ++r) cs.codes[i].gen[r] = 0;
        cs.idx[i] = idx;
        const int req = requested_lb(codes[i]);
        const int top = max_lb(codes[i]);
        cs.lb[i] = req == kGroupLb ? kGroupLb
                   : idx < 0 || (req < 0 && auto_lb == kWaveLb && codes[i].mapping != PBVD_MAP_LANES) ? kWaveLb
                   : req >= 0 ? req : (auto_lb < 0 || auto_lb > top ? top : auto_lb);
        if (cs.lb[i] == kGroupLb) (void)group_tables(cs.codes[i], &cs.gtab[i]);  // checked by check_code
    }
    cs.n = n;
    *out = cs;
    return PBVD_OK;
}

namespace {

// Waves per workgroup of a tile launch: 4 (PBVD_TILE_WAVES_PER_BLOCK = 1, 2
// or 4 overrides it).
int tile_waves_per_block() {
    if (const char *env = getenv("PBVD_TILE_WAVES_PER_BLOCK")) {
        const int w = atoi(env);
        if (w == 1 || w == 2 || w == 4) return w;
    }
    return pbvd::kBlockThreads / pbvd::kWave;
}

// One parallel block of one frame (Sec. III-A), in the batch's coordinates.
struct PbRec {
    int64_t sym, out_bit;
    int32_t len, store0, dec_end, flags;
};

}  // namespace

pbvd_status build_work_list(const CodeSet &cs, const pbvd_frame *frames, int64_t n_frames,
                            int64_t sym_bytes, int64_t out_bytes, WorkList *wl, bool fuse_waves,
                            bool pair_tiles) {
    std::vector<std::vector<PbRec>> per_code(cs.n);
    std::vector<std::pair<int64_t, int64_t>> outs;
    outs.reserve((size_t)n_frames);
    wl->n_blocks = 0;
    wl->n_stages = 0;
    for (int64_t f = 0; f < n_frames; ++f) {
        const pbvd_frame &fr = frames[f];
        if (fr.code < 0 || fr.code >= cs.n || fr.reserved != 0)
            return fail(PBVD_EINVAL, "frame %lld: bad code index %d", (long long)f, fr.code);
        const pbvd_code &c = cs.codes[fr.code];
        if (fr.n_bits < 1) return fail(PBVD_EINVAL, "frame %lld: n_bits must be >= 1", (long long)f);
        const int64_t T = fr.n_bits + (c.terminated ? c.K - 1 : 0);
        if (fr.sym_offset < 0 || fr.sym_offset > sym_bytes - T * c.R)
            return fail(PBVD_EINVAL, "frame %lld: symbols outside the %lld-byte input", (long long)f,
                        (long long)sym_bytes);
        const int64_t nbytes = ceil_div(fr.n_bits, 8);
        if (fr.out_offset < 0 || fr.out_offset > out_bytes - nbytes)
            return fail(PBVD_EINVAL, "frame %lld: output outside the %lld-byte buffer", (long long)f,
                        (long long)out_bytes);
        outs.emplace_back(fr.out_offset, fr.out_offset + nbytes);
        const int64_t D = c.D, L = c.L;
        const int64_t nb = ceil_div(fr.n_bits, D);
        for (int64_t pb = 0; pb < nb; ++pb) {
            const int64_t d0 = pb * D;
            const int64_t f0 = d0 - L < 0 ? 0 : d0 - L;
            const int64_t f1 = d0 + D + L > T ? T : d0 + D + L;
            const int64_t d1 = d0 + D > fr.n_bits ? fr.n_bits : d0 + D;
            PbRec r;
            r.sym = fr.sym_offset + f0 * c.R;
            r.out_bit = fr.out_offset * 8 + d0;
            r.len = (int32_t)(f1 - f0);
            r.store0 = (int32_t)(d0 - f0);
            r.dec_end = (int32_t)(d1 - f0);
            r.flags = pbvd::kLaneActive | (f0 == 0 ? pbvd::kLaneKnown : 0) |
                      (f1 == T && !c.terminated ? pbvd::kLaneArgmin : 0);
            per_code[fr.code].push_back(r);
            wl->n_stages += r.len;
        }
        wl->n_blocks += nb;
    }
    std::sort(outs.begin(), outs.end());
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].first < outs[i - 1].second)
            return fail(PBVD_EINVAL, "frame output ranges overlap at byte %lld", (long long)outs[i].first);

    wl->lanes.clear();
    wl->heads.clear();
    wl->descs.clear();
    for (FusedGroup &fg : wl->fused) fg = FusedGroup{};
    if (fuse_waves) {
        // one descriptor list per K over all its state-parallel codes, the
        // longest PBs first (the persistent waves take them in this order,
        // so the longest finish first and the short ones fill the tail)
        for (int K = kMinK; K <= kMaxK; ++K) {
            FusedGroup &fg = wl->fused[K - kMinK];
            std::vector<PbRec> v;
            for (int ci = 0; ci < cs.n; ++ci) {
                if (cs.lb[ci] != kWaveLb || cs.codes[ci].K != K) continue;
                const int slot = fg.n_codes++;
                fg.codes[slot] = ci;
                fg.sp_wave_dwords = std::max(fg.sp_wave_dwords, wave_slot_dwords(cs.codes[ci]));
                for (PbRec r : per_code[ci]) {
                    r.flags |= slot << pbvd::wave::kDescCodeShift;
                    v.push_back(r);
                }
                per_code[ci].clear();
            }
            std::stable_sort(v.begin(), v.end(), [](const PbRec &x, const PbRec &y) { return x.len > y.len; });
            fg.desc_begin = (int64_t)wl->descs.size();
            fg.n_descs = (int64_t)v.size();
            for (const PbRec &r : v)
                wl->descs.push_back(pbvd::LaneDesc{r.sym, r.out_bit, r.len, r.store0, r.dec_end, r.flags});
        }
    }
    // register-kernel tiles per code (heads, 64 lane descriptors each),
    // emitted after the loop: code by code, a pair's two codes merged
    std::vector<std::vector<pbvd::TileHead>> th(cs.n);
    std::vector<std::vector<pbvd::LaneDesc>> tl(cs.n);
    for (int ci = 0; ci < cs.n; ++ci) {
        const pbvd_code &c = cs.codes[ci];
        const int64_t U = pbvd::trip_stages(c.K);
        const int64_t ND = pbvd::trip_fetch_dwords(c.K, c.R);
        const int lb = cs.lb[ci];
        if (lb == kGroupLb) {
            // tiles of 64 PBs, longest first (a tile runs as long as its
            // longest PB); the last tile padded with inactive descriptors
            std::vector<PbRec> &v = per_code[ci];
            std::stable_sort(v.begin(), v.end(), [](const PbRec &x, const PbRec &y) { return x.len > y.len; });
            const int64_t tp = pbvd::group::kTilePbs;
            const int64_t nt = ceil_div((int64_t)v.size(), tp);
            wl->groups[ci].tile_begin = (int64_t)wl->descs.size();
            for (int64_t k = 0; k < nt * tp; ++k) {
                const PbRec &r = v[k < (int64_t)v.size() ? k : 0];
                pbvd::LaneDesc d{r.sym, r.out_bit, r.len, r.store0, r.dec_end, r.flags};
                if (k >= (int64_t)v.size()) d.flags &= ~pbvd::kLaneActive;
                wl->descs.push_back(d);
            }
            wl->groups[ci].n_tiles = nt;
            wl->groups[ci].sp_wave_dwords = group_tile_dwords(c);
            wl->groups[ci].lb = lb;
            continue;
        }
        if (lb == kWaveLb) {
            // one wave per PB, longest first (fused: already listed, empty here)
            std::vector<PbRec> &v = per_code[ci];
            std::stable_sort(v.begin(), v.end(), [](const PbRec &x, const PbRec &y) { return x.len > y.len; });
            wl->groups[ci].tile_begin = (int64_t)wl->descs.size();
            for (const PbRec &r : v)
                wl->descs.push_back(pbvd::LaneDesc{r.sym, r.out_bit, r.len, r.store0, r.dec_end, r.flags});
            wl->groups[ci].n_tiles = (int64_t)v.size();
            wl->groups[ci].sp_wave_dwords = wave_slot_dwords(c);
            wl->groups[ci].lb = lb;
            continue;
        }
        const size_t pw = (size_t)(pbvd::kWave >> lb);  // PBs per tile
        std::vector<PbRec> &v = per_code[ci];
        // PBs that start their traceback from the best state must share a
        // tile with PBs of the same length only, so that all of a tile's
        // final metrics are taken at one stage.  The others by first traced
        // stage, then longest first (load balance): equal geometries next to
        // each other, so that most tiles hold PBs of one geometry and run the
        // kernel's uniform-wave path, and tiles of PBs of different lengths
        // mostly share their first traced stage (phase-aligned traceback).
        std::stable_sort(v.begin(), v.end(), [](const PbRec &x, const PbRec &y) {
            const bool ax = x.flags & pbvd::kLaneArgmin, ay = y.flags & pbvd::kLaneArgmin;
            if (ax != ay) return ax < ay;
            if (x.store0 != y.store0) return x.store0 < y.store0;
            if (x.len != y.len) return x.len > y.len;
            return x.dec_end < y.dec_end;
        });
        size_t i = 0;
        while (i < v.size()) {
            size_t e = std::min(v.size(), i + pw);
            if (v[i].flags & pbvd::kLaneArgmin) {
                size_t k = i + 1;
                while (k < e && (v[k].flags & pbvd::kLaneArgmin) && v[k].len == v[i].len) ++k;
                e = k;
            } else {
                // a tile ends where the first traced stage changes: its PBs
                // share it, so that tiles of PBs of different lengths take
                // the phase-aligned traceback
                size_t k = i + 1;
                while (k < e && !(v[k].flags & pbvd::kLaneArgmin) && v[k].store0 == v[i].store0) ++k;
                e = k;
            }
            pbvd::TileHead h{};
            h.len = 0;
            h.store0_min = 0x7fffffff;
            int64_t i_safe = INT64_MAX;
            bool wide = true, final_needed = false, uniform = true, same_store0 = true;
            for (size_t k = i; k < i + pw; ++k) {
                // PBs past the tile's repeat its first PB, inactive; every
                // lane of a PB's group gets the PB's descriptor
                const PbRec &r = v[k < e ? k : i];
                pbvd::LaneDesc d;
                d.sym = r.sym;
                d.out_bit = r.out_bit;
                d.len = r.len;
                d.store0 = r.store0;
                d.dec_end = r.dec_end;
                d.flags = k < e ? r.flags : (r.flags & ~pbvd::kLaneActive);
                for (int g = 0; g < (1 << lb); ++g) tl[ci].push_back(d);
                if (r.len != v[i].len || r.store0 != v[i].store0 || r.dec_end != v[i].dec_end) uniform = false;
                if (r.store0 != v[i].store0) same_store0 = false;
                if (r.len > h.len) h.len = r.len;
                if (r.store0 < h.store0_min) h.store0_min = r.store0;
                const int64_t last_trip = ((r.len - 1) / U) * U;
                if (r.sym + last_trip * c.R + 4 * ND > sym_bytes) {
                    // the lane's wide fetches are in bounds up to stage t
                    wide = false;
                    const int64_t room = sym_bytes - 4 * ND - r.sym;
                    i_safe = std::min(i_safe, room < 0 ? -1 : room / c.R);
                }
                if (r.flags & pbvd::kLaneArgmin) final_needed = true;
            }
            // only the trips past the first unsafe fetch take byte loads
            h.i_safe = wide ? h.len : (int32_t)std::min<int64_t>(i_safe, h.len);
            h.flags = (wide ? pbvd::kTileWide : 0) | (final_needed ? pbvd::kTileFinal : 0) |
                      (uniform ? pbvd::kTileUniform : 0) | (same_store0 ? pbvd::kTileStore0 : 0);
            th[ci].push_back(h);
            i = e;
        }
        wl->groups[ci].sp_wave_dwords = slot_dwords(c, lb);
        wl->groups[ci].lb = lb;
    }

    // registered pairs among the register codes (one launch for both)
    int partner[kMaxCodes], pair_of[kMaxCodes];
    bool second[kMaxCodes];
    for (int ci = 0; ci < cs.n; ++ci) partner[ci] = pair_of[ci] = -1, second[ci] = false;
    auto register_code = [&](int ci) { return cs.idx[ci] >= 0 && cs.lb[ci] >= 0 && cs.lb[ci] <= 3; };
    for (int ci = 0; pair_tiles && ci < cs.n; ++ci) {
        for (int cj = ci + 1; cj < cs.n && partner[ci] < 0; ++cj) {
            const pbvd_code &a = cs.codes[ci], &b = cs.codes[cj];
            if (partner[cj] >= 0 || !register_code(ci) || !register_code(cj) || cs.lb[ci] != cs.lb[cj] ||
                a.pm_bits != 16 || b.pm_bits != 16 || a.input_kind != b.input_kind || th[ci].empty() ||
                th[cj].empty())
                continue;
            bool ci_first = true;
            const int p = find_pair(cs.idx[ci], cs.idx[cj], &ci_first);
            if (p < 0) continue;
            partner[ci] = cj;
            partner[cj] = ci;
            pair_of[ci] = pair_of[cj] = p;
            second[ci] = !ci_first;
            second[cj] = ci_first;
        }
    }
    for (int ci = 0; ci < cs.n; ++ci) {
        if (!register_code(ci) || (partner[ci] >= 0 && partner[ci] < ci)) continue;
        TileGroup &g = wl->groups[ci];
        g.tile_begin = (int64_t)wl->heads.size();
        if (partner[ci] < 0) {
            wl->heads.insert(wl->heads.end(), th[ci].begin(), th[ci].end());
            wl->lanes.insert(wl->lanes.end(), tl[ci].begin(), tl[ci].end());
            g.n_tiles = (int64_t)th[ci].size();
            continue;
        }
        // both codes' tiles, longest first over the two; the tiles of the
        // pair's second code carry kTileCode1
        const int cj = partner[ci];
        std::vector<std::pair<int, size_t>> order;
        order.reserve(th[ci].size() + th[cj].size());
        for (size_t k = 0; k < th[ci].size(); ++k) order.emplace_back(ci, k);
        for (size_t k = 0; k < th[cj].size(); ++k) order.emplace_back(cj, k);
        std::stable_sort(order.begin(), order.end(), [&](const std::pair<int, size_t> &x,
                                                         const std::pair<int, size_t> &y) {
            return th[x.first][x.second].len > th[y.first][y.second].len;
        });
        for (const auto &o : order) {
            pbvd::TileHead h = th[o.first][o.second];
            if (second[o.first]) h.flags |= pbvd::kTileCode1;
            wl->heads.push_back(h);
            const size_t l0 = o.second * (size_t)pbvd::kWave;
            wl->lanes.insert(wl->lanes.end(), tl[o.first].begin() + l0, tl[o.first].begin() + l0 + pbvd::kWave);
        }
        g.n_tiles = (int64_t)order.size();
        g.sp_wave_dwords = std::max(g.sp_wave_dwords, wl->groups[cj].sp_wave_dwords);
        g.pair = pair_of[ci];
        wl->groups[cj].tile_begin = g.tile_begin;
        wl->groups[cj].n_tiles = 0;
    }
    return PBVD_OK;
}

pbvd_status launch_group(const CodeSet &cs, int ci, const TileGroup &g, const uint8_t *d_syms,
                         int64_t sym_bytes, uint8_t *d_out, const pbvd::LaneDesc *d_lanes,
                         const pbvd::TileHead *d_heads, const pbvd::LaneDesc *d_descs, uint32_t *sp,
                         int64_t per_launch, hipStream_t stream) {
    if (g.lb == kGroupLb) {
        const pbvd_code &c = cs.codes[ci];
        pbvd::GroupLaunchRequest req{};
        pbvd::group::GroupArgs &a = req.args;
        a = cs.gtab[ci];
        a.syms = d_syms;
        a.in_end = d_syms + sym_bytes;
        a.out = d_out;
        a.out_mode = pbvd::kOutBytes;
        a.kind = c.input_kind;
        a.final_pm = nullptr;
        a.sp = sp;
        a.sp_tile_dwords = g.sp_wave_dwords;
        a.descs = d_descs + g.tile_begin;
        req.R = c.R;
        req.stream = stream;
        for (int64_t t0 = 0; t0 < g.n_tiles; t0 += per_launch) {
            a.tile_begin = t0;
            a.n_tiles = std::min(per_launch, g.n_tiles - t0);
            req.grid = (unsigned)a.n_tiles;
            hipError_t e = launch_group_kernel(c.K, req);
            if (e != hipSuccess) return fail_hip(e, "batch group kernel launch");
        }
        return PBVD_OK;
    }
    if (g.lb == kWaveLb) {
        const pbvd_code &c = cs.codes[ci];
        pbvd::WaveLaunchRequest req{};
        pbvd::wave::Args &a = req.args;
        a.syms = d_syms;
        a.in_end = d_syms + sym_bytes;
        a.out = d_out;
        a.out_mode = pbvd::kOutBytes;
        a.sp = sp;
        a.sp_wave_dwords = g.sp_wave_dwords;
        a.descs = d_descs + g.tile_begin;
        a.codes[0] = wave_code(c);
        req.stream = stream;
        const int waves_per_block = pbvd::kBlockThreads / pbvd::kWave;
        for (int64_t t0 = 0; t0 < g.n_tiles; t0 += per_launch) {
            a.wave_begin = t0;
            a.n_waves = std::min(per_launch, g.n_tiles - t0);
            req.grid = (unsigned)ceil_div(a.n_waves, waves_per_block);
            hipError_t e = launch_wave(c.K, req);
            if (e != hipSuccess) return fail_hip(e, "batch wave kernel launch");
        }
        return PBVD_OK;
    }
    const int waves_per_block = tile_waves_per_block();
    for (int64_t t0 = 0; t0 < g.n_tiles; t0 += per_launch) {
        pbvd::TileLaunchRequest req{};
        pbvd::TileArgs &a = req.args;
        a.syms = d_syms;
        a.sym_bytes = sym_bytes;
        a.out = d_out;
        a.lanes = d_lanes;
        a.heads = d_heads;
        a.sp = sp;
        a.sp_wave_dwords = g.sp_wave_dwords;
        a.tile_begin = g.tile_begin + t0;
        a.n_tiles = std::min(per_launch, g.n_tiles - t0);
        req.pm_bits = cs.codes[ci].pm_bits;
        req.input_kind = cs.codes[ci].input_kind;
        req.lb = g.lb;
        req.grid = (unsigned)ceil_div(a.n_tiles, waves_per_block);
        req.block_threads = (unsigned)(waves_per_block * pbvd::kWave);
        req.stream = stream;
        hipError_t e = g.pair >= 0 ? launch_tiles_pair(g.pair, req) : launch_tiles(cs.idx[ci], req);
        if (e != hipSuccess) return fail_hip(e, "batch kernel launch");
    }
    return PBVD_OK;
}

pbvd_status launch_fused(const CodeSet &cs, int K, const FusedGroup &g, const uint8_t *d_syms,
                         int64_t sym_bytes, uint8_t *d_out, const pbvd::LaneDesc *d_descs, uint32_t *sp,
                         int64_t waves, uint32_t *counter, hipStream_t stream) {
    if (g.n_descs == 0) return PBVD_OK;
    // a kernel, not a memset node: the launch may be captured into a graph
    hipError_t e = pbvd::fill_u32(counter, pbvd::wave::kCounters * pbvd::wave::kCounterStride, 0u, stream);
    if (e != hipSuccess) return fail_hip(e, "work counter reset");
    pbvd::WaveLaunchRequest req{};
    pbvd::wave::Args &a = req.args;
    a.syms = d_syms;
    a.in_end = d_syms + sym_bytes;
    a.out = d_out;
    a.out_mode = pbvd::kOutBytes;
    a.sp = sp;
    a.sp_wave_dwords = g.sp_wave_dwords;
    a.descs = d_descs + g.desc_begin;
    a.counter = counter;
    a.n_items = g.n_descs;
    for (int k = 0; k < g.n_codes; ++k) a.codes[k] = wave_code(cs.codes[g.codes[k]]);
    a.wave_begin = 0;
    a.n_waves = std::max<int64_t>(1, std::min(waves, g.n_descs));
    req.grid = (unsigned)ceil_div(a.n_waves, pbvd::kBlockThreads / pbvd::kWave);
    req.stream = stream;
    e = launch_wave(K, req);
    if (e != hipSuccess) return fail_hip(e, "persistent wave kernel launch");
    return PBVD_OK;
}

}  // namespace pbvd_host

using namespace pbvd_host;

struct pbvd_batch {
    CodeSet cs;
    int device = 0;
    TileGroup groups[kMaxCodes];
    int64_t per_launch[kMaxCodes];  // waves per launch of each code
    int64_t sp_off[kMaxCodes];      // dword offset of each code's survivor area
    // state-parallel codes: one persistent launch per K
    FusedGroup fused[kMaxK - kMinK + 1];
    int64_t fused_waves[kMaxK - kMinK + 1];
    int64_t fused_sp_off[kMaxK - kMinK + 1];
    uint32_t *counters = nullptr;   // the work counters of each K, kCounterDwords apart
    size_t counters_bytes = 0;
    int64_t n_tiles = 0, n_blocks = 0, n_stages = 0;
    int64_t sym_bytes = 0, out_bytes = 0;
    pbvd::LaneDesc *d_lanes = nullptr;
    pbvd::TileHead *d_heads = nullptr;
    pbvd::LaneDesc *d_descs = nullptr;
    size_t lanes_bytes = 0, heads_bytes = 0, descs_bytes = 0;
    uint32_t *sp = nullptr;
    size_t sp_bytes = 0;
    // launch units (a code's tiles, or a K's persistent launch) after the
    // first run on these streams, forked from and joined to the caller's
    // stream with events
    hipStream_t aux[kMaxCodes] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kMaxCodes] = {};
    // recorded on the caller's stream after the last decode launched outside
    // graph capture (its forked codes joined back first)
    hipEvent_t done = nullptr;
    bool done_recorded = false;
};

namespace {

constexpr int64_t kCounterDwords = pbvd::wave::kCounters * pbvd::wave::kCounterStride;

void release(pbvd_batch *b) {
    DeviceGuard dg(b->device);
    if (b->sp || b->d_lanes || b->d_heads || b->d_descs || b->counters) (void)hipDeviceSynchronize();
    if (b->sp) (void)hipFree(b->sp);
    if (b->d_lanes) (void)hipFree(b->d_lanes);
    if (b->d_heads) (void)hipFree(b->d_heads);
    if (b->d_descs) (void)hipFree(b->d_descs);
    if (b->counters) (void)hipFree(b->counters);
    for (int i = 0; i < kMaxCodes; ++i) {
        if (b->aux[i]) (void)hipStreamDestroy(b->aux[i]);
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->done) (void)hipEventDestroy(b->done);
}

}  // namespace

extern "C" {

pbvd_status pbvd_batch_create(const pbvd_code *codes, int32_t n_codes, pbvd_batch **out) {
    g_last_error[0] = 0;
    if (!codes || !out) return fail(PBVD_EINVAL, "codes and out must not be NULL");
    CodeSet cs;
    const pbvd_status st = make_code_set(codes, n_codes, &cs);
    if (st != PBVD_OK) return st;
    pbvd_batch *b = new (std::nothrow) pbvd_batch();
    if (!b) return fail(PBVD_ENOMEM, "host allocation failed");
    b->cs = cs;
    if (hipGetDevice(&b->device) != hipSuccess) b->device = 0;
    (void)hipGetLastError();
    *out = b;
    return PBVD_OK;
}

pbvd_status pbvd_batch_set_frames(pbvd_batch *b, const pbvd_frame *frames, int64_t n_frames,
                                  int64_t sym_bytes, int64_t out_bytes) {
    g_last_error[0] = 0;
    if (!b) return fail(PBVD_EINVAL, "batch is NULL");
    if (n_frames < 0 || (n_frames > 0 && !frames)) return fail(PBVD_EINVAL, "bad frame array");
    if (sym_bytes < 0 || out_bytes < 0) return fail(PBVD_EINVAL, "negative buffer size");
    // codes that leave the lanes per PB open: one lane per PB when the PBs
    // of the launch give every SIMD a wave, the largest lane group otherwise
    // (the two codes of a registered pair share a launch: their PBs count
    // together, and they take one width so that they do share it)
    CodeSet cs = b->cs;
    {
        int64_t pbs[kMaxCodes] = {};
        for (int64_t f = 0; f < n_frames; ++f)
            if (frames[f].code >= 0 && frames[f].code < cs.n && frames[f].n_bits > 0)
                pbs[frames[f].code] += ceil_div(frames[f].n_bits, cs.codes[frames[f].code].D);
        for (int ci = 0; ci < cs.n; ++ci) {
            if (requested_lb(cs.codes[ci]) >= 0 || cs.idx[ci] < 0) continue;
            int64_t n = pbs[ci];
            int top = max_lb(cs.codes[ci]);
            for (int cj = 0; cj < cs.n; ++cj) {
                bool first = true;
                if (cj == ci || requested_lb(cs.codes[cj]) >= 0 || cs.idx[cj] < 0 ||
                    cs.codes[ci].pm_bits != 16 || cs.codes[cj].pm_bits != 16 ||
                    cs.codes[ci].input_kind != cs.codes[cj].input_kind ||
                    find_pair(cs.idx[ci], cs.idx[cj], &first) < 0)
                    continue;
                n += pbs[cj];
                top = std::min(top, max_lb(cs.codes[cj]));
                break;
            }
            cs.lb[ci] = ceil_div(n, pbvd::kWave) >= 1024 ? 0 : top;
        }
    }
    WorkList wl;
    pbvd_status st;
    try {
        st = build_work_list(cs, frames, n_frames, sym_bytes, out_bytes, &wl, true, true);
    } catch (...) {
        st = fail(PBVD_ENOMEM, "host allocation failed while building the work list");
    }
    if (st != PBVD_OK) return st;
    DeviceGuard dg(b->device);
    if (!dg.ok) return fail(PBVD_EHIP, "cannot select device %d", b->device);
    if (b->done_recorded) {
        // earlier decodes of this batch may still read the work list and
        // the survivor area that are replaced below: wait for them (and for
        // nothing else on the device)
        hipError_t e = hipEventSynchronize(b->done);
        if (e != hipSuccess) return fail_hip(e, "waiting for earlier decodes");
        b->done_recorded = false;
    }
    // from here on the old work list is gone: a call that fails below leaves
    // an empty batch (its decodes write nothing) until frames are set again
    b->n_tiles = 0;
    b->n_blocks = 0;
    b->n_stages = 0;
    for (int ci = 0; ci < kMaxCodes; ++ci) b->groups[ci] = TileGroup{};
    for (FusedGroup &fg : b->fused) fg = FusedGroup{};
    {
        // streams and events of the fork, made once, outside any capture
        hipError_t e = hipSuccess;
        if (!b->fork) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e == hipSuccess && !b->done) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
        for (int i = 1; i < b->cs.n && e == hipSuccess; ++i) {
            if (!b->aux[i]) e = hipStreamCreateWithFlags(&b->aux[i], hipStreamNonBlocking);
            if (e == hipSuccess && !b->join[i]) e = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming);
        }
        if (e != hipSuccess) return fail_hip(e, "stream/event creation");
    }
    // survivor areas: each code gets its own (codes run concurrently); all of
    // a code's tiles in one launch when the budget allows, else the budget is
    // split evenly between the codes and their launches reuse their area.  A
    // persistent launch needs an area per resident wave only, whatever its
    // PB count (fewer waves when the budget is short).
    const int64_t budget = workspace_budget_bytes();
    int64_t fused_waves[kMaxK - kMinK + 1] = {};
    int64_t full = 0;
    for (int ci = 0; ci < b->cs.n; ++ci) full += wl.groups[ci].n_tiles * wl.groups[ci].sp_wave_dwords * 4;
    for (int K = kMinK; K <= kMaxK; ++K) {
        const FusedGroup &fg = wl.fused[K - kMinK];
        if (fg.n_descs == 0) continue;
        int64_t res = resident_waves(K);
        if (res <= 0) return fail(PBVD_EHIP, "occupancy query of the K=%d persistent kernel failed", K);
        // PBVD_PERSISTENT_WAVES caps the waves (tests: many PBs per wave)
        if (const char *env = getenv("PBVD_PERSISTENT_WAVES"))
            if (atoll(env) > 0) res = std::min<int64_t>(res, atoll(env));
        fused_waves[K - kMinK] = std::min(fg.n_descs, res);
        full += fused_waves[K - kMinK] * fg.sp_wave_dwords * 4;
    }
    int64_t per_launch[kMaxCodes], sp_off[kMaxCodes], total = 0;
    for (int ci = 0; ci < b->cs.n; ++ci) {
        const TileGroup &g = wl.groups[ci];
        int64_t n = g.n_tiles;
        if (full > budget) n = std::min(n, std::max<int64_t>(1, budget / b->cs.n / (g.sp_wave_dwords * 4)));
        per_launch[ci] = std::max<int64_t>(1, n);
        sp_off[ci] = total;
        total += g.n_tiles > 0 ? per_launch[ci] * g.sp_wave_dwords : 0;
    }
    int64_t fused_sp_off[kMaxK - kMinK + 1] = {};
    for (int K = kMinK; K <= kMaxK; ++K) {
        const FusedGroup &fg = wl.fused[K - kMinK];
        int64_t &w = fused_waves[K - kMinK];
        if (fg.n_descs == 0) continue;
        if (full > budget) w = std::min(w, std::max<int64_t>(1, budget / b->cs.n / (fg.sp_wave_dwords * 4)));
        fused_sp_off[K - kMinK] = total;
        total += w * fg.sp_wave_dwords;
    }
    st = ensure_buffer(&b->counters, &b->counters_bytes, (size_t)(kMaxK - kMinK + 1) * kCounterDwords * 4,
                       "work counters");
    if (st != PBVD_OK) return st;
    st = ensure_buffer(&b->sp, &b->sp_bytes, (size_t)std::max<int64_t>(total, 64) * 4, "survivors");
    if (st == PBVD_OK && fault_injected("batch_alloc"))
        st = fail(PBVD_ENOMEM, "injected allocation failure after the survivor area");
    if (st != PBVD_OK) return st;
    const size_t lb = std::max<size_t>(wl.lanes.size(), 1) * sizeof(pbvd::LaneDesc);
    const size_t hb = std::max<size_t>(wl.heads.size(), 1) * sizeof(pbvd::TileHead);
    st = ensure_buffer(reinterpret_cast<uint32_t **>(&b->d_lanes), &b->lanes_bytes, lb, "work list");
    if (st != PBVD_OK) return st;
    st = ensure_buffer(reinterpret_cast<uint32_t **>(&b->d_heads), &b->heads_bytes, hb, "work list");
    if (st != PBVD_OK) return st;
    const size_t db = std::max<size_t>(wl.descs.size(), 1) * sizeof(pbvd::LaneDesc);
    st = ensure_buffer(reinterpret_cast<uint32_t **>(&b->d_descs), &b->descs_bytes, db, "work list");
    if (st != PBVD_OK) return st;
    if (!wl.lanes.empty()) {
        hipError_t e = hipMemcpy(b->d_lanes, wl.lanes.data(), wl.lanes.size() * sizeof(pbvd::LaneDesc),
                                 hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_heads, wl.heads.data(), wl.heads.size() * sizeof(pbvd::TileHead),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail_hip(e, "work-list upload");
    }
    if (!wl.descs.empty()) {
        hipError_t e = hipMemcpy(b->d_descs, wl.descs.data(), wl.descs.size() * sizeof(pbvd::LaneDesc),
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail_hip(e, "work-list upload");
    }
    b->cs = cs;
    for (int ci = 0; ci < b->cs.n; ++ci) {
        b->groups[ci] = wl.groups[ci];
        b->per_launch[ci] = per_launch[ci];
        b->sp_off[ci] = sp_off[ci];
    }
    for (int k = 0; k <= kMaxK - kMinK; ++k) {
        b->fused[k] = wl.fused[k];
        b->fused_waves[k] = fused_waves[k];
        b->fused_sp_off[k] = fused_sp_off[k];
    }
    b->n_tiles = (int64_t)(wl.heads.size() + wl.descs.size());
    b->n_blocks = wl.n_blocks;
    b->n_stages = wl.n_stages;
    b->sym_bytes = sym_bytes;
    b->out_bytes = out_bytes;
    return PBVD_OK;
}

pbvd_status pbvd_batch_decode(pbvd_batch *b, const void *d_syms, uint8_t *d_out, void *hip_stream) {
    g_last_error[0] = 0;
    if (!b) return fail(PBVD_EINVAL, "batch is NULL");
    if (b->n_tiles == 0) return PBVD_OK;
    if (!d_syms || !d_out) return fail(PBVD_EINVAL, "NULL buffer");
    if (fault_injected("launch")) return fail(PBVD_EHIP, "injected launch failure");
    DeviceGuard dg(b->device);
    if (!dg.ok) return fail(PBVD_EHIP, "cannot select device %d", b->device);
    hipStream_t s = (hipStream_t)hip_stream;
    // launch units: codes with register-kernel tiles (u >= 0: code index)
    // and persistent launches (u < 0: -1 - (K - kMinK)); there are at most
    // as many as codes
    int units[kMaxCodes], n_units = 0;
    for (int ci = 0; ci < b->cs.n; ++ci)
        if (b->groups[ci].n_tiles > 0) units[n_units++] = ci;
    for (int k = 0; k <= kMaxK - kMinK; ++k)
        if (b->fused[k].n_descs > 0) units[n_units++] = -1 - k;
    if (n_units == 0) return PBVD_OK;
    auto launch_unit = [&](int u, hipStream_t st) -> pbvd_status {
        if (u >= 0)
            return launch_group(b->cs, u, b->groups[u], (const uint8_t *)d_syms, b->sym_bytes, d_out, b->d_lanes,
                                b->d_heads, b->d_descs, b->sp + b->sp_off[u], b->per_launch[u], st);
        const int k = -1 - u;
        return launch_fused(b->cs, k + kMinK, b->fused[k], (const uint8_t *)d_syms, b->sym_bytes, d_out, b->d_descs,
                            b->sp + b->fused_sp_off[k], b->fused_waves[k], b->counters + kCounterDwords * k, st);
    };
    if (n_units > 1) {
        hipError_t e = hipEventRecord(b->fork, s);
        if (e != hipSuccess) return fail_hip(e, "fork event");
    }
    // units after the first on their own streams, the first on the caller's,
    // then the caller's stream waits for all of them
    for (int k = 1; k < n_units; ++k) {
        hipError_t e = hipStreamWaitEvent(b->aux[k], b->fork, 0);
        if (e != hipSuccess) return fail_hip(e, "fork wait");
        pbvd_status st = launch_unit(units[k], b->aux[k]);
        if (st != PBVD_OK) return st;
        e = hipEventRecord(b->join[k], b->aux[k]);
        if (e != hipSuccess) return fail_hip(e, "join event");
    }
    pbvd_status st = launch_unit(units[0], s);
    if (st != PBVD_OK) return st;
    for (int k = 1; k < n_units; ++k) {
        hipError_t e = hipStreamWaitEvent(s, b->join[k], 0);
        if (e != hipSuccess) return fail_hip(e, "join wait");
    }
    // remember the end of this decode for the next pbvd_batch_set_frames
    // (not inside a graph capture: a replay's completion is the caller's)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return fail_hip(e, "capture query");
    if (cap == hipStreamCaptureStatusNone) {
        e = hipEventRecord(b->done, s);
        if (e != hipSuccess) return fail_hip(e, "completion event");
        b->done_recorded = true;
    }
    return PBVD_OK;
}

pbvd_status pbvd_batch_info(const pbvd_batch *b, int64_t *n_tiles, int64_t *n_blocks,
                            int64_t *n_forward_stages, int64_t *workspace_bytes) {
    if (!b) return fail(PBVD_EINVAL, "batch is NULL");
    if (n_tiles) *n_tiles = b->n_tiles;
    if (n_blocks) *n_blocks = b->n_blocks;
    if (n_forward_stages) *n_forward_stages = b->n_stages;
    if (workspace_bytes) *workspace_bytes = (int64_t)(b->sp_bytes + b->lanes_bytes + b->heads_bytes + b->descs_bytes);
    return PBVD_OK;
}

void pbvd_batch_destroy(pbvd_batch *b) {
    if (!b) return;
    release(b);
    delete b;
}

}  // extern "C"
