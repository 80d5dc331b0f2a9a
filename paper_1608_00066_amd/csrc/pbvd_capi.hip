// C ABI of the decoder (declared in include/pbvd.h): argument validation,
// plan and workspace management, the block decomposition of a call into
// kernel launches, and error reporting.  No C++ exception leaves this file.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "pbvd.h"
#include "pbvd_aux.hpp"
#include "pbvd_host.hpp"
#include "pbvd_registry.hpp"

#define PBVD_ROW(i, K, R, g0, g1, g2, g3) {K, R, {g0, g1, g2, g3}},
const RegisteredCode kRegisteredCodes[kNumCodes] = {PBVD_CODE_LIST(PBVD_ROW)};
#undef PBVD_ROW

namespace {

using LaunchFn = hipError_t (*)(const pbvd::LaunchRequest &);
#define PBVD_FN(i, K, R, g0, g1, g2, g3) &pbvd::launch_code<i>,
const LaunchFn kLaunchTable[kNumCodes] = {PBVD_CODE_LIST(PBVD_FN)};
#undef PBVD_FN
using WaveLaunchFn = hipError_t (*)(const pbvd::WaveLaunchRequest &);
const WaveLaunchFn kWaveLaunchTable[7] = {&pbvd::launch_wave<3>, &pbvd::launch_wave<4>, &pbvd::launch_wave<5>,
                                          &pbvd::launch_wave<6>, &pbvd::launch_wave<7>, &pbvd::launch_wave<8>,
                                          &pbvd::launch_wave<9>};
using OccupancyFn = int (*)();
const OccupancyFn kWaveOccupancyTable[7] = {
    &pbvd::wave_persistent_blocks_per_cu<3>, &pbvd::wave_persistent_blocks_per_cu<4>,
    &pbvd::wave_persistent_blocks_per_cu<5>, &pbvd::wave_persistent_blocks_per_cu<6>,
    &pbvd::wave_persistent_blocks_per_cu<7>, &pbvd::wave_persistent_blocks_per_cu<8>,
    &pbvd::wave_persistent_blocks_per_cu<9>};
using GroupLaunchFn = hipError_t (*)(const pbvd::GroupLaunchRequest &);
const GroupLaunchFn kGroupLaunchTable[7] = {
    &pbvd::launch_group_kernel<3>, &pbvd::launch_group_kernel<4>, &pbvd::launch_group_kernel<5>,
    &pbvd::launch_group_kernel<6>, &pbvd::launch_group_kernel<7>, &pbvd::launch_group_kernel<8>,
    &pbvd::launch_group_kernel<9>};
using TileLaunchFn = hipError_t (*)(const pbvd::TileLaunchRequest &);
#define PBVD_TFN(i, K, R, g0, g1, g2, g3) &pbvd::launch_tiles<i>,
const TileLaunchFn kTileLaunchTable[kNumCodes] = {PBVD_CODE_LIST(PBVD_TFN)};
#undef PBVD_TFN
#define PBVD_PFN(i, a, b) {&pbvd::launch_tiles_pair<i, pbvd::kSoftI8>, &pbvd::launch_tiles_pair<i, pbvd::kHardU8>},
const TileLaunchFn kPairLaunchTable[kNumPairs][2] = {PBVD_PAIR_LIST(PBVD_PFN)};
#undef PBVD_PFN
struct RegisteredPair {
    int first, second;  // registry indices
};
#define PBVD_PROW(i, a, b) {a, b},
const RegisteredPair kRegisteredPairs[kNumPairs] = {PBVD_PAIR_LIST(PBVD_PROW)};
#undef PBVD_PROW

int find_code(const pbvd_code &c) {
    for (int i = 0; i < kNumCodes; ++i) {
        const RegisteredCode &r = kRegisteredCodes[i];
        if (r.K != c.K || r.R != c.R) continue;
        bool same = true;
        for (int k = 0; k < c.R; ++k) same = same && r.gen[k] == c.gen[k];
        if (same) return i;
    }
    return -1;
}

}  // namespace

namespace pbvd_host {

thread_local char g_last_error[512];

pbvd_status fail(pbvd_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return s;
}

pbvd_status fail_hip(hipError_t e, const char *what) {
    return fail(PBVD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool fault_injected(const char *site) {
    const char *f = getenv("PBVD_FAULT_INJECT");
    return f && strcmp(f, site) == 0;
}

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
        ok = false;
        return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
}

DeviceGuard::~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

pbvd_status ensure_buffer(uint32_t **buf, size_t *have, size_t need, const char *what) {
    if (*have >= need) return PBVD_OK;
    if (*buf) {
        hipError_t e = hipFree(*buf);
        *buf = nullptr;
        *have = 0;
        if (e != hipSuccess) return fail_hip(e, "hipFree");
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PBVD_ENOMEM, "hipMalloc of %zu bytes for %s failed: %s", need, what,
                    hipGetErrorString(e));
    }
    *buf = (uint32_t *)p;
    *have = need;
    return PBVD_OK;
}

// Survivor dwords of one wave slot: every forward stage of a PB (at most
// D + 2L) is stored, one row per stage (or per few stages for small
// trellises); a row holds 64 >> lb PBs.
int64_t slot_dwords(const pbvd_code &c, int lb) {
    const int64_t rows = ceil_div((int64_t)c.D + 2 * (int64_t)c.L, pbvd::survivor_row_stages(c.K)) + 1;
    return ceil_div(rows * (pbvd::kWave >> lb) * pbvd::survivor_row_dwords(c.K), 64) * 64;
}

int requested_lb(const pbvd_code &c) {
    if (c.mapping == PBVD_MAP_GROUP) return kGroupLb;
    if (c.mapping == PBVD_MAP_WAVE || c.lanes_per_pb == 64) return kWaveLb;
    return c.lanes_per_pb == 8 ? 3 : c.lanes_per_pb == 4 ? 2 : c.lanes_per_pb == 2 ? 1 : c.lanes_per_pb == 1 ? 0 : -1;
}

int64_t wave_slot_dwords(const pbvd_code &c) {
    return ceil_div(pbvd::wave::pb_dwords(c.K - 1, (int64_t)c.D + 2 * (int64_t)c.L), 64) * 64;
}

bool group_tables(const pbvd_code &c, pbvd::group::GroupArgs *a) {
    if (!pbvd::group::shape_ok(c.K, c.R)) return false;
    const int V = c.K - 1, N = 1 << V, HALF = N / 2, NC = 1 << c.R, B = HALF / NC, WB = 2 * B;
    // code word c(d, x) of Eq. 2 as R bits (bit r = c^(r+1))
    auto word = [&](int d, int x) {
        const uint32_t reg = ((uint32_t)x << V) | (uint32_t)d;
        int cw = 0;
        for (int r = 0; r < c.R; ++r) cw |= (__builtin_popcount(c.gen[r] & reg) & 1) << r;
        return cw;
    };
    auto mask = [&](int cw) {
        uint32_t m = 0;
        for (int r = 0; r < c.R; ++r) m |= (uint32_t)((cw >> r) & 1) << (8 * r);
        return m;
    };
    int count[16] = {};
    for (int j = 0; j < HALF; ++j) {
        const int w = word(2 * j, 0);  // alpha, the group
        if (count[w] == B) return false;
        // beta, gamma, theta of the group follow from alpha (Eq. 4-6)
        const uint32_t m[4] = {mask(w), mask(word(2 * j, 1)), mask(word(2 * j + 1, 0)), mask(word(2 * j + 1, 1))};
        if (count[w] == 0) {
            for (int t = 0; t < 4; ++t) a->bm_mask[w][t] = m[t];
        } else {
            for (int t = 0; t < 4; ++t)
                if (a->bm_mask[w][t] != m[t]) return false;
        }
        const int b = count[w]++;
        a->jtab[w * B + b] = (uint8_t)j;
        // decision of S_j (pushed first) and S_j+N/2 of butterfly b: the
        // stage's field of group w, first pushed at its top bit
        a->ttab[j] = (uint8_t)(w * WB + 2 * b);
        a->ttab[j + HALF] = (uint8_t)(w * WB + 2 * b + 1);
    }
    for (int w = 0; w < NC; ++w)
        if (count[w] != B) return false;
    return true;
}

int64_t group_tile_dwords(const pbvd_code &c) {
    return pbvd::group::tile_dwords(c.K, c.R, (int64_t)c.D + 2 * (int64_t)c.L);
}

pbvd::wave::WaveCode wave_code(const pbvd_code &c) {
    pbvd::wave::WaveCode w{};
    for (int r = 0; r < 4; ++r) w.gen[r] = r < c.R ? c.gen[r] : 0u;
    w.R = c.R;
    w.kind = c.input_kind;
    return w;
}

hipError_t launch_wave(int K, const pbvd::WaveLaunchRequest &req) {
    if (K < 3 || K > 9) return hipErrorInvalidValue;
    return kWaveLaunchTable[K - 3](req);
}

hipError_t launch_group_kernel(int K, const pbvd::GroupLaunchRequest &req) {
    if (K < 3 || K > 9) return hipErrorInvalidValue;
    return kGroupLaunchTable[K - 3](req);
}

int64_t resident_waves(int K) {
    if (K < 3 || K > 9) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int per_cu = kWaveOccupancyTable[K - 3]();
    return (int64_t)cus * per_cu * (pbvd::kBlockThreads / pbvd::kWave);
}

int max_lb(const pbvd_code &c) {
    int lb = 0;
    while (lb < 3 && pbvd::lanes_allowed(c.K, c.pm_bits, lb + 1)) ++lb;
    return lb;
}

int64_t workspace_budget_bytes() {
    int64_t mb = 8192;
    if (const char *env = getenv("PBVD_WORKSPACE_MB")) {
        long long v = atoll(env);
        if (v > 0) mb = v;
    }
    return mb << 20;
}

// Validates one code/block parameter set and finds its registered kernels.
pbvd_status check_code(const pbvd_code &c, int *idx_out) {
    if (c.K < 3 || c.K > 9) return fail(PBVD_EINVAL, "K must be in [3, 9] (got %d)", c.K);
    if (c.R < 2 || c.R > 4) return fail(PBVD_EINVAL, "R must be in [2, 4] (got %d)", c.R);
    bool taps_input = false;
    for (int r = 0; r < c.R; ++r) {
        if (c.gen[r] >> c.K) return fail(PBVD_EINVAL, "generator %d (0%o) has bits above K-1", r, c.gen[r]);
        if (c.gen[r] == 0) return fail(PBVD_EINVAL, "generator %d is zero", r);
        taps_input = taps_input || ((c.gen[r] >> (c.K - 1)) & 1u);
    }
    if (!taps_input) return fail(PBVD_EINVAL, "no generator has bit K-1 set: constraint length is below K");
    if (c.D < 1) return fail(PBVD_EINVAL, "D must be >= 1 (got %d)", c.D);
    if (c.L < 0) return fail(PBVD_EINVAL, "L must be >= 0 (got %d)", c.L);
    if ((int64_t)c.D + 2 * (int64_t)c.L >= (1LL << 30)) return fail(PBVD_EINVAL, "D + 2L must be below 2^30");
    if (c.terminated != 0 && c.terminated != 1) return fail(PBVD_EINVAL, "terminated must be 0 or 1");
    if (c.input_kind != PBVD_SOFT_I8 && c.input_kind != PBVD_HARD_U8)
        return fail(PBVD_EINVAL, "input_kind must be PBVD_SOFT_I8 or PBVD_HARD_U8");
    if (c.pm_bits != 16 && c.pm_bits != 32) return fail(PBVD_EINVAL, "pm_bits must be 16 or 32");
    if (c.mapping != PBVD_MAP_AUTO && c.mapping != PBVD_MAP_LANES && c.mapping != PBVD_MAP_WAVE &&
        c.mapping != PBVD_MAP_GROUP)
        return fail(PBVD_EINVAL,
                    "mapping must be PBVD_MAP_AUTO, PBVD_MAP_LANES, PBVD_MAP_WAVE or PBVD_MAP_GROUP (got %d)",
                    c.mapping);
    if (c.mapping == PBVD_MAP_GROUP) {
        if (c.lanes_per_pb != 0 && c.lanes_per_pb != (1 << c.R))
            return fail(PBVD_EINVAL, "the group mapping uses 2^R = %d lanes per PB (lanes_per_pb %d)", 1 << c.R,
                        c.lanes_per_pb);
        pbvd::group::GroupArgs t{};
        if (!group_tables(c, &t))
            return fail(PBVD_ENOTSUP,
                        "the group mapping needs K - 2 - R >= 0, at most 32 decisions per group and stage, "
                        "and 2^R butterfly groups of one size (K=%d R=%d)",
                        c.K, c.R);
        if ((int64_t)c.D + 2 * (int64_t)c.L > (1 << 20))
            return fail(PBVD_ENOTSUP, "the group mapping's 32-bit metrics take D + 2L <= 2^20");
        *idx_out = -1;
        return PBVD_OK;
    }
    if (c.lanes_per_pb != 0 && c.lanes_per_pb != 1 && c.lanes_per_pb != 2 && c.lanes_per_pb != 4 &&
        c.lanes_per_pb != 8 && c.lanes_per_pb != 64)
        return fail(PBVD_EINVAL, "lanes_per_pb must be 0, 1, 2, 4, 8 or 64 (got %d)", c.lanes_per_pb);
    const bool wave_only = c.mapping == PBVD_MAP_WAVE || c.lanes_per_pb == 64;
    if (c.mapping == PBVD_MAP_WAVE && c.lanes_per_pb != 0 && c.lanes_per_pb != 64)
        return fail(PBVD_EINVAL, "the wave mapping uses 64 lanes per PB (lanes_per_pb %d)", c.lanes_per_pb);
    if (c.mapping == PBVD_MAP_LANES && c.lanes_per_pb == 64)
        return fail(PBVD_EINVAL, "the register mapping uses 1, 2, 4 or 8 lanes per PB, not 64");
    {
        // survivor words of one PB of the wave kernel use 32-bit offsets
        const int64_t slot = wave_slot_dwords(c) * 4;
        if (slot >= (1LL << 31) - 4096)
            return fail(PBVD_ENOTSUP, "D + 2L too large for the survivor buffer of one PB (%lld bytes)",
                        (long long)slot);
    }
    const int idx = find_code(c);
    if (wave_only) {
        *idx_out = -1;
        return PBVD_OK;
    }
    // the register kernel: compiled generator sets, 32-bit metrics up to K = 8
    const bool want_lanes = c.mapping == PBVD_MAP_LANES || c.lanes_per_pb != 0;
    const bool lanes_ok = idx >= 0 && !(c.pm_bits == 32 && c.K > 8);
    if (!lanes_ok && want_lanes)
        return fail(PBVD_ENOTSUP, idx < 0 ? "no register kernel compiled for this generator set "
                                            "(PBVD_MAP_WAVE or PBVD_MAP_AUTO decode any code)"
                                          : "the register kernel's 32-bit path metrics need K <= 8");
    if (c.lanes_per_pb > 1 && !pbvd::lanes_allowed(c.K, c.pm_bits, requested_lb(c)))
        return fail(PBVD_ENOTSUP, "%d lanes per PB need 16-bit metrics and K >= %d", c.lanes_per_pb,
                    c.lanes_per_pb == 2 ? 7 : c.lanes_per_pb == 4 ? 8 : 9);
    if (lanes_ok) {
        // survivor rows of one wave slot are addressed with 32-bit offsets
        const int64_t row_bytes = 64LL * pbvd::survivor_row_dwords(c.K) * 4;
        const int64_t slot =
            (((int64_t)c.D + 2 * (int64_t)c.L) / pbvd::survivor_row_stages(c.K) + 2) * row_bytes;
        if (slot >= (1LL << 31) - 4096)
            return fail(PBVD_ENOTSUP, "D + 2L too large for the survivor buffer of one wave (%lld bytes)",
                        (long long)slot);
    }
    *idx_out = lanes_ok ? idx : -1;
    return PBVD_OK;
}

hipError_t launch_tiles(int code_idx, const pbvd::TileLaunchRequest &req) {
    return kTileLaunchTable[code_idx](req);
}

int find_pair(int idx_a, int idx_b, bool *a_first) {
    for (int i = 0; i < kNumPairs; ++i) {
        const RegisteredPair &p = kRegisteredPairs[i];
        if ((p.first == idx_a && p.second == idx_b) || (p.first == idx_b && p.second == idx_a)) {
            *a_first = p.first == idx_a;
            return i;
        }
    }
    return -1;
}

hipError_t launch_tiles_pair(int pair_idx, const pbvd::TileLaunchRequest &req) {
    if (req.input_kind != pbvd::kSoftI8 && req.input_kind != pbvd::kHardU8) return hipErrorInvalidValue;
    return kPairLaunchTable[pair_idx][req.input_kind == pbvd::kHardU8 ? 1 : 0](req);
}

}  // namespace pbvd_host

using namespace pbvd_host;

namespace {

// Block decomposition of one call (Sec. III-A with M = L): PBs with the full
// forward range [bD-L, bD+D+L) and decoded range [bD, bD+D) are "interior"
// and go 64 >> lb to a wave; the others (stream ends) fill the slots the
// interior leaves free (n_fold of them, in wave 0) and then get a wave each.
// PBs that start their traceback from the best state (the end of an
// unterminated stream) are not folded: a wave takes all final metrics at one
// stage.  For the same reason nothing is folded when the caller asks for
// final metrics.  Folding runs wave 0 with per-lane geometry, a little slower
// than the others, so it is done only where it saves a wave on the busiest
// SIMD: when ceil(waves / SIMDs) drops (fold_simds = the device's SIMD count;
// 0 = never fold).
struct CallGeometry {
    int64_t T, pb_first, pb_end;
    int64_t b_lo, b_hi, n_head, n_tail, n_fold;
    int64_t n_int_waves, n_waves;
    int64_t out_bits;
};

CallGeometry call_geometry(const pbvd_code &c, int64_t n, int64_t pb_first, int64_t pb_count, int lb,
                           int64_t fold_simds = 0) {
    CallGeometry g{};
    const int64_t D = c.D, L = c.L;
    g.T = n + (c.terminated ? c.K - 1 : 0);
    g.pb_first = pb_first;
    g.pb_end = pb_first + pb_count;
    int64_t lo = ceil_div(L, D);
    if (lo < pb_first) lo = pb_first;
    // interior: bD + D + L <= T and bD + D <= n; on an unterminated stream a
    // block ending exactly at T starts its traceback from the best state,
    // so it is handled as an edge block
    const int64_t tlim = g.T - D - L - (c.terminated ? 0 : 1);
    const int64_t lim = tlim < (n - D) ? tlim : (n - D);
    int64_t hi = lim < 0 ? 0 : lim / D + 1;
    if (hi > g.pb_end) hi = g.pb_end;
    if (lo < hi) {
        g.b_lo = lo;
        g.b_hi = hi;
        g.n_head = lo - pb_first;
        g.n_tail = g.pb_end - hi;
        const int64_t pw = pbvd::kWave >> lb;
        g.n_int_waves = ceil_div(hi - lo, pw);
        const int64_t spare = g.n_int_waves * pw - (hi - lo);
        const int64_t foldable = c.terminated ? g.n_head + g.n_tail : g.n_head;
        const int64_t n_fold = spare < foldable ? spare : foldable;
        const int64_t w = g.n_int_waves + g.n_head + g.n_tail;
        if (fold_simds > 0 && ceil_div(w - n_fold, fold_simds) < ceil_div(w, fold_simds)) g.n_fold = n_fold;
    } else {
        g.b_lo = g.b_hi = g.pb_end;
        g.n_head = pb_count;
        g.n_tail = 0;
        g.n_int_waves = 0;
    }
    g.n_waves = g.n_int_waves + g.n_head + g.n_tail - g.n_fold;
    const int64_t end_bit = g.pb_end * D < n ? g.pb_end * D : n;
    g.out_bits = pb_count > 0 ? end_bit - pb_first * D : 0;
    return g;
}

// Wide-fetch bounds of wave 0 when it holds folded edge PBs: every lane
// fetches the symbols of a trip with one window of trip_fetch_dwords dwords,
// never past its own last trip.  *i_safe is the last trip start at which
// every lane's window is inside the T*R input bytes; *wide is 1 when all of
// them are (mirrors the kernel's per-lane geometry of that wave).
void fold_fetch_bounds(const pbvd_code &c, const CallGeometry &g, int32_t *i_safe, int32_t *wide) {
    const int64_t D = c.D, L = c.L, R = c.R;
    const int64_t len = D + 2 * L;
    *i_safe = (int32_t)len;
    *wide = 1;
    if (g.n_fold == 0) return;
    const int64_t U = pbvd::trip_stages(c.K);
    const int64_t ND = pbvd::trip_fetch_dwords(c.K, c.R);
    const int64_t in_bytes = g.T * R;
    const int64_t n_pb = g.n_fold + (g.b_hi - g.b_lo);
    int64_t lim = len;
    for (int64_t s = 0; s < n_pb && s < pbvd::kWave; ++s) {
        const int64_t b = s < g.n_fold ? (s < g.n_head ? g.pb_first + s : g.b_hi + (s - g.n_head))
                                       : g.b_lo + (s - g.n_fold);
        const int64_t d0 = b * D;
        const int64_t f0 = d0 - L < 0 ? 0 : d0 - L;
        const int64_t f1 = d0 + D + L > g.T ? g.T : d0 + D + L;
        const int64_t last_trip = ((f1 - f0 - 1) / U) * U;
        if (f0 * R + last_trip * R + 4 * ND <= in_bytes) continue;
        *wide = 0;
        const int64_t room = in_bytes - f0 * R - 4 * ND;
        const int64_t i = room < 0 ? -1 : room / R;
        if (i < lim) lim = i;
    }
    *i_safe = (int32_t)lim;
}

}  // namespace

namespace {

// Device scratch of one decode in flight: survivor rows of one launch and the
// output staging words (used when D % 32 != 0 or the output is unaligned).
// A fixed workspace is carved from the library's static scratch: it is
// never grown or freed, and a call that needs more fails.
struct Workspace {
    uint32_t *sp = nullptr;
    size_t sp_bytes = 0;
    uint32_t *words = nullptr;
    size_t words_bytes = 0;
    bool fixed = false;
};

void free_workspace(Workspace &w) {
    if (!w.fixed) {
        if (w.sp) (void)hipFree(w.sp);
        if (w.words) (void)hipFree(w.words);
    }
    w = Workspace{};
}

// Survivor area / output staging of at least `need` bytes.
pbvd_status ws_survivors(Workspace &ws, size_t need) {
    if (!ws.fixed) return ensure_buffer(&ws.sp, &ws.sp_bytes, need, "survivors");
    if (need > ws.sp_bytes)
        return fail(PBVD_EINVAL, "survivors of one launch need %zu bytes, the static scratch has %zu", need,
                    ws.sp_bytes);
    return PBVD_OK;
}
pbvd_status ws_staging(Workspace &ws, size_t need) {
    if (!ws.fixed) return ensure_buffer(&ws.words, &ws.words_bytes, need, "output staging");
    if (need > ws.words_bytes)
        return fail(PBVD_EINVAL, "output staging needs %zu bytes, the static scratch has %zu", need,
                    ws.words_bytes);
    return PBVD_OK;
}

constexpr int kMaxPipeStreams = 8;

// Host-buffer decoding (pbvd_decode_host): per stream a workspace, device
// chunk buffers and pinned staging, grown on demand.
struct PipeStream {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Workspace ws;
    uint8_t *d_in = nullptr, *d_out = nullptr;
    size_t d_in_bytes = 0, d_out_bytes = 0;
    uint8_t *h_in = nullptr, *h_out = nullptr;    // pinned staging
    size_t h_in_bytes = 0, h_out_bytes = 0;
    // chunk whose bits still wait in h_out (staged mode)
    int64_t pend_byte = -1, pend_bytes = 0;
};

}  // namespace

namespace {

// Static device scratch of pbvd_decode_ex_noalloc: survivor rows and output
// staging for callers that cannot allocate.  Every device the library runs
// on holds one copy from the moment the library's code object is loaded
// until the process ends; calls on one device share it.
constexpr size_t kStaticScratchBytes = PBVD_STATIC_SCRATCH_BYTES;
__device__ __align__(256) uint32_t scratch[kStaticScratchBytes / 4];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current: looked
// up once per device (the array's name is a host-side stand-in, not an
// address the kernels can use).
pbvd_status static_scratch(int dev, uint32_t **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(PBVD_EINVAL, "device %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail_hip(e == hipSuccess ? hipErrorInvalidSymbol : e, "static scratch address");
        }
        g_scratch_ptr[dev] = (uint32_t *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return PBVD_OK;
}

}  // namespace

struct pbvd_plan {
    pbvd_code code;
    int code_idx;             // register kernel's registry index, -1: none
    int64_t wave_max_pbs;     // auto mapping: the wave kernel up to this many PBs
    pbvd::group::GroupArgs gt;  // group mapping: the code's tables
    int device;
    int ndw;                  // survivor dwords per stored row
    int row_stages;           // stages per stored row
    int64_t budget_bytes;     // survivor workspace limit
    int64_t n_simd;           // SIMDs of the device (4 per compute unit)
    Workspace ws;             // pbvd_decode / pbvd_decode_ex
    PipeStream pipe[kMaxPipeStreams];
};

namespace {

// Waves (or PBs of the wave kernel) of one launch: as many survivor slots of
// sp_wave_dwords as the budget holds, at least one; a fixed workspace holds
// what fits it (possibly none).
int64_t launch_limit(const pbvd_plan *p, const Workspace &ws, int64_t sp_wave_dwords) {
    int64_t w = p->budget_bytes / (sp_wave_dwords * 4);
    if (w < 1) w = 1;
    if (ws.fixed) w = std::min<int64_t>(w, (int64_t)(ws.sp_bytes / (size_t)(sp_wave_dwords * 4)));
    return w;
}

// Lanes per PB of one call: the code's choice, or else
//   one lane per PB for trellises of at most 64 states (32 packed registers)
//   when that gives 4 waves per SIMD (4096): enough to hide latency;
//   pairs of lanes where the code allows them when that gives every SIMD a
//   wave (fewer registers per lane, so more waves hide each other's latency);
//   the largest group the code allows otherwise (short streams).
int call_lb(const pbvd_plan *p, int64_t n_bits, int64_t pb_first, int64_t pb_count) {
    const int req = requested_lb(p->code);
    if (req >= 0) return req;
    // PBVD_MAP_LANES keeps the register kernel whatever the PB count
    if (p->code_idx < 0 || (p->code.mapping != PBVD_MAP_LANES && pb_count <= p->wave_max_pbs)) return kWaveLb;
    const int top = max_lb(p->code);
    if (top == 0) return 0;
    if (p->code.K <= 7 && call_geometry(p->code, n_bits, pb_first, pb_count, 0).n_waves >= 4096) return 0;
    return call_geometry(p->code, n_bits, pb_first, pb_count, 1).n_waves >= 1024 ? 1 : top;
}

pbvd_status validate_call(const pbvd_plan *p, const void *d_syms, int64_t n_bits, int64_t pb_first,
                          int64_t pb_count, const uint8_t *d_out) {
    if (!p) return fail(PBVD_EINVAL, "plan is NULL");
    if (!d_syms) return fail(PBVD_EINVAL, "d_syms is NULL");
    if (n_bits < 1) return fail(PBVD_EINVAL, "n_bits must be >= 1 (got %lld)", (long long)n_bits);
    const int64_t nb = ceil_div(n_bits, p->code.D);
    if (pb_first < 0 || pb_count < 0 || pb_first > nb || pb_count > nb - pb_first)
        return fail(PBVD_EINVAL, "PB range [%lld, %lld) outside [0, %lld)", (long long)pb_first,
                    (long long)(pb_first + pb_count), (long long)nb);
    if (pb_count > 0 && !d_out) return fail(PBVD_EINVAL, "d_out_bits is NULL");
    return PBVD_OK;
}

// The state-parallel kernel for one call: one wave per PB, in launches of
// as many PBs as the survivor workspace holds.
pbvd_status run_decode_wave(pbvd_plan *p, Workspace &ws, const void *d_syms, int64_t n_bits,
                            int64_t pb_first, int64_t pb_count, uint8_t *d_out, int32_t *d_final_pm,
                            hipStream_t stream, CallGeometry *geo_out, bool single_launch) {
    const pbvd_code &c = p->code;
    const int64_t D = c.D;
    const int64_t T = n_bits + (c.terminated ? c.K - 1 : 0);
    if (geo_out) {
        *geo_out = CallGeometry{};
        geo_out->T = T;
        geo_out->pb_first = pb_first;
        geo_out->pb_end = pb_first + pb_count;
        geo_out->n_waves = pb_count;
    }
    if (pb_count == 0) return PBVD_OK;
    const int64_t slot = wave_slot_dwords(c);
    // single_launch (the debug survivor export): each wave also stores its
    // per-stage decisions, after the path words of all waves
    const int64_t per_launch = launch_limit(p, ws, single_launch ? 2 * slot : slot);
    if (per_launch < 1)
        return fail(PBVD_EINVAL, "one PB's survivors (%lld bytes) do not fit the static scratch",
                    (long long)(slot * 4));
    if (single_launch && pb_count > per_launch)
        return fail(PBVD_EINVAL, "%lld PBs do not fit one launch (limit %lld)", (long long)pb_count,
                    (long long)per_launch);
    if (fault_injected("launch")) return fail(PBVD_EHIP, "injected launch failure");
    const int64_t launch_pbs = std::min(pb_count, per_launch);
    pbvd_status st = ws_survivors(ws, (size_t)(launch_pbs * slot * 4 * (single_launch ? 2 : 1)));
    if (st != PBVD_OK) return st;
    const int64_t end_bit = std::min(n_bits, (pb_first + pb_count) * D);
    const int64_t out_bits = end_bit - pb_first * D;
    const int64_t out_bytes = ceil_div(out_bits, 8);
    const bool direct = (D % 32 == 0) && (((uintptr_t)d_out & 3u) == 0);
    if (!direct) {
        const int64_t nwords = ceil_div(out_bits, 32) + 2;
        st = ws_staging(ws, (size_t)nwords * 4);
        if (st != PBVD_OK) return st;
        hipError_t e = pbvd::fill_u32(ws.words, nwords, 0u, stream);
        if (e != hipSuccess) return fail_hip(e, "zero-fill launch");
    }
    pbvd::WaveLaunchRequest req{};
    pbvd::wave::Args &a = req.args;
    a.syms = (const uint8_t *)d_syms;
    a.in_end = a.syms + T * c.R;
    a.out = d_out;
    a.out_words = direct ? nullptr : ws.words;
    a.out_bytes = out_bytes;
    a.final_pm = d_final_pm;
    a.sp = ws.sp;
    a.sp_wave_dwords = slot;
    a.n = n_bits;
    a.T = T;
    a.pb_first = pb_first;
    a.D = c.D;
    a.L = c.L;
    a.terminated = c.terminated;
    a.out_mode = direct ? pbvd::kOutDirect : pbvd::kOutAtomic;
    a.descs = nullptr;
    a.dec_sp = single_launch ? ws.sp + launch_pbs * slot : nullptr;
    a.codes[0] = wave_code(c);
    req.stream = stream;
    const int waves_per_block = pbvd::kBlockThreads / pbvd::kWave;
    for (int64_t w0 = 0; w0 < pb_count; w0 += launch_pbs) {
        a.wave_begin = w0;
        a.n_waves = std::min(launch_pbs, pb_count - w0);
        req.grid = (unsigned)ceil_div(a.n_waves, waves_per_block);
        hipError_t e = launch_wave(c.K, req);
        if (e != hipSuccess) return fail_hip(e, "wave decode kernel launch");
    }
    if (!direct) {
        hipError_t e = pbvd::words_to_bytes(ws.words, d_out, out_bytes, stream);
        if (e != hipSuccess) return fail_hip(e, "output copy launch");
    }
    return PBVD_OK;
}

// The group-mapped kernel for one call: tiles of 64 consecutive PBs, in
// launches of as many tiles as the survivor workspace holds.
pbvd_status run_decode_group(pbvd_plan *p, Workspace &ws, const void *d_syms, int64_t n_bits,
                             int64_t pb_first, int64_t pb_count, uint8_t *d_out, int32_t *d_final_pm,
                             hipStream_t stream, CallGeometry *geo_out, bool single_launch) {
    const pbvd_code &c = p->code;
    const int64_t D = c.D;
    const int64_t T = n_bits + (c.terminated ? c.K - 1 : 0);
    const int64_t tiles = ceil_div(pb_count, pbvd::group::kTilePbs);
    if (geo_out) {
        *geo_out = CallGeometry{};
        geo_out->T = T;
        geo_out->pb_first = pb_first;
        geo_out->pb_end = pb_first + pb_count;
        geo_out->n_waves = tiles << c.R;
    }
    if (pb_count == 0) return PBVD_OK;
    if (single_launch) return fail(PBVD_ENOTSUP, "the group mapping has no survivor export");
    const int64_t slot = group_tile_dwords(c);
    const int64_t per_launch = launch_limit(p, ws, slot);
    if (per_launch < 1)
        return fail(PBVD_EINVAL, "one tile's survivors (%lld bytes) do not fit the static scratch",
                    (long long)(slot * 4));
    if (fault_injected("launch")) return fail(PBVD_EHIP, "injected launch failure");
    const int64_t launch_tiles = std::min(tiles, per_launch);
    pbvd_status st = ws_survivors(ws, (size_t)(launch_tiles * slot * 4));
    if (st != PBVD_OK) return st;
    const int64_t end_bit = std::min(n_bits, (pb_first + pb_count) * D);
    const int64_t out_bits = end_bit - pb_first * D;
    const int64_t out_bytes = ceil_div(out_bits, 8);
    const bool direct = (D % 32 == 0) && (((uintptr_t)d_out & 3u) == 0);
    if (!direct) {
        const int64_t nwords = ceil_div(out_bits, 32) + 2;
        st = ws_staging(ws, (size_t)nwords * 4);
        if (st != PBVD_OK) return st;
        hipError_t e = pbvd::fill_u32(ws.words, nwords, 0u, stream);
        if (e != hipSuccess) return fail_hip(e, "zero-fill launch");
    }
    pbvd::GroupLaunchRequest req{};
    pbvd::group::GroupArgs &a = req.args;
    a = p->gt;
    a.syms = (const uint8_t *)d_syms;
    a.in_end = a.syms + T * c.R;
    a.out = d_out;
    a.out_words = direct ? nullptr : ws.words;
    a.out_bytes = out_bytes;
    a.out_mode = direct ? pbvd::kOutDirect : pbvd::kOutAtomic;
    a.kind = c.input_kind;
    a.final_pm = d_final_pm;
    a.sp = ws.sp;
    a.sp_tile_dwords = slot;
    a.n = n_bits;
    a.T = T;
    a.pb_first = pb_first;
    a.pb_count = pb_count;
    a.D = c.D;
    a.L = c.L;
    a.terminated = c.terminated;
    a.descs = nullptr;
    req.R = c.R;
    req.stream = stream;
    for (int64_t t0 = 0; t0 < tiles; t0 += launch_tiles) {
        a.tile_begin = t0;
        a.n_tiles = std::min(launch_tiles, tiles - t0);
        req.grid = (unsigned)a.n_tiles;
        hipError_t e = launch_group_kernel(c.K, req);
        if (e != hipSuccess) return fail_hip(e, "group decode kernel launch");
    }
    if (!direct) {
        hipError_t e = pbvd::words_to_bytes(ws.words, d_out, out_bytes, stream);
        if (e != hipSuccess) return fail_hip(e, "output copy launch");
    }
    return PBVD_OK;
}

// Runs the decode kernels of one call; fills *geo with the decomposition.
pbvd_status run_decode(pbvd_plan *p, Workspace &ws, const void *d_syms, int64_t n_bits,
                       int64_t pb_first, int64_t pb_count, uint8_t *d_out, int32_t *d_final_pm,
                       hipStream_t stream, CallGeometry *geo_out, bool single_launch,
                       int *lb_out = nullptr) {
    const pbvd_code &c = p->code;
    const int lb = call_lb(p, n_bits, pb_first, pb_count);
    if (lb == kWaveLb) {
        if (lb_out) *lb_out = lb;
        return run_decode_wave(p, ws, d_syms, n_bits, pb_first, pb_count, d_out, d_final_pm, stream,
                               geo_out, single_launch);
    }
    if (lb == kGroupLb) {
        if (lb_out) *lb_out = lb;
        return run_decode_group(p, ws, d_syms, n_bits, pb_first, pb_count, d_out, d_final_pm, stream,
                                geo_out, single_launch);
    }
    const int64_t sp_wave_dwords = slot_dwords(c, lb);
    const CallGeometry g = call_geometry(c, n_bits, pb_first, pb_count, lb, d_final_pm ? 0 : p->n_simd);
    if (geo_out) *geo_out = g;
    if (lb_out) *lb_out = lb;
    if (pb_count == 0) return PBVD_OK;
    const int64_t per_launch = launch_limit(p, ws, sp_wave_dwords);
    if (per_launch < 1)
        return fail(PBVD_EINVAL, "one wave's survivors (%lld bytes) do not fit the static scratch",
                    (long long)(sp_wave_dwords * 4));
    if (single_launch && g.n_waves > per_launch)
        return fail(PBVD_EINVAL, "%lld waves do not fit one launch (limit %lld)",
                    (long long)g.n_waves, (long long)per_launch);
    if (fault_injected("launch")) return fail(PBVD_EHIP, "injected launch failure");

    const int64_t launch_waves = g.n_waves < per_launch ? g.n_waves : per_launch;
    pbvd_status st = ws_survivors(ws, (size_t)(launch_waves * sp_wave_dwords * 4));
    if (st != PBVD_OK) return st;

    const int64_t out_bytes = ceil_div(g.out_bits, 8);
    const bool direct = (c.D % 32 == 0) && (((uintptr_t)d_out & 3u) == 0);
    if (!direct) {
        const int64_t nwords = ceil_div(g.out_bits, 32) + 2;
        st = ws_staging(ws, (size_t)nwords * 4);
        if (st != PBVD_OK) return st;
        hipError_t e = pbvd::fill_u32(ws.words, nwords, 0u, stream);
        if (e != hipSuccess) return fail_hip(e, "zero-fill launch");
    }

    pbvd::LaunchRequest req{};
    pbvd::KernelArgs &a = req.args;
    a.syms = (const uint8_t *)d_syms;
    a.out = d_out;
    a.out_words = direct ? nullptr : ws.words;
    a.final_pm = d_final_pm;
    a.sp = ws.sp;
    a.n = n_bits;
    a.T = g.T;
    a.pb_first = pb_first;
    a.b_lo = g.b_lo;
    a.b_hi = g.b_hi;
    a.n_head = g.n_head;
    a.n_fold = g.n_fold;
    a.n_int_waves = g.n_int_waves;
    fold_fetch_bounds(c, g, &a.fold_i_safe, &a.fold_wide);
    a.out_bytes = out_bytes;
    a.sp_wave_dwords = sp_wave_dwords;
    a.D = c.D;
    a.L = c.L;
    a.terminated = c.terminated;
    a.direct_out = direct ? 1 : 0;
    req.pm_bits = c.pm_bits;
    req.input_kind = c.input_kind;
    req.lb = lb;
    req.stream = stream;
    const int waves_per_block = pbvd::kBlockThreads / pbvd::kWave;
    for (int64_t w0 = 0; w0 < g.n_waves; w0 += launch_waves) {
        a.wave_begin = w0;
        a.n_waves = (g.n_waves - w0) < launch_waves ? (g.n_waves - w0) : launch_waves;
        req.grid = (unsigned)ceil_div(a.n_waves, waves_per_block);
        hipError_t e = kLaunchTable[p->code_idx](req);
        if (e != hipSuccess) return fail_hip(e, "decode kernel launch");
    }
    if (!direct) {
        hipError_t e = pbvd::words_to_bytes(ws.words, d_out, out_bytes, stream);
        if (e != hipSuccess) return fail_hip(e, "output copy launch");
    }
    return PBVD_OK;
}

}  // namespace

extern "C" {

pbvd_status pbvd_create(const pbvd_code *code, pbvd_plan **out) {
    g_last_error[0] = 0;
    if (!code || !out) return fail(PBVD_EINVAL, "code and out must not be NULL");
    const pbvd_code &c = *code;
    int idx = -1;
    pbvd_status vs = check_code(c, &idx);
    if (vs != PBVD_OK) return vs;
    pbvd_plan *p = new (std::nothrow) pbvd_plan();
    if (!p) return fail(PBVD_ENOMEM, "host allocation failed");
    p->code = c;
    for (int r = c.R; r < 4; ++r) p->code.gen[r] = 0;
    p->code_idx = idx;
    if (c.mapping == PBVD_MAP_GROUP) (void)group_tables(p->code, &p->gt);  // checked by check_code
    if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
    (void)hipGetLastError();
    p->ndw = pbvd::survivor_row_dwords(c.K);
    p->row_stages = pbvd::survivor_row_stages(c.K);
    p->budget_bytes = workspace_budget_bytes();
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cus < 1)
        cus = 256;
    (void)hipGetLastError();
    p->n_simd = 4 * (int64_t)cus;
    // the wave kernel runs a PB 64 lanes wide; the register kernel is faster
    // once a call has enough PBs to fill the device with lanes
    p->wave_max_pbs = c.K <= 7 ? 16384 : 8192;
    if (const char *env = getenv("PBVD_WAVE_MAX_PBS")) p->wave_max_pbs = atoll(env);
    {
        // set up the static scratch of this device (pbvd_decode_ex_noalloc);
        // a failure here is reported by that call, which tries again
        uint32_t *unused = nullptr;
        DeviceGuard dg(p->device);
        if (dg.ok && static_scratch(p->device, &unused) != PBVD_OK) g_last_error[0] = 0;
    }
    // PBVD_FOLD_SIMDS overrides the SIMD count of the edge-folding rule
    // (1: fold whenever it saves a wave, 0: never fold)
    if (const char *env = getenv("PBVD_FOLD_SIMDS")) p->n_simd = atoll(env) < 0 ? 0 : atoll(env);
    *out = p;
    return PBVD_OK;
}

pbvd_status pbvd_decode_ex(pbvd_plan *p, const void *d_syms, int64_t n_bits, int64_t pb_first,
                           int64_t pb_count, uint8_t *d_out_bits, int32_t *d_final_pm,
                           void *hip_stream) {
    g_last_error[0] = 0;
    pbvd_status st = validate_call(p, d_syms, n_bits, pb_first, pb_count, d_out_bits);
    if (st != PBVD_OK || pb_count == 0) return st;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(PBVD_EHIP, "cannot select device %d", p->device);
    return run_decode(p, p->ws, d_syms, n_bits, pb_first, pb_count, d_out_bits, d_final_pm,
                      (hipStream_t)hip_stream, nullptr, false);
}

pbvd_status pbvd_decode_ex_noalloc(pbvd_plan *p, const void *d_syms, int64_t n_bits, int64_t pb_first,
                                   int64_t pb_count, uint8_t *d_out_bits, int32_t *d_final_pm,
                                   void *hip_stream) {
    g_last_error[0] = 0;
    pbvd_status st = validate_call(p, d_syms, n_bits, pb_first, pb_count, d_out_bits);
    if (st != PBVD_OK || pb_count == 0) return st;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(PBVD_EHIP, "cannot select device %d", p->device);
    uint32_t *base = nullptr;
    st = static_scratch(p->device, &base);
    if (st != PBVD_OK) return st;
    // [output staging (only for unaligned output) | survivor rows]
    const int64_t D = p->code.D;
    const int64_t end_bit = std::min(n_bits, (pb_first + pb_count) * D);
    const int64_t out_bits = end_bit - pb_first * D;
    const bool direct = (D % 32 == 0) && (((uintptr_t)d_out_bits & 3u) == 0);
    const size_t staging = direct ? 0 : (size_t)ceil_div((ceil_div(out_bits, 32) + 2) * 4, 256) * 256;
    if (staging >= kStaticScratchBytes)
        return fail(PBVD_EINVAL, "output staging of %lld bits needs %zu bytes, more than the %zu-byte static "
                                 "scratch (use a 4-byte aligned output and D %% 32 == 0, or pbvd_decode_ex)",
                    (long long)out_bits, staging, kStaticScratchBytes);
    Workspace ws;
    ws.fixed = true;
    ws.words = base;
    ws.words_bytes = staging;
    ws.sp = base + staging / 4;
    ws.sp_bytes = kStaticScratchBytes - staging;
    return run_decode(p, ws, d_syms, n_bits, pb_first, pb_count, d_out_bits, d_final_pm,
                      (hipStream_t)hip_stream, nullptr, false);
}

pbvd_status pbvd_decode(pbvd_plan *p, const void *d_syms, int64_t n_bits, uint8_t *d_out_bits,
                        void *hip_stream) {
    if (!p) return fail(PBVD_EINVAL, "plan is NULL");
    if (n_bits < 1) return fail(PBVD_EINVAL, "n_bits must be >= 1 (got %lld)", (long long)n_bits);
    return pbvd_decode_ex(p, d_syms, n_bits, 0, ceil_div(n_bits, p->code.D), d_out_bits, nullptr,
                          hip_stream);
}

int32_t pbvd_call_lanes(const pbvd_plan *p, int64_t n_bits, int64_t pb_first, int64_t pb_count) {
    if (!p || n_bits < 1 || pb_first < 0 || pb_count < 0) return 0;
    const int lb = call_lb(p, n_bits, pb_first, pb_count);
    return lb == kGroupLb ? 1 << p->code.R : 1 << lb;
}

int64_t pbvd_num_blocks(const pbvd_plan *p, int64_t n_bits) {
    if (!p || n_bits < 1) return 0;
    return ceil_div(n_bits, p->code.D);
}

pbvd_status pbvd_block_geometry(const pbvd_plan *p, int64_t n_bits, int64_t pb_first,
                                int64_t pb_count, int64_t *out) {
    g_last_error[0] = 0;
    if (!p) return fail(PBVD_EINVAL, "plan is NULL");
    if (n_bits < 1) return fail(PBVD_EINVAL, "n_bits must be >= 1");
    const int64_t nb = ceil_div(n_bits, p->code.D);
    if (pb_first < 0 || pb_count < 0 || pb_first > nb || pb_count > nb - pb_first)
        return fail(PBVD_EINVAL, "PB range outside [0, %lld)", (long long)nb);
    if (pb_count > 0 && !out) return fail(PBVD_EINVAL, "out is NULL");
    const int64_t D = p->code.D, L = p->code.L;
    const int64_t T = n_bits + (p->code.terminated ? p->code.K - 1 : 0);
    for (int64_t i = 0; i < pb_count; ++i) {
        const int64_t d0 = (pb_first + i) * D;
        out[4 * i + 0] = d0 - L < 0 ? 0 : d0 - L;
        out[4 * i + 1] = d0 + D + L > T ? T : d0 + D + L;
        out[4 * i + 2] = d0;
        out[4 * i + 3] = d0 + D > n_bits ? n_bits : d0 + D;
    }
    return PBVD_OK;
}

pbvd_status pbvd_debug_survivors(pbvd_plan *p, const void *d_syms, int64_t n_bits,
                                 int64_t pb_first, int64_t pb_count, uint8_t *d_out_bits,
                                 uint8_t *d_dec, void *hip_stream) {
    g_last_error[0] = 0;
    pbvd_status st = validate_call(p, d_syms, n_bits, pb_first, pb_count, d_out_bits);
    if (st != PBVD_OK) return st;
    if (pb_count > 0 && !d_dec) return fail(PBVD_EINVAL, "d_dec is NULL");
    if (pb_count == 0) return PBVD_OK;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(PBVD_EHIP, "cannot select device %d", p->device);
    hipStream_t s = (hipStream_t)hip_stream;
    CallGeometry g{};
    int lb = 0;
    st = run_decode(p, p->ws, d_syms, n_bits, pb_first, pb_count, d_out_bits, nullptr, s, &g, true, &lb);
    if (st != PBVD_OK || pb_count == 0) return st;
    pbvd::SurvivorView v{};
    // the state-parallel kernel's per-stage decisions follow its path words
    v.sp = lb == kWaveLb ? p->ws.sp + pb_count * wave_slot_dwords(p->code) : p->ws.sp;
    v.wave = lb == kWaveLb ? 1 : 0;
    v.sp_wave_dwords = lb == kWaveLb ? wave_slot_dwords(p->code) : slot_dwords(p->code, lb);
    v.lb = lb;
    v.T = g.T;
    v.pb_first = pb_first;
    v.pb_count = pb_count;
    v.b_lo = g.b_lo;
    v.b_hi = g.b_hi;
    v.n_head = g.n_head;
    v.n_fold = g.n_fold;
    v.n_int_waves = g.n_int_waves;
    v.K = p->code.K;
    v.D = p->code.D;
    v.L = p->code.L;
    v.byte_perm = (p->code.pm_bits == 16 && p->code.K >= 6) ? 1 : 0;
    hipError_t e = pbvd::unpack_survivors(v, d_dec, s);
    if (e != hipSuccess) return fail_hip(e, "survivor expansion launch");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    return PBVD_OK;
}

pbvd_status pbvd_debug_group_table(const pbvd_code *code, int32_t *alpha, int32_t *masks) {
    g_last_error[0] = 0;
    if (!code || !alpha || !masks) return fail(PBVD_EINVAL, "NULL argument");
    pbvd_code c = *code;
    c.mapping = PBVD_MAP_GROUP;
    c.lanes_per_pb = 0;
    int idx = -1;
    const pbvd_status st = check_code(c, &idx);
    if (st != PBVD_OK) return st;
    pbvd::group::GroupArgs t{};
    if (!group_tables(c, &t)) return fail(PBVD_ENOTSUP, "no group table for this code");
    const int HALF = 1 << (c.K - 2), NC = 1 << c.R, B = HALF / NC;
    // table bit r (byte r of a mask) is c^(r+1); the export puts c^(1) first
    auto word = [&](uint32_t m) {
        int32_t v = 0;
        for (int r = 0; r < c.R; ++r) v |= (int32_t)((m >> (8 * r)) & 1u) << (c.R - 1 - r);
        return v;
    };
    for (int w = 0; w < NC; ++w) {
        for (int b = 0; b < B; ++b) alpha[t.jtab[w * B + b]] = word(t.bm_mask[w][0]);
        for (int k = 0; k < 4; ++k) masks[4 * word(t.bm_mask[w][0]) + k] = word(t.bm_mask[w][k]);
    }
    return PBVD_OK;
}

pbvd_status pbvd_debug_branch_metrics(pbvd_plan *p, const void *d_syms, int64_t n_stages,
                                      int32_t *d_bm, void *hip_stream) {
    g_last_error[0] = 0;
    if (!p) return fail(PBVD_EINVAL, "plan is NULL");
    if (n_stages < 0) return fail(PBVD_EINVAL, "n_stages must be >= 0");
    if (n_stages > 0 && (!d_syms || !d_bm)) return fail(PBVD_EINVAL, "NULL buffer");
    if (n_stages == 0) return PBVD_OK;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(PBVD_EHIP, "cannot select device %d", p->device);
    hipError_t e = pbvd::branch_metrics(p->code.R, p->code.input_kind, (const uint8_t *)d_syms,
                                        n_stages, d_bm, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail_hip(e, "branch-metric launch");
    return PBVD_OK;
}

pbvd_status pbvd_decode_host(pbvd_plan *p, const void *h_syms, int64_t n_bits, uint8_t *h_out,
                             int32_t n_streams, int64_t chunk_pbs, uint32_t flags) {
    g_last_error[0] = 0;
    if (!p) return fail(PBVD_EINVAL, "plan is NULL");
    if (!h_syms || !h_out) return fail(PBVD_EINVAL, "NULL host buffer");
    if (n_bits < 1) return fail(PBVD_EINVAL, "n_bits must be >= 1 (got %lld)", (long long)n_bits);
    if (n_streams < 1 || n_streams > kMaxPipeStreams)
        return fail(PBVD_EINVAL, "n_streams must be in [1, %d]", kMaxPipeStreams);
    if (flags & ~(uint32_t)PBVD_HOST_PINNED) return fail(PBVD_EINVAL, "unknown flags 0x%x", flags);
    const pbvd_code &c = p->code;
    const int64_t D = c.D, L = c.L, R = c.R;
    const int64_t nb = ceil_div(n_bits, D);
    const int64_t T = n_bits + (c.terminated ? c.K - 1 : 0);
    // chunks start on byte boundaries of the output
    int64_t g = D, e8 = 8;
    while (e8) { const int64_t t = g % e8; g = e8; e8 = t; }
    const int64_t unit = 8 / g;
    if (chunk_pbs < 0) return fail(PBVD_EINVAL, "chunk_pbs must be >= 0");
    if (chunk_pbs == 0) chunk_pbs = ceil_div(ceil_div(nb, 2 * (int64_t)n_streams), unit) * unit;
    if (chunk_pbs % unit != 0)
        return fail(PBVD_EINVAL, "chunk_pbs * D must be a multiple of 8 (chunk_pbs %% %lld != 0)", (long long)unit);
    if (chunk_pbs > nb) chunk_pbs = ceil_div(nb, unit) * unit;
    const bool pinned = (flags & PBVD_HOST_PINNED) != 0;
    const int64_t n_chunks = ceil_div(nb, chunk_pbs);
    const int used = (int)std::min<int64_t>(n_streams, n_chunks);
    // the kernels read up to a dword before a PB's first symbol and up to
    // one trip's window past its last one: pad the chunk buffer on both sides
    constexpr int64_t kPad = 256;
    const int64_t in_max = (chunk_pbs * D + 2 * L) * R + 2 * kPad;
    const int64_t out_max = ceil_div(chunk_pbs * D, 8) + 8;
    if (fault_injected("launch")) return fail(PBVD_EHIP, "injected launch failure");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(PBVD_EHIP, "cannot select device %d", p->device);
    for (int si = 0; si < used; ++si) {
        PipeStream &ps = p->pipe[si];
        hipError_t e = hipSuccess;
        if (!ps.stream) e = hipStreamCreateWithFlags(&ps.stream, hipStreamNonBlocking);
        if (e == hipSuccess && !ps.done) e = hipEventCreateWithFlags(&ps.done, hipEventDisableTiming);
        if (e != hipSuccess) return fail_hip(e, "pipeline stream creation");
        pbvd_status st = ensure_buffer(reinterpret_cast<uint32_t **>(&ps.d_in), &ps.d_in_bytes, (size_t)in_max, "chunk input");
        if (st == PBVD_OK)
            st = ensure_buffer(reinterpret_cast<uint32_t **>(&ps.d_out), &ps.d_out_bytes, (size_t)out_max, "chunk output");
        if (st != PBVD_OK) return st;
        if (!pinned) {
            if (ps.h_in_bytes < (size_t)in_max) {
                if (ps.h_in) (void)hipHostFree(ps.h_in);
                ps.h_in = nullptr;
                ps.h_in_bytes = 0;
                e = hipHostMalloc((void **)&ps.h_in, (size_t)in_max, hipHostMallocDefault);
                if (e != hipSuccess) return fail_hip(e, "pinned staging");
                ps.h_in_bytes = (size_t)in_max;
            }
            if (ps.h_out_bytes < (size_t)out_max) {
                if (ps.h_out) (void)hipHostFree(ps.h_out);
                ps.h_out = nullptr;
                ps.h_out_bytes = 0;
                e = hipHostMalloc((void **)&ps.h_out, (size_t)out_max, hipHostMallocDefault);
                if (e != hipSuccess) return fail_hip(e, "pinned staging");
                ps.h_out_bytes = (size_t)out_max;
            }
        }
        ps.pend_byte = -1;
    }
    const uint8_t *hs = (const uint8_t *)h_syms;
    bool busy[kMaxPipeStreams] = {};
    pbvd_status result = PBVD_OK;
    for (int64_t ch = 0; ch < n_chunks && result == PBVD_OK; ++ch) {
        PipeStream &ps = p->pipe[ch % used];
        const int64_t pb0 = ch * chunk_pbs;
        const int64_t pbn = std::min(chunk_pbs, nb - pb0);
        const int64_t f0 = std::max<int64_t>(0, pb0 * D - L);
        const int64_t f1 = std::min(T, (pb0 + pbn) * D + L);
        const int64_t in_bytes = (f1 - f0) * R;
        const int64_t out_bits = std::min(n_bits, (pb0 + pbn) * D) - pb0 * D;
        const int64_t out_bytes = ceil_div(out_bits, 8);
        const int64_t byte0 = pb0 * D / 8;
        const uint8_t *src = hs + f0 * R;
        if (!pinned) {
            // reuse this stream's staging: its previous chunk must be done
            if (busy[ch % used]) {
                hipError_t e = hipEventSynchronize(ps.done);
                if (e != hipSuccess) return fail_hip(e, "pipeline wait");
                if (ps.pend_byte >= 0) memcpy(h_out + ps.pend_byte, ps.h_out, (size_t)ps.pend_bytes);
                ps.pend_byte = -1;
            }
            memcpy(ps.h_in, src, (size_t)in_bytes);
            src = ps.h_in;
        }
        hipError_t e = hipMemcpyAsync(ps.d_in + kPad, src, (size_t)in_bytes, hipMemcpyHostToDevice, ps.stream);
        if (e != hipSuccess) return fail_hip(e, "chunk upload");
        // stage 0 of the stream at a virtual address: the chunk's stages [f0, f1) land in d_in
        const uint8_t *base = ps.d_in + kPad - f0 * R;
        result = run_decode(p, ps.ws, base, n_bits, pb0, pbn, ps.d_out, nullptr, ps.stream, nullptr, false);
        if (result != PBVD_OK) break;
        uint8_t *dst = pinned ? h_out + byte0 : ps.h_out;
        e = hipMemcpyAsync(dst, ps.d_out, (size_t)out_bytes, hipMemcpyDeviceToHost, ps.stream);
        if (e == hipSuccess) e = hipEventRecord(ps.done, ps.stream);
        if (e != hipSuccess) return fail_hip(e, "chunk read-back");
        busy[ch % used] = true;
        if (!pinned) {
            ps.pend_byte = byte0;
            ps.pend_bytes = out_bytes;
        }
    }
    for (int si = 0; si < used; ++si) {
        PipeStream &ps = p->pipe[si];
        if (!busy[si]) continue;
        hipError_t e = hipEventSynchronize(ps.done);
        if (e != hipSuccess && result == PBVD_OK) result = fail_hip(e, "pipeline wait");
        if (result == PBVD_OK && !pinned && ps.pend_byte >= 0)
            memcpy(h_out + ps.pend_byte, ps.h_out, (size_t)ps.pend_bytes);
        ps.pend_byte = -1;
    }
    return result;
}

void pbvd_destroy(pbvd_plan *p) {
    if (!p) return;
    {
        DeviceGuard dg(p->device);
        bool any = p->ws.sp || p->ws.words;
        for (const PipeStream &ps : p->pipe) any = any || ps.stream;
        if (any) (void)hipDeviceSynchronize();
        free_workspace(p->ws);
        for (PipeStream &ps : p->pipe) {
            free_workspace(ps.ws);
            if (ps.d_in) (void)hipFree(ps.d_in);
            if (ps.d_out) (void)hipFree(ps.d_out);
            if (ps.h_in) (void)hipHostFree(ps.h_in);
            if (ps.h_out) (void)hipHostFree(ps.h_out);
            if (ps.done) (void)hipEventDestroy(ps.done);
            if (ps.stream) (void)hipStreamDestroy(ps.stream);
        }
    }
    delete p;
}

const char *pbvd_strerror(pbvd_status s) {
    switch (s) {
    case PBVD_OK: return "success";
    case PBVD_EINVAL: return "invalid argument";
    case PBVD_ENOTSUP: return "not supported";
    case PBVD_ENOMEM: return "out of device memory";
    case PBVD_EHIP: return "HIP runtime error";
    case PBVD_EAGAIN: return "not ready / queue full";
    }
    return "unknown status";
}

const char *pbvd_last_error(void) { return g_last_error; }

}  // extern "C"
