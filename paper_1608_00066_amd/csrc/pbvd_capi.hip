// C ABI of the decoder (declared in include/pbvd.h): argument validation,
// plan and workspace management, the block decomposition of a call into
// kernel launches, and error reporting.  No C++ exception leaves this file.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "pbvd.h"
#include "pbvd_aux.hpp"
#include "pbvd_registry.hpp"

#define PBVD_ROW(i, K, R, g0, g1, g2, g3) {K, R, {g0, g1, g2, g3}},
const RegisteredCode kRegisteredCodes[kNumCodes] = {PBVD_CODE_LIST(PBVD_ROW)};
#undef PBVD_ROW

namespace {

using LaunchFn = hipError_t (*)(const pbvd::LaunchRequest &);
#define PBVD_FN(i, K, R, g0, g1, g2, g3) &pbvd::launch_code<i>,
const LaunchFn kLaunchTable[kNumCodes] = {PBVD_CODE_LIST(PBVD_FN)};
#undef PBVD_FN
using TileLaunchFn = hipError_t (*)(const pbvd::TileLaunchRequest &);
#define PBVD_TFN(i, K, R, g0, g1, g2, g3) &pbvd::launch_tiles<i>,
const TileLaunchFn kTileLaunchTable[kNumCodes] = {PBVD_CODE_LIST(PBVD_TFN)};
#undef PBVD_TFN

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

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Block decomposition of one call (Sec. III-A with M = L): PBs with the full
// forward range [bD-L, bD+D+L) and decoded range [bD, bD+D) are "interior"
// and go 64 to a wave; the others (stream ends) get a wave each.
struct CallGeometry {
    int64_t T, pb_first, pb_end;
    int64_t b_lo, b_hi, n_head, n_tail;
    int64_t n_int_waves, n_waves;
    int64_t out_bits;
};

CallGeometry call_geometry(const pbvd_code &c, int64_t n, int64_t pb_first, int64_t pb_count) {
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
        g.n_int_waves = ceil_div(hi - lo, pbvd::kWave);
    } else {
        g.b_lo = g.b_hi = g.pb_end;
        g.n_head = pb_count;
        g.n_tail = 0;
        g.n_int_waves = 0;
    }
    g.n_waves = g.n_int_waves + g.n_head + g.n_tail;
    const int64_t end_bit = g.pb_end * D < n ? g.pb_end * D : n;
    g.out_bits = pb_count > 0 ? end_bit - pb_first * D : 0;
    return g;
}

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

bool fault_injected(const char *site) {
    const char *f = getenv("PBVD_FAULT_INJECT");
    return f && strcmp(f, site) == 0;
}

}  // namespace

struct pbvd_plan {
    pbvd_code code;
    int code_idx;
    int device;
    int ndw;                  // survivor dwords per stored row
    int row_stages;           // stages per stored row
    int64_t sp_wave_dwords;   // survivor dwords per wave slot
    int64_t budget_bytes;     // survivor workspace limit
    uint32_t *sp;
    size_t sp_bytes;
    uint32_t *words;
    size_t words_bytes;
};

namespace {

// Makes the plan's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) {
            ok = false;
            return;
        }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

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

int64_t waves_per_launch(const pbvd_plan *p) {
    int64_t w = p->budget_bytes / (p->sp_wave_dwords * 4);
    return w < 1 ? 1 : w;
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

// Runs the decode kernels of one call; fills *geo with the decomposition.
pbvd_status run_decode(pbvd_plan *p, const void *d_syms, int64_t n_bits, int64_t pb_first,
                       int64_t pb_count, uint8_t *d_out, int32_t *d_final_pm, hipStream_t stream,
                       CallGeometry *geo_out, bool single_launch) {
    const pbvd_code &c = p->code;
    const CallGeometry g = call_geometry(c, n_bits, pb_first, pb_count);
    if (geo_out) *geo_out = g;
    if (pb_count == 0) return PBVD_OK;
    const int64_t per_launch = waves_per_launch(p);
    if (single_launch && g.n_waves > per_launch)
        return fail(PBVD_EINVAL, "%lld waves do not fit one launch (limit %lld)",
                    (long long)g.n_waves, (long long)per_launch);
    if (fault_injected("launch")) return fail(PBVD_EHIP, "injected launch failure");

    const int64_t launch_waves = g.n_waves < per_launch ? g.n_waves : per_launch;
    pbvd_status st = ensure_buffer(&p->sp, &p->sp_bytes,
                                   (size_t)(launch_waves * p->sp_wave_dwords * 4), "survivors");
    if (st != PBVD_OK) return st;

    const int64_t out_bytes = ceil_div(g.out_bits, 8);
    const bool direct = (c.D % 32 == 0) && (((uintptr_t)d_out & 3u) == 0);
    if (!direct) {
        const int64_t nwords = ceil_div(g.out_bits, 32) + 2;
        st = ensure_buffer(&p->words, &p->words_bytes, (size_t)nwords * 4, "output staging");
        if (st != PBVD_OK) return st;
        hipError_t e = pbvd::fill_u32(p->words, nwords, 0u, stream);
        if (e != hipSuccess) return fail_hip(e, "zero-fill launch");
    }

    pbvd::LaunchRequest req{};
    pbvd::KernelArgs &a = req.args;
    a.syms = (const uint8_t *)d_syms;
    a.out = d_out;
    a.out_words = direct ? nullptr : p->words;
    a.final_pm = d_final_pm;
    a.sp = p->sp;
    a.n = n_bits;
    a.T = g.T;
    a.pb_first = pb_first;
    a.b_lo = g.b_lo;
    a.b_hi = g.b_hi;
    a.n_head = g.n_head;
    a.n_int_waves = g.n_int_waves;
    a.out_bytes = out_bytes;
    a.sp_wave_dwords = p->sp_wave_dwords;
    a.D = c.D;
    a.L = c.L;
    a.terminated = c.terminated;
    a.direct_out = direct ? 1 : 0;
    req.pm_bits = c.pm_bits;
    req.input_kind = c.input_kind;
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
        hipError_t e = pbvd::words_to_bytes(p->words, d_out, out_bytes, stream);
        if (e != hipSuccess) return fail_hip(e, "output copy launch");
    }
    return PBVD_OK;
}

// Survivor dwords of one wave slot: every forward stage of a PB (at most
// D + 2L) is stored, one row per stage (or per few stages for small trellises).
int64_t slot_dwords(const pbvd_code &c) {
    const int64_t rows = ceil_div((int64_t)c.D + 2 * (int64_t)c.L, pbvd::survivor_row_stages(c.K)) + 1;
    return ceil_div(rows * pbvd::kWave * pbvd::survivor_row_dwords(c.K), 64) * 64;
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
    if (c.pm_bits == 32 && c.K > 8) return fail(PBVD_ENOTSUP, "32-bit path metrics need K <= 8");
    {
        // survivor rows of one wave slot are addressed with 32-bit offsets
        const int64_t row_bytes = 64LL * pbvd::survivor_row_dwords(c.K) * 4;
        const int64_t slot =
            (((int64_t)c.D + 2 * (int64_t)c.L) / pbvd::survivor_row_stages(c.K) + 2) * row_bytes;
        if (slot >= (1LL << 31) - 4096)
            return fail(PBVD_ENOTSUP, "D + 2L too large for the survivor buffer of one wave (%lld bytes)",
                        (long long)slot);
    }
    const int idx = find_code(c);
    if (idx < 0) return fail(PBVD_ENOTSUP, "no kernel compiled for this generator set");
    *idx_out = idx;
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
    if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
    (void)hipGetLastError();
    p->ndw = pbvd::survivor_row_dwords(c.K);
    p->row_stages = pbvd::survivor_row_stages(c.K);
    p->sp_wave_dwords = slot_dwords(c);
    p->budget_bytes = workspace_budget_bytes();
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
    return run_decode(p, d_syms, n_bits, pb_first, pb_count, d_out_bits, d_final_pm,
                      (hipStream_t)hip_stream, nullptr, false);
}

pbvd_status pbvd_decode(pbvd_plan *p, const void *d_syms, int64_t n_bits, uint8_t *d_out_bits,
                        void *hip_stream) {
    if (!p) return fail(PBVD_EINVAL, "plan is NULL");
    if (n_bits < 1) return fail(PBVD_EINVAL, "n_bits must be >= 1 (got %lld)", (long long)n_bits);
    return pbvd_decode_ex(p, d_syms, n_bits, 0, ceil_div(n_bits, p->code.D), d_out_bits, nullptr,
                          hip_stream);
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
    st = run_decode(p, d_syms, n_bits, pb_first, pb_count, d_out_bits, nullptr, s, &g, true);
    if (st != PBVD_OK || pb_count == 0) return st;
    pbvd::SurvivorView v{};
    v.sp = p->sp;
    v.sp_wave_dwords = p->sp_wave_dwords;
    v.T = g.T;
    v.pb_first = pb_first;
    v.pb_count = pb_count;
    v.b_lo = g.b_lo;
    v.b_hi = g.b_hi;
    v.n_head = g.n_head;
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

void pbvd_destroy(pbvd_plan *p) {
    if (!p) return;
    {
        DeviceGuard dg(p->device);
        if (p->sp || p->words) (void)hipDeviceSynchronize();
        if (p->sp) (void)hipFree(p->sp);
        if (p->words) (void)hipFree(p->words);
    }
    delete p;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched decoding
// ---------------------------------------------------------------------------
#include <algorithm>
#include <vector>

namespace {

constexpr int kMaxBatchCodes = 16;

struct BatchGroup {
    int64_t tile_begin = 0, n_tiles = 0;
    int64_t sp_wave_dwords = 0;
};

}  // namespace

struct pbvd_batch {
    int n_codes = 0;
    pbvd_code codes[kMaxBatchCodes];
    int code_idx[kMaxBatchCodes];
    int device = 0;
    BatchGroup groups[kMaxBatchCodes];
    int64_t n_tiles = 0, n_blocks = 0, n_stages = 0;
    int64_t sym_bytes = 0, out_bytes = 0;
    int64_t waves_per_launch = 1;
    pbvd::LaneDesc *d_lanes = nullptr;
    pbvd::TileHead *d_heads = nullptr;
    size_t lanes_bytes = 0, heads_bytes = 0;
    uint32_t *sp = nullptr;
    size_t sp_bytes = 0;
};

namespace {

struct PbRec {
    int64_t sym, out_bit;
    int32_t len, store0, dec_end, flags;
};

pbvd_status build_tiles(pbvd_batch *b, const pbvd_frame *frames, int64_t n_frames,
                        std::vector<pbvd::LaneDesc> &lanes, std::vector<pbvd::TileHead> &heads,
                        BatchGroup *groups, int64_t *n_blocks, int64_t *n_stages) {
    std::vector<std::vector<PbRec>> per_code(b->n_codes);
    std::vector<std::pair<int64_t, int64_t>> outs;
    outs.reserve((size_t)n_frames);
    *n_blocks = 0;
    *n_stages = 0;
    for (int64_t f = 0; f < n_frames; ++f) {
        const pbvd_frame &fr = frames[f];
        if (fr.code < 0 || fr.code >= b->n_codes || fr.reserved != 0)
            return fail(PBVD_EINVAL, "frame %lld: bad code index %d", (long long)f, fr.code);
        const pbvd_code &c = b->codes[fr.code];
        if (fr.n_bits < 1) return fail(PBVD_EINVAL, "frame %lld: n_bits must be >= 1", (long long)f);
        const int64_t T = fr.n_bits + (c.terminated ? c.K - 1 : 0);
        if (fr.sym_offset < 0 || fr.sym_offset > b->sym_bytes - T * c.R)
            return fail(PBVD_EINVAL, "frame %lld: symbols outside the %lld-byte input", (long long)f,
                        (long long)b->sym_bytes);
        const int64_t nbytes = ceil_div(fr.n_bits, 8);
        if (fr.out_offset < 0 || fr.out_offset > b->out_bytes - nbytes)
            return fail(PBVD_EINVAL, "frame %lld: output outside the %lld-byte buffer", (long long)f,
                        (long long)b->out_bytes);
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
            *n_stages += r.len;
        }
        *n_blocks += nb;
    }
    std::sort(outs.begin(), outs.end());
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].first < outs[i - 1].second)
            return fail(PBVD_EINVAL, "frame output ranges overlap at byte %lld", (long long)outs[i].first);

    lanes.clear();
    heads.clear();
    for (int ci = 0; ci < b->n_codes; ++ci) {
        const pbvd_code &c = b->codes[ci];
        const int64_t U = pbvd::trip_stages(c.K);
        const int64_t ND = pbvd::trip_fetch_dwords(c.K, c.R);
        std::vector<PbRec> &v = per_code[ci];
        // longest first (load balance); PBs that start their traceback from
        // the best state must share a tile with PBs of the same length only,
        // so that all of a tile's final metrics are taken at one stage
        std::stable_sort(v.begin(), v.end(), [](const PbRec &x, const PbRec &y) {
            const bool ax = x.flags & pbvd::kLaneArgmin, ay = y.flags & pbvd::kLaneArgmin;
            if (ax != ay) return ax < ay;
            return x.len > y.len;
        });
        groups[ci].tile_begin = (int64_t)heads.size();
        size_t i = 0;
        while (i < v.size()) {
            size_t e = std::min(v.size(), i + (size_t)pbvd::kWave);
            if (v[i].flags & pbvd::kLaneArgmin) {
                size_t k = i + 1;
                while (k < e && (v[k].flags & pbvd::kLaneArgmin) && v[k].len == v[i].len) ++k;
                e = k;
            } else {
                size_t k = i + 1;
                while (k < e && !(v[k].flags & pbvd::kLaneArgmin)) ++k;
                e = k;
            }
            pbvd::TileHead h{};
            h.len = 0;
            h.store0_min = 0x7fffffff;
            bool wide = true, final_needed = false;
            for (size_t k = i; k < i + pbvd::kWave; ++k) {
                const PbRec &r = v[k < e ? k : i];
                pbvd::LaneDesc d;
                d.sym = r.sym;
                d.out_bit = r.out_bit;
                d.len = r.len;
                d.store0 = r.store0;
                d.dec_end = r.dec_end;
                d.flags = k < e ? r.flags : (r.flags & ~pbvd::kLaneActive);
                lanes.push_back(d);
                if (r.len > h.len) h.len = r.len;
                if (r.store0 < h.store0_min) h.store0_min = r.store0;
                const int64_t last_trip = ((r.len - 1) / U) * U;
                if (r.sym + last_trip * c.R + 4 * ND > b->sym_bytes) wide = false;
                if (r.flags & pbvd::kLaneArgmin) final_needed = true;
            }
            h.flags = (wide ? pbvd::kTileWide : 0) | (final_needed ? pbvd::kTileFinal : 0);
            heads.push_back(h);
            i = e;
        }
        groups[ci].n_tiles = (int64_t)heads.size() - groups[ci].tile_begin;
        groups[ci].sp_wave_dwords = slot_dwords(c);
    }
    return PBVD_OK;
}

}  // namespace

extern "C" {

pbvd_status pbvd_batch_create(const pbvd_code *codes, int32_t n_codes, pbvd_batch **out) {
    g_last_error[0] = 0;
    if (!codes || !out) return fail(PBVD_EINVAL, "codes and out must not be NULL");
    if (n_codes < 1 || n_codes > kMaxBatchCodes)
        return fail(PBVD_EINVAL, "n_codes must be in [1, %d]", kMaxBatchCodes);
    pbvd_batch *b = new (std::nothrow) pbvd_batch();
    if (!b) return fail(PBVD_ENOMEM, "host allocation failed");
    for (int i = 0; i < n_codes; ++i) {
        int idx = -1;
        pbvd_status st = check_code(codes[i], &idx);
        if (st == PBVD_OK && codes[i].D % 8 != 0)
            st = fail(PBVD_EINVAL, "code %d: batched decoding needs D %% 8 == 0 (got %d)", i, codes[i].D);
        if (st != PBVD_OK) {
            delete b;
            return st;
        }
        b->codes[i] = codes[i];
        for (int r = codes[i].R; r < 4; ++r) b->codes[i].gen[r] = 0;
        b->code_idx[i] = idx;
    }
    b->n_codes = n_codes;
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
    const int64_t keep_sym = b->sym_bytes, keep_out = b->out_bytes;
    b->sym_bytes = sym_bytes;
    b->out_bytes = out_bytes;
    std::vector<pbvd::LaneDesc> lanes;
    std::vector<pbvd::TileHead> heads;
    BatchGroup groups[kMaxBatchCodes];
    int64_t n_blocks = 0, n_stages = 0;
    pbvd_status st;
    try {
        st = build_tiles(b, frames, n_frames, lanes, heads, groups, &n_blocks, &n_stages);
    } catch (...) {
        st = fail(PBVD_ENOMEM, "host allocation failed while building the work list");
    }
    if (st != PBVD_OK) {
        b->sym_bytes = keep_sym;
        b->out_bytes = keep_out;
        return st;
    }
    DeviceGuard dg(b->device);
    if (!dg.ok) return fail(PBVD_EHIP, "cannot select device %d", b->device);
    // survivor workspace: every group's tiles in one launch when the budget
    // allows, else the largest launch the budget allows
    const int64_t budget = workspace_budget_bytes();
    int64_t max_slot = 64;
    for (int ci = 0; ci < b->n_codes; ++ci) max_slot = std::max(max_slot, groups[ci].sp_wave_dwords);
    int64_t max_tiles = 0;
    for (int ci = 0; ci < b->n_codes; ++ci) max_tiles = std::max(max_tiles, groups[ci].n_tiles);
    int64_t per_launch = std::max<int64_t>(1, budget / (max_slot * 4));
    if (per_launch > max_tiles) per_launch = std::max<int64_t>(1, max_tiles);
    st = ensure_buffer(&b->sp, &b->sp_bytes, (size_t)(per_launch * max_slot * 4), "survivors");
    if (st != PBVD_OK) return st;
    const size_t lb = std::max<size_t>(lanes.size(), 1) * sizeof(pbvd::LaneDesc);
    const size_t hb = std::max<size_t>(heads.size(), 1) * sizeof(pbvd::TileHead);
    st = ensure_buffer(reinterpret_cast<uint32_t **>(&b->d_lanes), &b->lanes_bytes, lb, "work list");
    if (st != PBVD_OK) return st;
    st = ensure_buffer(reinterpret_cast<uint32_t **>(&b->d_heads), &b->heads_bytes, hb, "work list");
    if (st != PBVD_OK) return st;
    if (!lanes.empty()) {
        hipError_t e = hipMemcpy(b->d_lanes, lanes.data(), lanes.size() * sizeof(pbvd::LaneDesc),
                                 hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_heads, heads.data(), heads.size() * sizeof(pbvd::TileHead),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail_hip(e, "work-list upload");
    }
    for (int ci = 0; ci < b->n_codes; ++ci) b->groups[ci] = groups[ci];
    b->n_tiles = (int64_t)heads.size();
    b->n_blocks = n_blocks;
    b->n_stages = n_stages;
    b->waves_per_launch = per_launch;
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
    const int waves_per_block = pbvd::kBlockThreads / pbvd::kWave;
    for (int ci = 0; ci < b->n_codes; ++ci) {
        const BatchGroup &g = b->groups[ci];
        for (int64_t t0 = 0; t0 < g.n_tiles; t0 += b->waves_per_launch) {
            pbvd::TileLaunchRequest req{};
            pbvd::TileArgs &a = req.args;
            a.syms = (const uint8_t *)d_syms;
            a.sym_bytes = b->sym_bytes;
            a.out = d_out;
            a.lanes = b->d_lanes;
            a.heads = b->d_heads;
            a.sp = b->sp;
            a.sp_wave_dwords = g.sp_wave_dwords;
            a.tile_begin = g.tile_begin + t0;
            a.n_tiles = std::min(b->waves_per_launch, g.n_tiles - t0);
            req.pm_bits = b->codes[ci].pm_bits;
            req.input_kind = b->codes[ci].input_kind;
            req.grid = (unsigned)ceil_div(a.n_tiles, waves_per_block);
            req.stream = (hipStream_t)hip_stream;
            hipError_t e = kTileLaunchTable[b->code_idx[ci]](req);
            if (e != hipSuccess) return fail_hip(e, "batch kernel launch");
        }
    }
    return PBVD_OK;
}

pbvd_status pbvd_batch_info(const pbvd_batch *b, int64_t *n_tiles, int64_t *n_blocks,
                            int64_t *n_forward_stages, int64_t *workspace_bytes) {
    if (!b) return fail(PBVD_EINVAL, "batch is NULL");
    if (n_tiles) *n_tiles = b->n_tiles;
    if (n_blocks) *n_blocks = b->n_blocks;
    if (n_forward_stages) *n_forward_stages = b->n_stages;
    if (workspace_bytes) *workspace_bytes = (int64_t)(b->sp_bytes + b->lanes_bytes + b->heads_bytes);
    return PBVD_OK;
}

void pbvd_batch_destroy(pbvd_batch *b) {
    if (!b) return;
    {
        DeviceGuard dg(b->device);
        if (b->sp || b->d_lanes || b->d_heads) (void)hipDeviceSynchronize();
        if (b->sp) (void)hipFree(b->sp);
        if (b->d_lanes) (void)hipFree(b->d_lanes);
        if (b->d_heads) (void)hipFree(b->d_heads);
    }
    delete b;
}

const char *pbvd_strerror(pbvd_status s) {
    switch (s) {
    case PBVD_OK: return "success";
    case PBVD_EINVAL: return "invalid argument";
    case PBVD_ENOTSUP: return "not supported";
    case PBVD_ENOMEM: return "out of device memory";
    case PBVD_EHIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *pbvd_last_error(void) { return g_last_error; }

}  // extern "C"
