// Host-side pieces shared by the C ABI units (single-stream plans, batches,
// the request server): error reporting, code validation, device buffers and
// the work-list builder of batched decoding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pbvd.h"
#include "pbvd_registry.hpp"

namespace pbvd_host {

// Detail of the last failure of the calling thread (pbvd_last_error).
extern thread_local char g_last_error[512];

pbvd_status fail(pbvd_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
pbvd_status fail_hip(hipError_t e, const char *what);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// PBVD_FAULT_INJECT=<site> makes the named host step fail (error-path tests).
bool fault_injected(const char *site);

// Makes a device current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

// Grows a device buffer to at least `need` bytes (contents are not kept).
pbvd_status ensure_buffer(uint32_t **buf, size_t *have, size_t need, const char *what);

// log2 of the lanes per PB of the state-parallel kernel (a whole wave).
constexpr int kWaveLb = 6;
// Marks the group mapping (2^R lanes per PB, one wave per butterfly group)
// where a lane-group width is expected.
constexpr int kGroupLb = 7;

// The group mapping's tables of a code (Sec. III-B): branch-metric masks,
// the butterflies of each group and the traceback positions; false when the
// code's groups are not all of one size (alpha map below full rank) or the
// shape is outside the mapping.
bool group_tables(const pbvd_code &c, pbvd::group::GroupArgs *a);

// Survivor dwords of one tile (64 PBs of at most D + 2L stages) of the
// group mapping.
int64_t group_tile_dwords(const pbvd_code &c);

// Launches the group-mapped kernel of constraint length K.
hipError_t launch_group_kernel(int K, const pbvd::GroupLaunchRequest &req);

// Validates a code/block parameter set; *idx_out receives its registry index
// (-1: no register kernel; the wave mapping decodes it).
pbvd_status check_code(const pbvd_code &c, int *idx_out);

// Survivor dwords of one wave slot of the state-parallel kernel (one PB of
// at most D + 2L forward stages).
int64_t wave_slot_dwords(const pbvd_code &c);

// Run-time code description of the state-parallel kernel.
pbvd::wave::WaveCode wave_code(const pbvd_code &c);

// Launches the state-parallel kernel of constraint length K.
hipError_t launch_wave(int K, const pbvd::WaveLaunchRequest &req);

// Survivor dwords of one wave slot of a code (all D + 2L forward rows) with
// 2^lb lanes per PB.
int64_t slot_dwords(const pbvd_code &c, int lb);

// log2 of the lanes per PB a code asks for (kWaveLb for the wave mapping,
// -1: the library chooses).
int requested_lb(const pbvd_code &c);
// The largest lane group a code supports.
int max_lb(const pbvd_code &c);

// Survivor workspace limit of one plan or batch (PBVD_WORKSPACE_MB, default 8 GiB).
int64_t workspace_budget_bytes();

// Launches the tile kernel of registry entry code_idx.
hipError_t launch_tiles(int code_idx, const pbvd::TileLaunchRequest &req);
// Registered pair of the registry codes idx_a and idx_b (either order), -1 if
// none; *a_first tells whether idx_a is the pair's first code.
int find_pair(int idx_a, int idx_b, bool *a_first);
hipError_t launch_tiles_pair(int pair_idx, const pbvd::TileLaunchRequest &req);

// ---- batched decoding work list --------------------------------------------

constexpr int kMaxCodes = 16;

struct CodeSet {
    int n = 0;
    pbvd_code codes[kMaxCodes];
    int idx[kMaxCodes];
    int lb[kMaxCodes];   // lanes per PB used for each code (log2; kWaveLb, kGroupLb)
    pbvd::group::GroupArgs gtab[kMaxCodes];  // tables of the group-mapped codes
};

// Validates n codes for batched use (D % 8 == 0) into *out.  Codes that let
// the library choose their lanes per PB get auto_lb (clipped to what the
// code supports; -1: the largest it supports; kWaveLb: the wave mapping);
// codes without a register kernel, or that ask for the wave mapping, get
// kWaveLb.
pbvd_status make_code_set(const pbvd_code *codes, int32_t n, CodeSet *out, int auto_lb = 0);

// The work of one code: tiles of the register kernel (waves of 64 >> lb
// PBs; tile_begin indexes the heads, 64 lane descriptors per tile), or, with
// lb == kWaveLb, PBs of the state-parallel kernel (one wave each;
// tile_begin indexes the PB descriptors), or, with lb == kGroupLb, tiles of
// 64 PBs of the group-mapped kernel (tile_begin indexes the PB descriptors,
// 64 per tile; sp_wave_dwords is per tile).
struct TileGroup {
    int64_t tile_begin = 0, n_tiles = 0;
    int64_t sp_wave_dwords = 0;
    int lb = 0;
    // register codes of a registered pair: the group of the first code of
    // the two in the code set holds both codes' tiles (pair launch), the
    // other's is empty
    int pair = -1;
};

// The PBs of every state-parallel code of one constraint length, for one
// persistent launch: descriptors [desc_begin, + n_descs), longest first,
// each naming its code by its slot in `codes` (flag bits from
// pbvd::wave::kDescCodeShift).
struct FusedGroup {
    int n_codes = 0;
    int codes[kMaxCodes];           // code set index of each slot
    int64_t desc_begin = 0, n_descs = 0;
    int64_t sp_wave_dwords = 0;     // the largest slot of its codes
};
constexpr int kMinK = 3, kMaxK = 9;

// Tiles (waves of 64 PBs) of a set of frames, grouped by code.
struct WorkList {
    std::vector<pbvd::LaneDesc> lanes;   // 64 per tile (register kernel)
    std::vector<pbvd::TileHead> heads;   // one per tile (register kernel)
    std::vector<pbvd::LaneDesc> descs;   // one per PB (state-parallel kernel)
    TileGroup groups[kMaxCodes];
    FusedGroup fused[kMaxK - kMinK + 1];  // by K (fuse_waves only)
    int64_t n_blocks = 0, n_stages = 0;
};

// Builds the work list of `frames` (validated against the buffer sizes).
// fuse_waves: the state-parallel codes of one K share one fused group (and
// their own groups stay empty); else each code has its own group.
// pair_tiles: register codes that form a registered pair (same lanes per PB,
// 16-bit metrics, same input kind) share one group, launched as one.
pbvd_status build_work_list(const CodeSet &cs, const pbvd_frame *frames, int64_t n_frames,
                            int64_t sym_bytes, int64_t out_bytes, WorkList *wl, bool fuse_waves = false,
                            bool pair_tiles = false);

// Launches the tile kernels of one code group: tiles [g.tile_begin, + g.n_tiles)
// of the uploaded work list, at most `per_launch` waves per launch sharing
// the survivor area `sp` one launch after another.
pbvd_status launch_group(const CodeSet &cs, int ci, const TileGroup &g, const uint8_t *d_syms,
                         int64_t sym_bytes, uint8_t *d_out, const pbvd::LaneDesc *d_lanes,
                         const pbvd::TileHead *d_heads, const pbvd::LaneDesc *d_descs, uint32_t *sp,
                         int64_t per_launch, hipStream_t stream);

// Launches one persistent state-parallel kernel over fused group g: `waves`
// waves (survivor area sp, g.sp_wave_dwords each) take its PBs from the
// work counters at `counter` (pbvd::wave::kCounters of them), which a fill
// kernel on `stream` zeroes first.
pbvd_status launch_fused(const CodeSet &cs, int K, const FusedGroup &g, const uint8_t *d_syms,
                         int64_t sym_bytes, uint8_t *d_out, const pbvd::LaneDesc *d_descs, uint32_t *sp,
                         int64_t waves, uint32_t *counter, hipStream_t stream);

// Waves of the persistent state-parallel kernel of constraint length K that
// the device can hold at once (0 on error).
int64_t resident_waves(int K);

}  // namespace pbvd_host
