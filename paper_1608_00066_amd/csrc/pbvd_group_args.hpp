// Launch arguments of the group-mapped decoder kernel (pbvd_group.hpp),
// shared by the kernel and the host code that fills them.
#pragma once

#include <stdint.h>

#include "pbvd_kernel.hpp"

namespace pbvd {
namespace group {

// PBs of one workgroup: lane l of every wave works on PB l of the tile.
constexpr int kTilePbs = 64;

// Constraint lengths and rates the mapping takes: every butterfly group
// non-empty and of one size B = 2^(K-2-R) (the alpha map of Sec. III-B has
// full rank R), and a group's decisions of one stage fit a dword.
__host__ __device__ constexpr bool shape_ok(int K, int R) {
    return R >= 2 && R <= 4 && K - 2 - R >= 0 && (2 << (K - 2 - R)) <= 32;
}

// Stages of a survivor dword: 32 / (2B) (a group's 2B decisions per stage).
__host__ __device__ constexpr int stages_per_dword(int K, int R) { return 32 / (2 << (K - 2 - R)); }

// Survivor dwords of one tile whose longest PB has len stages:
// [stage dword][PB][group].
__host__ __device__ constexpr int64_t tile_dwords(int K, int R, int64_t len) {
    return (len + stages_per_dword(K, R) - 1) / stages_per_dword(K, R) * kTilePbs * (1 << R);
}

struct GroupArgs {
    const uint8_t *syms;      // symbol buffer (stream mode: stage 0 of the stream)
    const uint8_t *in_end;    // end of the readable symbol bytes
    uint8_t *out;
    uint32_t *out_words;      // kOutAtomic staging
    int64_t out_bytes;        // kOutDirect bound
    int32_t out_mode;         // kOutDirect / kOutAtomic / kOutBytes
    int32_t kind;             // kSoftI8 / kHardU8
    int32_t *final_pm;        // stream mode: [pb][N] or null
    uint32_t *sp;             // survivor area, sp_tile_dwords per workgroup
    int64_t sp_tile_dwords;
    // stream mode (descs == null): PBs pb_first + tile*64 + lane of a stream
    int64_t n, T, pb_first, pb_count;
    int32_t D, L, terminated;
    // batch mode: one descriptor per PB, 64 per tile (inactive padding)
    const LaneDesc *descs;
    int64_t tile_begin;       // first tile of this launch
    int64_t n_tiles;
    // per group w (its alpha, Sec. III-B Eq. 3-6): byte masks of the code
    // words alpha, beta, gamma, theta for the branch-metric dot products
    uint32_t bm_mask[16][4];
    // group w's butterflies j, ascending: jtab[w*B .. w*B + B)
    uint8_t jtab[128];
    // per state S: position of its decision in a stage's row of group
    // words, w*2B + 2*(rank of j = S mod N/2 in its group) + (S >= N/2)
    uint8_t ttab[256];
};

}  // namespace group
}  // namespace pbvd
