// Launch arguments and survivor layout of the state-parallel (one wave per
// PB) decoder kernel of pbvd_wave.hpp, shared with the host code.
#pragma once

#include <stdint.h>

#include "pbvd_kernel.hpp"

namespace pbvd {
namespace wave {

// Stages per survivor dword: a whole number of phase cycles.
__host__ __device__ constexpr int trip_stages(int V) { return V * (32 / V); }
// Register slots per lane (2^V states over 64 lanes).
__host__ __device__ constexpr int slots(int V) { return V > 6 ? 1 << (V - 6) : 1; }
// Survivor dwords of one PB of len forward stages.
__host__ __device__ constexpr int64_t pb_dwords(int V, int64_t len) {
    return (len + trip_stages(V) - 1) / trip_stages(V) * slots(V) * kWave;
}

// A code of the state-parallel kernel: the kernel takes the generators, the
// rate and the input kind at run time, so one kernel per K decodes them all.
struct WaveCode {
    uint32_t gen[4];   // gen[r] bit k = g_k of Eq. 2; 0 for r >= R
    int32_t R;         // symbols per stage (2..4)
    int32_t kind;      // kSoftI8 / kHardU8
};
constexpr int kMaxWaveCodes = 16;
// Work counters of a persistent launch: one per XCD, a cache line apart.
constexpr int kCounters = 8;
constexpr int kCounterStride = 64;
// Kernel modes (decode_wave_kernel).
enum { kModeList = 0, kModePersist = 1, kModeDecisions = 2 };
// Descriptor flags (LaneDesc::flags) carry the PB's code index in bits 8..15.
constexpr int kDescCodeShift = 8;

struct Args {
    const uint8_t *syms;     // symbols; stream mode: stage 0 of the stream
    const uint8_t *in_end;   // end of the readable symbol bytes
    uint8_t *out;            // packed decoded bits
    uint32_t *out_words;     // zeroed word staging (atomic output) or null
    int64_t out_bytes;       // bytes of `out` (direct output bound)
    int32_t *final_pm;       // [PB][2^V] normalized final metrics or null
    uint32_t *sp;            // survivor scratch, sp_wave_dwords per wave
    int64_t sp_wave_dwords;
    // stream mode (descs == null): PBs [pb_first + wave_begin, + n_waves)
    int64_t n, T, pb_first;
    int32_t D, L, terminated;
    int32_t out_mode;        // kOutDirect / kOutAtomic / kOutBytes
    // tile mode: one descriptor per PB (lane descriptor of the batch work list)
    const LaneDesc *descs;
    int64_t wave_begin;      // first PB of this launch (relative to pb_first / descs)
    int64_t n_waves;         // PBs of this launch; persistent mode: waves of the grid
    // persistent mode (counter != null): the waves take descriptors
    // [0, n_items) one at a time from kCounters work counters, kCounterStride
    // dwords apart (all zero at launch)
    uint32_t *counter;
    int64_t n_items;
    // debug mode (kModeDecisions): every stage's decisions, sp_wave_dwords
    // per wave, the same [trip][slot][lane] layout as sp
    uint32_t *dec_sp;
    WaveCode codes[kMaxWaveCodes];  // stream mode: codes[0]
};

}  // namespace wave
}  // namespace pbvd
