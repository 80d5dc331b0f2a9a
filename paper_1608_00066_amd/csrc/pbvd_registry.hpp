// Codes that have decoder kernels compiled in, and the launch interface each
// per-code translation unit implements.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbvd_group_args.hpp"
#include "pbvd_kernel.hpp"
#include "pbvd_wave_args.hpp"

// X(index, K, R, g0, g1, g2, g3): generators in octal, gen[r] bit k = g_k.
// The first four are the codes of the benchmark workloads; the others are
// common maximum-free-distance codes for every K in 3..9 and R in 2..4, plus
// two codes whose first and last taps differ between generators.
#define PBVD_CODE_LIST(X)                   \
    X(0, 3, 2, 07, 05, 0, 0)                \
    X(1, 7, 2, 0171, 0133, 0, 0)            \
    X(2, 7, 3, 0133, 0171, 0165, 0)         \
    X(3, 9, 3, 0557, 0663, 0711, 0)         \
    X(4, 3, 2, 05, 07, 0, 0)                \
    X(5, 4, 2, 015, 017, 0, 0)              \
    X(6, 5, 2, 023, 035, 0, 0)              \
    X(7, 6, 2, 053, 075, 0, 0)              \
    X(8, 7, 2, 0133, 0171, 0, 0)            \
    X(9, 8, 2, 0247, 0371, 0, 0)            \
    X(10, 9, 2, 0561, 0753, 0, 0)           \
    X(11, 3, 3, 05, 07, 07, 0)              \
    X(12, 4, 3, 013, 015, 017, 0)           \
    X(13, 5, 3, 025, 033, 037, 0)           \
    X(14, 6, 3, 047, 053, 075, 0)           \
    X(15, 5, 4, 025, 027, 033, 037)         \
    X(16, 7, 4, 0117, 0127, 0155, 0171)     \
    X(17, 5, 2, 031, 027, 0, 0)             \
    X(18, 6, 2, 046, 073, 0, 0)

#define PBVD_COUNT_ONE(i, K, R, g0, g1, g2, g3) +1
constexpr int kNumCodes = 0 PBVD_CODE_LIST(PBVD_COUNT_ONE);
#undef PBVD_COUNT_ONE

// Pairs of registered codes of one constraint length whose batch tiles share
// one launch of the register kernel (16-bit metrics): X(index, code a, code b)
// with the registry indices above.  The rate-1/2 and rate-1/3 K=7 codes that
// are mixed in one batch of frames.
#define PBVD_PAIR_LIST(X) \
    X(0, 1, 2)

#define PBVD_COUNT_PAIR(i, a, b) +1
constexpr int kNumPairs = 0 PBVD_PAIR_LIST(PBVD_COUNT_PAIR);
#undef PBVD_COUNT_PAIR

struct RegisteredCode {
    int K, R;
    uint32_t gen[4];
};

// host-visible table, defined in pbvd_capi.hip
extern const RegisteredCode kRegisteredCodes[kNumCodes];

namespace pbvd {

struct LaunchRequest {
    KernelArgs args;
    int pm_bits;        // 16 or 32
    int input_kind;     // kSoftI8 or kHardU8
    int lb;             // log2 of lanes per PB (0, 1, 2)
    unsigned grid;      // workgroups of kBlockThreads
    hipStream_t stream;
};

constexpr int kBlockThreads = 256;

struct TileLaunchRequest {
    TileArgs args;
    int pm_bits;
    int input_kind;
    int lb;
    unsigned grid;
    unsigned block_threads;  // 64, 128 or 256 (one wave per tile)
    hipStream_t stream;
};

// Implemented by the translation unit compiled for code index IDX.
template <int IDX>
hipError_t launch_code(const LaunchRequest &req);
template <int IDX>
hipError_t launch_tiles(const TileLaunchRequest &req);
// Implemented by the translation unit compiled for pair index IDX and input
// kind KIND (tiles of both codes in one launch, 16-bit metrics only).
template <int IDX, int KIND>
hipError_t launch_tiles_pair(const TileLaunchRequest &req);

// State-parallel kernel (one wave per PB, run-time generators).
struct WaveLaunchRequest {
    wave::Args args;
    unsigned grid;       // workgroups of kBlockThreads (4 waves each)
    hipStream_t stream;
};
// Implemented by the translation unit compiled for constraint length K.
template <int K>
hipError_t launch_wave(const WaveLaunchRequest &req);
// Group-mapped kernel (a workgroup of 2^R waves per tile of 64 PBs).
struct GroupLaunchRequest {
    group::GroupArgs args;
    int R;
    unsigned grid;       // tiles of this launch
    hipStream_t stream;
};
// Implemented by the translation unit compiled for constraint length K.
template <int K>
hipError_t launch_group_kernel(const GroupLaunchRequest &req);

// Workgroups of the persistent state-parallel kernel of constraint length K
// that one compute unit holds at once (0 on error).
template <int K>
int wave_persistent_blocks_per_cu();

// Survivor layout of a code: dwords per stored row and stages per row.
__host__ __device__ constexpr int survivor_row_dwords(int K) { return (1 << (K - 2)) >= 16 ? (1 << (K - 2)) / 16 : 1; }
__host__ __device__ constexpr int survivor_row_stages(int K) { return (1 << (K - 2)) >= 16 ? 1 : 16 / (1 << (K - 2)); }
// Stages of one unrolled loop trip and dwords of one trip's symbol fetch
// (the same numbers Layout<> derives on the device).
__host__ __device__ constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }
__host__ __device__ constexpr int trip_stages(int K) {
    return (K - 1) / gcd_int(K - 1, survivor_row_stages(K)) * survivor_row_stages(K);
}
__host__ __device__ constexpr int trip_fetch_dwords(int K, int R) { return (trip_stages(K) * R + 3) / 4 + 1; }
// Lane groups of 2^lb lanes per PB (lb <= 3): 16-bit metrics and at least 16 packed
// registers per lane (the host mirror of lanes_supported<>).
__host__ __device__ constexpr bool lanes_allowed(int K, int pm_bits, int lb) {
    return lb == 0 || (lb >= 1 && lb <= 3 && pm_bits == 16 && ((1 << (K - 2)) >> lb) >= 16);
}

}  // namespace pbvd
