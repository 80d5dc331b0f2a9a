// Host launchers of the helper kernels in pbvd_aux.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbvd {

// Where the forward pass of one decode launch left its survivors.
struct SurvivorView {
    const uint32_t *sp;
    int64_t sp_wave_dwords;
    int64_t T, pb_first, pb_count;
    int64_t b_lo, b_hi, n_head, n_fold, n_int_waves;
    int32_t K, D, L;
    int32_t byte_perm;  // survivor bit layout: 1 = byte-permute, 0 = shift
    int32_t lb;         // 2^lb lanes per PB (64 >> lb PBs per wave)
    int32_t wave;       // 1: the state-parallel kernel's layout (one PB per
                        // slot of sp_wave_dwords, [trip][slot][lane] words)
};

hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t words_to_bytes(const uint32_t *w, uint8_t *out, int64_t nbytes, hipStream_t s);
hipError_t unpack_survivors(const SurvivorView &v, uint8_t *dec, hipStream_t s);
hipError_t branch_metrics(int R, int kind, const uint8_t *syms, int64_t n_stages, int32_t *out,
                          hipStream_t s);

}  // namespace pbvd
