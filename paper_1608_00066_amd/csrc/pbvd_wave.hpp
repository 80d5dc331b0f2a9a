// State-parallel decoder kernel: one wave decodes one parallel block (PB) of
// the parallel block-based Viterbi decoder (arXiv 1608.00066, Sec. III-A),
// one lane per trellis state (Sec. IV-A spreads a PB over threads in the
// same spirit: every thread updates a part of the states of each stage).
//
// Unlike the register kernel of pbvd_kernel.hpp (one lane per PB, the code a
// compile-time parameter) this kernel takes the generators as run-time
// arguments, so it decodes any rate-1/R code with 3 <= K <= 9, R <= 4, and a
// PB's D + 2L stages run 64 lanes wide: a short stream or a single frame
// finishes in a few microseconds instead of the hundreds a lane needs.
//
// Position map.  State d of stage t lives at position u = rotl_V^(t mod V)(d)
// (V = K-1 bits).  Then the butterfly of Sec. III-B at stage t pairs the
// positions that differ in bit ph = t mod V: the even one holds the upper
// predecessor S_2j, the odd one S_2j+1, and the new metrics of S_j (input 0)
// and S_j+2^(V-1) (input 1) go back to the even and the odd position.
// Position u is lane u mod 64, register slot u / 64 (K = 8: 2 slots, K = 9:
// 4).  For K < 7 the lanes above 2^V repeat the low ones.
//
// Exchanges.  At phase ph every position needs the metric of the pair's
// even and odd position: lane bits 0 and 1 with DPP quad permutes, bits 2
// and 3 with DPP row shifts restricted to the banks that read across, bit 4
// and 5 with the gfx950 permlane16/permlane32 swaps (one instruction gives
// both halves), slot bits inside the lane.
//
// Branch metrics.  A branch's code word is c = (c^(1)..c^(R)) of Eq. 2; its
// metric is sum over r of c_r q_r (the Sec. II distance minus a constant
// shared by all branches of the stage, which changes no decision).  Each lane
// keeps, per phase and slot, the code-word bits of its two branches as byte
// masks and forms each metric with one v_dot4_i32_i8 of the stage's R
// symbols (packed in one dword) and the mask.
//
// Survivors.  dec = 1 when the lower branch (from S_2j+1) is strictly
// cheaper, as Eq. 1 with ties to the upper branch.  The survivor memory is
// kept by register exchange within a trip of W = V * floor(32 / V) stages (a
// trip starts at phase 0): each position carries the decisions of the
// survivor path into it, h = h_pred << 1 | dec, its predecessor's word
// exchanged like the metric.  At the end of a trip the words go to HBM,
// [trip][slot][lane]: the word at position u holds the W decisions of the
// survivor into u over the trip, the k-th stage's at bit W-1-k.
//
// Traceback (Alg. 1, Kernel 2), a trip at a time on the scalar unit.  A
// state's input bit is bit t mod V of its position, and the predecessor's
// position is the position with that bit replaced by the decision; after a
// whole trip (a multiple of V stages) every bit has been replaced.  So from
// the position P at a trip's end and its word h (v_readlane of lane P mod
// 64), the position at the trip's start is the decisions of the trip's
// first V stages, and the input bits of the trip are the decisions of its
// stages V.. (for the first W-V stages) followed by the bits of P: two bit
// reversals and shifts per trip instead of a step per stage.  A debug
// variant also stores the per-stage decisions of every position, the
// survivor layout of the plain method.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "pbvd_kernel.hpp"
#include "pbvd_wave_args.hpp"

namespace pbvd {
namespace wave {

// Even and odd position's value of the pair whose bit is lane bit B.
template <int B>
__device__ __forceinline__ void pair_values(int v, int &e, int &o) {
    if constexpr (B == 0) {
        e = __builtin_amdgcn_mov_dpp(v, quad_sel(0, 0, 2, 2), 0xf, 0xf, false);
        o = __builtin_amdgcn_mov_dpp(v, quad_sel(1, 1, 3, 3), 0xf, 0xf, false);
    } else if constexpr (B == 1) {
        e = __builtin_amdgcn_mov_dpp(v, quad_sel(0, 1, 0, 1), 0xf, 0xf, false);
        o = __builtin_amdgcn_mov_dpp(v, quad_sel(2, 3, 2, 3), 0xf, 0xf, false);
    } else if constexpr (B == 2) {
        // banks (groups of 4 lanes) 1 and 3 read 4 lanes down, 0 and 2 up
        e = __builtin_amdgcn_update_dpp(v, v, 0x114, 0xf, 0xa, false);
        o = __builtin_amdgcn_update_dpp(v, v, 0x104, 0xf, 0x5, false);
    } else if constexpr (B == 3) {
        e = __builtin_amdgcn_update_dpp(v, v, 0x118, 0xf, 0xc, false);
        o = __builtin_amdgcn_update_dpp(v, v, 0x108, 0xf, 0x3, false);
    } else if constexpr (B == 4) {
        // rows 1, 3 of the first operand swap with rows 0, 2 of the second:
        // the first result holds rows (0, 0, 2, 2), the second (1, 1, 3, 3)
        const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
        e = (int)r[0];
        o = (int)r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
        e = (int)r[0];
        o = (int)r[1];
    }
}

// up += dot(q of lane LANE of the row, mu); lo += dot(q of lane LANE, ml):
// v_dot4c_i32_i8 with the symbol dword broadcast by DPP row_newbcast (written
// out: the compiler does not fold the broadcast into the dot product).  A
// dot product's result may be read by another vector instruction only three
// wait states after it is written, so the pair ends with s_nop 2 (the
// compiler cannot see into the statement to insert them).
template <int LANE>
__device__ __forceinline__ void dot_pair(int &up, int &lo, uint32_t q, uint32_t mu, uint32_t ml) {
    asm("v_dot4c_i32_i8_dpp %0, %2, %3 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
        "v_dot4c_i32_i8_dpp %1, %2, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 2"
        : "+v"(up), "+v"(lo)
        : "v"(q), "v"(mu), "v"(ml), "n"(LANE));
}

// acc << 1 | (diff's sign bit)
__device__ __forceinline__ uint32_t push_sign(uint32_t acc, int diff) {
    return __builtin_amdgcn_alignbit(acc, (uint32_t)diff, 31);
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v = min(v, __shfl_xor(v, m, kWave));
    return v;
}

__device__ __forceinline__ int parity32(uint32_t x) { return __builtin_popcount(x) & 1; }

// A 64-bit value every lane holds alike, made provably wave-uniform.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int V>
__device__ __forceinline__ uint32_t rotr_rt32(uint32_t u, int s) {
    s %= V;
    return s == 0 ? u : (((u >> s) | (u << (V - s))) & ((1u << V) - 1u));
}

// The PB a wave decodes.
struct Job {
    const uint8_t *in;   // symbols of the first forward stage
    int len;             // forward stages
    int store0;          // first traced (decoded) stage
    int dec_end;         // end of the decoded range (stage index)
    bool known;          // starts from encoder state 0
    bool argmin;         // traceback from the least-metric state
    int64_t out_bit0;    // output bit of the first decoded stage
    int32_t *pm_out;     // final metrics or null
};

// New metric and path word of a position from its two candidates: the
// lower (odd) branch wins only when strictly cheaper (Eq. 1, ties to the
// upper branch); h = (the winner's word) << 1 | dec in one add with carry
// (h + h + dec).  Written out because the compiler spends three
// instructions on the word.  A VCC written by a vector instruction is read
// as a mask two wait states later, and the words written here may be read
// by DPP (two wait states) right after the statement.
__device__ __forceinline__ void select_path(int &pm, uint32_t &h, int up, int lo, uint32_t he, uint32_t ho) {
    asm("v_cmp_lt_i32 vcc, %[lo], %[up]\n\t"
        "v_min_i32 %[pm], %[lo], %[up]\n\t"
        "s_nop 0\n\t"
        "v_cndmask_b32 %[h], %[he], %[ho], vcc\n\t"
        "v_addc_co_u32 %[h], vcc, %[h], %[h], vcc\n\t"
        "s_nop 1"
        : [pm] "=&v"(pm), [h] "=&v"(h)
        : [lo] "v"(lo), [up] "v"(up), [he] "v"(he), [ho] "v"(ho)
        : "vcc");
}

// DEC: also store each stage's decisions (the debug survivor export) at
// dec_wave, in the [trip][slot][lane] layout of the path words.
template <int V, bool DEC>
__device__ __forceinline__ void decode_pb(const Args &a, const Job &j, const WaveCode &code, uint32_t *sp_wave,
                                          uint32_t *dec_wave) {
    constexpr int N = 1 << V;
    constexpr int SL = slots(V);
    constexpr int NL = N < kWave ? N : kWave;   // distinct positions per slot
    constexpr int LB = V < 6 ? V : 6;            // lane bits of a position
    constexpr int W = trip_stages(V);
    constexpr int G = (W + 15) / 16;             // symbol dwords per lane and trip

    // the lane number through an empty asm statement: what derives from it
    // (the branch masks above all) is recomputed for each PB instead of
    // being hoisted out of the persistent loop into registers of their own
    int lane = (int)(threadIdx.x & (kWave - 1));
    asm volatile("" : "+v"(lane));
    const int len = j.len;
    const int R = code.R;
    const bool hard = code.kind == kHardU8;
    // Trips are aligned to the end of the forward range: trip i holds
    // stages [i*W - off, (i+1)*W - off), so the first trip starts off
    // stages in and the last one ends at stage len, at phase 0.
    const int n_trips = (len + W - 1) / W;
    const int off = n_trips * W - len;

    // Symbols: the R symbols of stage t are packed in one dword (bytes
    // 0..R-1; the bytes above belong to the next stage and meet zero mask
    // bytes).  Lane l holds those of the trip's stage g*16 + (l mod 16) in
    // qv[g] (every row of 16 lanes the same), and each stage broadcasts its
    // dword from lane k mod 16 of every row into the dot product (DPP
    // row_newbcast).  A trip's symbols are loaded a trip ahead.
    const uint8_t *const in = j.in;
    const int sl = lane & 15;
    auto load_q = [&](uint32_t (&lo)[G], uint32_t (&hi)[G], uint32_t (&mis)[G], int tt0) PBVD_INLINE_LAMBDA {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            int t = tt0 + g * 16 + sl;
            t = t < 0 ? 0 : t;  // stages before the first are never used
            const uint8_t *p = in + (int64_t)t * R;  // R: the code's rate, wave-uniform
            mis[g] = (uint32_t)((uintptr_t)p & 3u);
            const uint8_t *pa = p - mis[g];
            if (pa + 8 <= a.in_end) {
                const uint32_t *w = reinterpret_cast<const uint32_t *>(pa);
                lo[g] = __builtin_nontemporal_load(w);
                hi[g] = __builtin_nontemporal_load(w + 1);
            } else {
                // the end of the input (bytes past it read as 0)
                uint32_t v0 = 0u, v1 = 0u;
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) {
                    if (pa + bb < a.in_end) v0 |= (uint32_t)pa[bb] << (8 * bb);
                    if (pa + 4 + bb < a.in_end) v1 |= (uint32_t)pa[4 + bb] << (8 * bb);
                }
                lo[g] = v0;
                hi[g] = v1;
            }
        }
    };
    auto make_q = [&](const uint32_t (&lo)[G], const uint32_t (&hi)[G], const uint32_t (&mis)[G],
                      uint32_t (&qv)[G]) PBVD_INLINE_LAMBDA {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            uint32_t q = __builtin_amdgcn_alignbyte(hi[g], lo[g], mis[g]);
            if (hard) q = 0x01010101u + (q & 0x01010101u) * 0xfeu;  // bit -> +1 / -1
            qv[g] = q;
        }
        // two wait states between these writes and the DPP reads of qv
        if constexpr (G == 1) asm volatile("s_nop 1" : "+v"(qv[0]));
        else asm volatile("s_nop 1" : "+v"(qv[0]), "+v"(qv[1]));
    };

    // the first trip's symbols are requested before the masks are formed
    // (with one slot: with more, the masks' registers leave no room)
    uint32_t nlo[G], nhi[G], nmis[G];
    if constexpr (SL == 1) load_q(nlo, nhi, nmis, -off);

    // ---- per-lane code-word masks of the two branches into each position,
    //      per phase and slot (Eq. 2 with the run-time generators) ----
    uint32_t mup[V][SL], mlo[V][SL];
#pragma unroll
    for (int ph = 0; ph < V; ++ph) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const uint32_t u = (uint32_t)(s * kWave + (lane & (NL - 1)));
            const uint32_t even = u & ~(1u << ph);
            const uint32_t se = rotr_rt32<V>(even, ph);   // the upper predecessor S_2j
            const uint32_t x = (u >> ph) & 1u;             // input bit of the branch
            const uint32_t reg = (x << V) | se;
            uint32_t mu = 0, ml = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {  // generators past R are 0: zero mask bytes
                mu |= (uint32_t)parity32(code.gen[r] & reg) << (8 * r);
                ml |= (uint32_t)parity32(code.gen[r] & (reg | 1u)) << (8 * r);
            }
            mup[ph][s] = mu;
            mlo[ph][s] = ml;
        }
    }

    if constexpr (SL > 1) load_q(nlo, nhi, nmis, -off);

    // ---- initial metrics: with a known start, state 0 (position 0 at any
    //      phase) at 0 and the others at 8192; otherwise all 0 ----
    int pm[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int u = s * kWave + (lane & (NL - 1));
        pm[s] = (j.known && u != 0) ? 8192 : 0;
    }

    // path words (register exchange within a trip)
    uint32_t hist[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) hist[s] = 0;

    uint32_t *const sp_lane = sp_wave + lane;  // [trip][slot][lane]

    // one trellis stage, the k-th of its trip (phase k mod V); each
    // candidate is its predecessor's metric plus the branch metric, the dot
    // product accumulating onto the exchanged metric; the path words follow
    // the metrics
    auto stage = [&](auto kc, const uint32_t (&qv)[G], uint32_t (&acc)[SL]) PBVD_INLINE_LAMBDA {
        constexpr int k = decltype(kc)::value;
        constexpr int PH = k % V;
        const uint32_t q = qv[k / 16];
        if constexpr (PH < LB) {
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                int up, lo, he, ho;
                pair_values<PH>(pm[s], up, lo);
                pair_values<PH>((int)hist[s], he, ho);
                dot_pair<k % 16>(up, lo, q, mup[PH][s], mlo[PH][s]);
                if constexpr (DEC) acc[s] = push_sign(acc[s], lo - up);
                select_path(pm[s], hist[s], up, lo, (uint32_t)he, (uint32_t)ho);
            }
        } else {
            constexpr int M = 1 << (PH - 6);  // slot bit
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                if (s & M) continue;
                int up0 = pm[s], lo0 = pm[s | M], up1 = pm[s], lo1 = pm[s | M];
                const uint32_t he = hist[s], ho = hist[s | M];
                dot_pair<k % 16>(up0, lo0, q, mup[PH][s], mlo[PH][s]);
                dot_pair<k % 16>(up1, lo1, q, mup[PH][s | M], mlo[PH][s | M]);
                if constexpr (DEC) {
                    acc[s] = push_sign(acc[s], lo0 - up0);
                    acc[s | M] = push_sign(acc[s | M], lo1 - up1);
                }
                select_path(pm[s], hist[s], up0, lo0, he, ho);
                select_path(pm[s | M], hist[s | M], up1, lo1, he, ho);
            }
        }
    };

    // The traceback reads the path words of trips trip_bot..n_trips-1
    // through a ring of kRing trips.  With one slot, the words of the last
    // trip stay in registers and the loads of the trips below it are issued
    // at the start of the last forward trip, so that they have arrived when
    // the traceback starts.
    const int trip_bot = (j.store0 + off) / W;
    constexpr int kRing = SL == 1 ? 8 : SL == 2 ? 6 : 4;
    constexpr bool kEarlyRing = SL == 1;
    uint32_t ring[kRing][SL];
    auto load_trip = [&](uint32_t (&dst)[SL], int trip) PBVD_INLINE_LAMBDA {
        trip = trip < trip_bot ? trip_bot : trip;
#pragma unroll
        for (int s = 0; s < SL; ++s) dst[s] = __builtin_nontemporal_load(sp_lane + (trip * SL + s) * kWave);
    };

    // ---- forward procedure (Eq. 1) ----
    for (int trip = 0; trip < n_trips; ++trip) {
        const int tt0 = trip * W - off;  // stage of the trip's step 0
        if constexpr (kEarlyRing) {
            if (trip + 1 == n_trips) {
                // trips below the last one are stored already (a clamped
                // load of the last trip itself is never used)
                static_for<1, kRing - 1>([&](auto dc) PBVD_INLINE_LAMBDA {
                    load_trip(ring[decltype(dc)::value], trip - decltype(dc)::value);
                    return true;
                });
            }
        }
        uint32_t qv[G];
        make_q(nlo, nhi, nmis, qv);
        if (trip + 1 < n_trips) load_q(nlo, nhi, nmis, tt0 + W);  // a trip ahead
        uint32_t acc[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) acc[s] = 0;
        if (trip > 0 || off == 0) {
            static_for<0, W>([&](auto kc) PBVD_INLINE_LAMBDA {
                stage(kc, qv, acc);
                return true;
            });
        } else {
            // the first trip starts at step off (its lower bits stay 0)
            static_for<0, W>([&](auto kc) PBVD_INLINE_LAMBDA {
                if (decltype(kc)::value >= off) stage(kc, qv, acc);
                return true;
            });
        }
        // step k of the trip at bit W-1-k
#pragma unroll
        for (int s = 0; s < SL; ++s) __builtin_nontemporal_store(hist[s], sp_lane + (trip * SL + s) * kWave);
        if constexpr (DEC) {
#pragma unroll
            for (int s = 0; s < SL; ++s)
                __builtin_nontemporal_store(acc[s], dec_wave + lane + (trip * SL + s) * kWave);
        }
        // exact renormalization: every metric minus one shared value
        const int ref = __builtin_amdgcn_readfirstlane(pm[0]);
#pragma unroll
        for (int s = 0; s < SL; ++s) pm[s] -= ref;
    }

    // ---- final metrics and traceback start (Sec. III-A; Sec. II at the end
    //      of an unterminated stream).  The forward range ends at phase 0:
    //      position u holds state u. ----
    uint32_t P = 0;
    if (j.argmin || j.pm_out) {
        int m = pm[0];
#pragma unroll
        for (int s = 1; s < SL; ++s) m = min(m, pm[s]);
        m = wave_min(m);
        if (j.argmin) {
            int best = N;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int u = s * kWave + (lane & (NL - 1));
                if (pm[s] == m && u < best) best = u;
            }
            P = (uint32_t)__builtin_amdgcn_readfirstlane(wave_min(best));
        }
        if (j.pm_out && lane < NL) {
#pragma unroll
            for (int s = 0; s < SL; ++s) j.pm_out[s * kWave + lane] = pm[s] - m;
        }
    }

    // ---- traceback (Alg. 1, Kernel 2) ----
    // A trip at a time from its path word (the last trip is full; stages
    // below the decoded range at the bottom are harmless); the input bits of
    // a trip form `word` (bit i = the trip's i-th stage) and the decoded
    // ones are merged into the output word under assembly.
    const int store0 = j.store0, dec_end = j.dec_end;
    const int n_dec = dec_end - store0;
    int cm = (n_dec - 1) >> 5;  // output word under assembly (relative to the PB)
    uint32_t cw = 0;

    auto flush = [&]() PBVD_INLINE_LAMBDA {
        if (lane != 0) return;
        const int rel = cm * 32;
        const int m = n_dec - rel < 32 ? n_dec - rel : 32;
        const int64_t bitpos = j.out_bit0 + rel;
        if (a.out_mode == kOutDirect) {
            const int64_t byte = bitpos >> 3;
            if (m == 32 && byte + 4 <= a.out_bytes) {
                *reinterpret_cast<uint32_t *>(a.out + byte) = cw;
            } else {
                for (int bb = 0; bb < ((m + 7) >> 3); ++bb)
                    if (byte + bb < a.out_bytes) a.out[byte + bb] = (uint8_t)(cw >> (8 * bb));
            }
        } else if (a.out_mode == kOutAtomic) {
            const uint32_t shf = (uint32_t)(bitpos & 31);
            uint32_t *wp = a.out_words + (bitpos >> 5);
            atomicOr(wp, cw << shf);
            if (shf && (cw >> (32 - shf))) atomicOr(wp + 1, cw >> (32 - shf));
        } else {
            uint8_t *ob = a.out + (bitpos >> 3);
            for (int bb = 0; bb < ((m + 7) >> 3); ++bb) ob[bb] = (uint8_t)(cw >> (8 * bb));
        }
    };

    auto run_trip = [&](const uint32_t (&hw)[SL], int trip) PBVD_INLINE_LAMBDA {
        uint32_t h;
        if constexpr (SL == 1) {
            h = (uint32_t)__builtin_amdgcn_readlane((int)hw[0], (int)(P & 63u));
        } else {
            const int l = (int)(P & 63u);
            const uint32_t slot = P >> 6;
            h = 0;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)hw[s], l);
                h = slot == (uint32_t)s ? v : h;
            }
        }
        // decision of the trip's stage k: bit W-1-k of h, i.e. bit
        // 32-W+k of its reversal
        const uint32_t rev = __builtin_bitreverse32(h);
        const uint32_t word = (rev >> (32 - W + V)) | (P << (W - V));
        P = (rev >> (32 - W)) & (uint32_t)(N - 1);
        // decoded stages of the trip: [lo, hi), at bits lo - tt0 .. of word
        const int tt0 = trip * W - off;
        const int lo = store0 > tt0 ? store0 : tt0;
        const int hi = dec_end < tt0 + W ? dec_end : tt0 + W;
        if (lo < hi) {
            const int nb = hi - lo;
            uint32_t bits = word >> (lo - tt0);
            bits = nb >= 32 ? bits : bits & ((1u << nb) - 1u);
            const int r = lo - store0;   // first decoded bit, relative
            const int base = cm * 32;
            if (r >= base) {
                cw |= bits << (r - base);
            } else {
                // the chunk reaches into the word below: the current one is
                // complete (r < base <= r + nb <= base + 32)
                const int dn = base - r;  // 1..32 bits below the current word
                if (dn < 32) cw |= bits >> dn;
                flush();
                --cm;
                cw = dn < 32 ? bits << (32 - dn) : bits;
            }
        }
    };

    const int trip_top = n_trips - 1;
    if constexpr (kEarlyRing) {
#pragma unroll
        for (int s = 0; s < SL; ++s) ring[0][s] = hist[s];
    } else {
        static_for<0, kRing - 1>([&](auto dc) PBVD_INLINE_LAMBDA {
            load_trip(ring[decltype(dc)::value], trip_top - decltype(dc)::value);
            return true;
        });
    }
    int trip = trip_top;
    for (;;) {
        const bool more = static_for<0, kRing>([&](auto dc) PBVD_INLINE_LAMBDA {
            constexpr int d = decltype(dc)::value;
            load_trip(ring[(d + kRing - 1) % kRing], trip - (kRing - 1));
            run_trip(ring[d], trip);
            if (trip <= trip_bot) return false;
            --trip;
            return true;
        });
        if (!more) break;
    }
    flush();  // word 0
}

// Job of PB `idx` of a stream (Sec. III-A geometry; stream mode).
template <int V>
__device__ __forceinline__ Job stream_job(const Args &a, const uint8_t *syms, int64_t idx) {
    constexpr int N = 1 << V;
    Job j;
    const int64_t b = a.pb_first + idx;
    const int64_t D = a.D, L = a.L;
    const int64_t d0 = b * D;
    const int64_t f0 = d0 - L < 0 ? 0 : d0 - L;
    const int64_t f1 = d0 + D + L > a.T ? a.T : d0 + D + L;
    const int64_t d1 = d0 + D > a.n ? a.n : d0 + D;
    j.in = syms + f0 * a.codes[0].R;
    j.len = (int)(f1 - f0);
    j.store0 = (int)(d0 - f0);
    j.dec_end = (int)(d1 - f0);
    j.known = f0 == 0;
    j.argmin = f1 == a.T && !a.terminated;
    j.out_bit0 = idx * D;
    j.pm_out = a.final_pm ? a.final_pm + idx * N : nullptr;
    return j;
}

// Job of descriptor idx of a work list (batches); *code_idx receives its code.
__device__ __forceinline__ Job desc_job(const Args &a, const uint8_t *syms, int64_t idx, int *code_idx, bool *active) {
    Job j;
    const LaneDesc &d = a.descs[idx];
    j.in = syms + uniform64(d.sym);
    j.len = __builtin_amdgcn_readfirstlane(d.len);
    j.store0 = __builtin_amdgcn_readfirstlane(d.store0);
    j.dec_end = __builtin_amdgcn_readfirstlane(d.dec_end);
    const int fl = __builtin_amdgcn_readfirstlane(d.flags);
    j.known = (fl & kLaneKnown) != 0;
    j.argmin = (fl & kLaneArgmin) != 0;
    j.out_bit0 = uniform64(d.out_bit);
    j.pm_out = nullptr;
    *code_idx = (fl >> kDescCodeShift) & 0xff;
    *active = (fl & kLaneActive) != 0;
    return j;
}

// One wave per PB; 4 independent waves per 256-thread workgroup.  Modes:
// kModeList, a stream's PBs (descs == null) or a work list's PBs (descs),
// one per wave; kModePersist, persistent waves that take the work list's
// PBs in list order (longest first) from work counters until it is exhausted --
// one launch for the PBs of every code of this K, whatever their count (a
// kernel of its own: the state it keeps across PBs would cost the other
// modes a wave per SIMD); kModeDecisions, a stream's PBs with every stage's
// decisions stored as well (a.dec_sp, the debug survivor export).
// syms: the symbol buffer (the same pointer as a.syms), a separate parameter
// so that its loads may use the scalar unit (nothing the kernel writes
// aliases it).
template <int V, int MODE>
__global__ void __launch_bounds__(256) decode_wave_kernel(const Args a, const uint8_t *__restrict__ syms) {
    const int64_t wl = (int64_t)blockIdx.x * (blockDim.x / kWave) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (wl >= a.n_waves) return;
    uint32_t *const sp = a.sp + wl * a.sp_wave_dwords;
    if constexpr (MODE == kModePersist) {
        // The next PB from the counter of this workgroup's XCD (workgroups
        // go to the 8 XCDs in turn): with nc counters (8, fewer for grids
        // of fewer workgroups, so that every counter has waves), counter x
        // hands out PBs x, x + nc, x + 2 nc, ... of the list, so each XCD
        // takes an equal share of every length, longest first, and the
        // counters spread the atomics.
        const int lane = (int)(threadIdx.x & (kWave - 1));
        const int nc = gridDim.x < (unsigned)kCounters ? (int)gridDim.x : kCounters;
        const int x = (int)(blockIdx.x % (unsigned)nc);
        for (;;) {
            uint32_t got = 0;
            if (lane == 0) got = atomicAdd(a.counter + kCounterStride * x, 1u);
            const int64_t idx = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)got) * nc + x;
            if (idx >= a.n_items) return;
            int ci;
            bool active;
            const Job j = desc_job(a, syms, idx, &ci, &active);
            if (active) decode_pb<V, false>(a, j, a.codes[ci], sp, nullptr);
        }
    } else if constexpr (MODE == kModeDecisions) {
        decode_pb<V, true>(a, stream_job<V>(a, syms, a.wave_begin + wl), a.codes[0], sp,
                           a.dec_sp + wl * a.sp_wave_dwords);
    } else {
        const int64_t idx = a.wave_begin + wl;
        int ci = 0;
        bool active = true;
        const Job j = a.descs ? desc_job(a, syms, idx, &ci, &active) : stream_job<V>(a, syms, idx);
        if (active) decode_pb<V, false>(a, j, a.codes[ci], sp, nullptr);
    }
}

}  // namespace wave
}  // namespace pbvd
