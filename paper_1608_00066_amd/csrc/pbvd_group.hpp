// Group-mapped decoder kernel: the intra-PB mapping of arXiv 1608.00066,
// Sec. III-B and Sec. IV-A (Alg. 1, Kernel 1).
//
// Grouping (Sec. III-B, Eq. 3-6).  The butterfly j (predecessors S_2j and
// S_2j+1, successors S_j and S_j+N/2) has the code words alpha (S_2j, input
// 0), beta = alpha ^ g_{K-1}, gamma = alpha ^ g_0 and theta = alpha ^
// g_{K-1} ^ g_0, so the N/2 butterflies fall into N_c = 2^R groups by alpha,
// and one group shares the four branch metrics of a stage.  The host lists
// each group's butterflies (codes whose alpha map has full rank R, so every
// group holds B = N/2/N_c of them).
//
// Mapping.  A workgroup decodes a tile of 64 PBs with N_c waves: wave w
// takes group w, lane l PB l of the tile, so the N_c lanes l of the waves
// form the paper's virtual processor of one PB.  Per stage a lane forms the
// four metrics of its group with one v_dot4_i32_i8 each (the correlation
// sum of c_r q_r over the stage's R int8 symbols, the Sec. II distance
// minus a constant shared by all branches, which changes no decision),
// reads the metrics of its B butterflies' predecessors from LDS, writes the
// successors' back (the layout is [state][PB], as the paper's PM[N][32], so
// a wave's accesses of one state fall in consecutive banks; two buffers, one
// barrier per stage), and shifts its 2B decisions (1 = the lower branch
// strictly cheaper, Eq. 1, ties to the upper) into a dword.
//
// Survivors.  A dword holds one group's decisions of 32 / 2B consecutive
// stages; the tile's survivor area is [stage dword][PB][group], so a PB's
// N_c group words of a stage are adjacent (one row) and the traceback reads
// a row per dword of stages, independent of the traced state (prefetched).
// Metrics are int32 with no renormalization (PBs up to 2^20 stages).
//
// PBs of one tile may differ in length: their stages are aligned at the
// end, and a PB holds its initial metrics until its first stage.
//
// Traceback (Alg. 1, Kernel 2): after the forward pass wave 0 traces the
// tile's 64 PBs, one per lane, from state 0 or from the least metric (the
// unterminated end of a stream); a state's decision sits at bit
// ttab[state] of the row, and the bits of the decoded range go out LSB
// first.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "pbvd_group_args.hpp"
#include "pbvd_kernel.hpp"

namespace pbvd {
namespace group {

constexpr int32_t kBig = 8192;

template <int V, int R>
__host__ __device__ constexpr size_t lds_bytes() {
    return (size_t)2 * (1 << V) * kTilePbs * 4 + (1 << V);
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v = max(v, __shfl_xor(v, m, kWave));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v = min(v, __shfl_xor(v, m, kWave));
    return __builtin_amdgcn_readfirstlane(v);
}

// Workgroup barrier for the metrics in LDS: this wave's LDS accesses done,
// then s_barrier.  Unlike __syncthreads it does not wait for the wave's
// global loads and stores (the next symbols in flight, the survivor stores),
// which only wave 0's traceback reads, after a full barrier.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int V, int R>
__global__ void __launch_bounds__(kTilePbs << R) decode_group_kernel(const GroupArgs a) {
    constexpr int N = 1 << V;
    constexpr int HALF = N / 2;
    constexpr int NC = 1 << R;
    constexpr int B = HALF / NC;          // butterflies of a group
    constexpr int WB = 2 * B;             // decisions of a group per stage
    constexpr int SPD = 32 / WB;          // stages per survivor dword
    constexpr int CH = 16;                // stages per symbol chunk
    constexpr int NDW = (CH * R + 3) / 4 + 2;
    constexpr int ROW = N * kTilePbs;     // int32 metrics of one buffer
    static_assert(B >= 1 && WB <= 32 && CH % SPD == 0, "shape outside the mapping");

    extern __shared__ int32_t lds[];
    uint8_t *const tt = reinterpret_cast<uint8_t *>(lds + 2 * ROW);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int64_t tile = a.tile_begin + blockIdx.x;

    for (int s = (int)threadIdx.x; s < N; s += (int)blockDim.x) tt[s] = a.ttab[s];

    // ---- this lane's PB (Sec. III-A geometry) ----
    const uint8_t *in = a.syms;
    int len = 0, store0 = 0, dec_end = 0;
    bool known = false, argmin = false;
    int64_t out_bit0 = 0, pb_row = -1;
    if (a.descs) {
        const LaneDesc &d = a.descs[tile * kTilePbs + lane];
        if (d.flags & kLaneActive) {
            in = a.syms + d.sym;
            len = d.len;
            store0 = d.store0;
            dec_end = d.dec_end;
            known = (d.flags & kLaneKnown) != 0;
            argmin = (d.flags & kLaneArgmin) != 0;
            out_bit0 = d.out_bit;
        }
    } else {
        const int64_t idx = tile * kTilePbs + lane;
        if (idx < a.pb_count) {
            const int64_t b = a.pb_first + idx;
            const int64_t d0 = b * a.D;
            const int64_t f0 = d0 - a.L < 0 ? 0 : d0 - a.L;
            const int64_t f1 = d0 + a.D + a.L > a.T ? a.T : d0 + a.D + a.L;
            const int64_t d1 = d0 + a.D > a.n ? a.n : d0 + a.D;
            in = a.syms + f0 * R;
            len = (int)(f1 - f0);
            store0 = (int)(d0 - f0);
            dec_end = (int)(d1 - f0);
            known = f0 == 0;
            argmin = f1 == a.T && !a.terminated;
            out_bit0 = idx * a.D;
            pb_row = idx;
        }
    }
    // every wave of the workgroup derives the same tile shape
    const int max_len = wave_max_i(len);
    if (max_len == 0) return;
    const int start = max_len - len;           // this PB's first step
    const int max_start = wave_max_i(len > 0 ? start : 0);

    // ---- this group's butterflies and branch-metric masks ----
    int rd[B], wr[B], init_lo[B], init_hi[B], init_e[B], init_o[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = a.jtab[w * B + b];
        rd[b] = 2 * j * kTilePbs + lane;   // S_2j (S_2j+1 one row further)
        wr[b] = j * kTilePbs + lane;       // S_j (S_j+N/2 HALF rows further)
        init_e[b] = (known && 2 * j != 0) ? kBig : 0;
        init_o[b] = known ? kBig : 0;
        init_lo[b] = (known && j != 0) ? kBig : 0;
        init_hi[b] = known ? kBig : 0;
    }
    const uint32_t m_al = a.bm_mask[w][0], m_be = a.bm_mask[w][1];
    const uint32_t m_ga = a.bm_mask[w][2], m_th = a.bm_mask[w][3];

    // initial metrics (Sec. III-A): with a known start, state 0 at 0 and the
    // others at 8192; else all 0.  Each state is a predecessor of exactly
    // one butterfly, so the group's waves cover every state once.
#pragma unroll
    for (int b = 0; b < B; ++b) {
        lds[rd[b]] = init_e[b];
        lds[rd[b] + kTilePbs] = init_o[b];
    }
    __syncthreads();

    uint32_t *const sp_tile = a.sp + (int64_t)blockIdx.x * a.sp_tile_dwords;
    const bool hard = a.kind == kHardU8;

    // ---- forward procedure (Eq. 1) ----
    // A chunk's symbols: the aligned dwords around the PB's stages
    // [k0 - start, k0 - start + CH), loaded a chunk ahead.
    auto load_chunk = [&](uint32_t (&dw)[NDW], uint32_t &mis, int k0) PBVD_INLINE_LAMBDA {
        const int t0 = k0 - start;
        const uint8_t *p = in + (int64_t)t0 * R;
        mis = (uint32_t)((uintptr_t)p & 3u);
        const uint8_t *pa = p - mis;
        if (len > 0 && pa >= a.syms && pa + 4 * NDW <= a.in_end) {
            const uint32_t *w32 = reinterpret_cast<const uint32_t *>(pa);
#pragma unroll
            for (int i = 0; i < NDW; ++i) dw[i] = w32[i];
        } else {
            // a chunk at either end of the buffer (bytes outside read as 0)
#pragma unroll
            for (int i = 0; i < NDW; ++i) {
                uint32_t v = 0;
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) {
                    const uint8_t *pb = pa + 4 * i + bb;
                    if (len > 0 && pb >= a.syms && pb < a.in_end) v |= (uint32_t)*pb << (8 * bb);
                }
                dw[i] = v;
            }
        }
    };
    uint32_t spw = 0;
    uint32_t dwn[NDW], misn;
    load_chunk(dwn, misn, 0);
    for (int k0 = 0; k0 < max_len; k0 += CH) {
        // byte i*R + r of q_[] is symbol r of the PB's stage k0 + i - start
        uint32_t q_[NDW - 1];
#pragma unroll
        for (int i = 0; i < NDW - 1; ++i) {
            uint32_t v = __builtin_amdgcn_alignbyte(dwn[i + 1], dwn[i], misn);
            if (hard) v = 0x01010101u + (v & 0x01010101u) * 0xfeu;  // bit -> +1 / -1
            q_[i] = v;
        }
        if (k0 + CH < max_len) load_chunk(dwn, misn, k0 + CH);
        static_for<0, CH>([&](auto ic) PBVD_INLINE_LAMBDA {
            constexpr int i = decltype(ic)::value;
            const int k = k0 + i;
            if (k >= max_len) return false;
            constexpr int BYTE = i * R;
            const uint32_t q = __builtin_amdgcn_alignbyte(q_[BYTE / 4 + 1], q_[BYTE / 4], BYTE % 4);
            const int bm_al = __builtin_amdgcn_sdot4((int)q, (int)m_al, 0, false);
            const int bm_be = __builtin_amdgcn_sdot4((int)q, (int)m_be, 0, false);
            const int bm_ga = __builtin_amdgcn_sdot4((int)q, (int)m_ga, 0, false);
            const int bm_th = __builtin_amdgcn_sdot4((int)q, (int)m_th, 0, false);
            // stage k reads buffer k & 1 (k0 is even: i & 1) and writes the other
            const int32_t *pin = lds + (i & 1) * ROW;
            int32_t *pout = lds + ((i + 1) & 1) * ROW;
            // SLOW: some PB of the tile has not started (its metrics stay at
            // their initial values)
            auto butterflies = [&](auto slow_c) PBVD_INLINE_LAMBDA {
                constexpr bool SLOW = decltype(slow_c)::value;
                const bool act = k >= start;
                // every predecessor metric first (one wait), then the
                // butterflies and their writes
                int32_t p1[B], p2[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    p1[b] = pin[rd[b]];
                    p2[b] = pin[rd[b] + kTilePbs];
                }
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int32_t x0 = p1[b] + bm_al, y0 = p2[b] + bm_ga;
                    const int32_t x1 = p1[b] + bm_be, y1 = p2[b] + bm_th;
                    spw = __builtin_amdgcn_alignbit(spw, (uint32_t)(y0 - x0), 31);
                    spw = __builtin_amdgcn_alignbit(spw, (uint32_t)(y1 - x1), 31);
                    int32_t n0 = min(x0, y0), n1 = min(x1, y1);
                    if constexpr (SLOW) {
                        n0 = act ? n0 : init_lo[b];
                        n1 = act ? n1 : init_hi[b];
                    }
                    pout[wr[b]] = n0;
                    pout[wr[b] + HALF * kTilePbs] = n1;
                }
            };
            if (k < max_start)
                butterflies(std::integral_constant<bool, true>{});
            else
                butterflies(std::integral_constant<bool, false>{});
            if ((k + 1) % SPD == 0 || k + 1 == max_len) {
                const int m = k / SPD;
                const int used = k % SPD + 1;   // stages in this dword
                const uint32_t v = used == SPD ? spw : spw << ((SPD - used) * WB);
                sp_tile[((int64_t)m * kTilePbs + lane) * NC + w] = v;
                spw = 0;
            }
            lds_barrier();
            return true;
        });
    }
    // the survivor stores of every wave are visible to wave 0 after a full
    // workgroup barrier
    __syncthreads();

    if (w != 0) return;

    // ---- final metrics and traceback start (Sec. III-A; Sec. II at the end
    //      of an unterminated stream) ----
    const int32_t *fin = lds + (max_len & 1) * ROW;
    uint32_t S = 0;
    const bool want_pm = a.final_pm != nullptr && pb_row >= 0;
    if (__builtin_amdgcn_readfirstlane(__ballot((argmin || want_pm) && len > 0) != 0 ? 1 : 0)) {
        int32_t m = 0x7fffffff;
        int best = 0;
        for (int s = 0; s < N; ++s) {
            const int32_t v = fin[s * kTilePbs + lane];
            if (v < m) {
                m = v;
                best = s;
            }
        }
        if (argmin) S = (uint32_t)best;
        if (want_pm)
            for (int s = 0; s < N; ++s) a.final_pm[pb_row * N + s] = fin[s * kTilePbs + lane] - m;
    }

    // ---- traceback (Alg. 1, Kernel 2) ----
    const int n_dec = dec_end - store0;
    const int k_lo = len > 0 ? start + store0 : max_len;   // this PB's last traced step
    const int k_out = start + dec_end;                      // steps below it are decoded
    const int k_bot = wave_min_i(k_lo);
    uint32_t cw = 0;
    auto flush = [&](int wi) PBVD_INLINE_LAMBDA {
        const int rel = wi * 32;
        const int nb = n_dec - rel < 32 ? n_dec - rel : 32;
        const int64_t bitpos = out_bit0 + rel;
        if (a.out_mode == kOutDirect) {
            const int64_t byte = bitpos >> 3;
            if (nb == 32 && byte + 4 <= a.out_bytes) {
                *reinterpret_cast<uint32_t *>(a.out + byte) = cw;
            } else {
                for (int bb = 0; bb < ((nb + 7) >> 3); ++bb)
                    if (byte + bb < a.out_bytes) a.out[byte + bb] = (uint8_t)(cw >> (8 * bb));
            }
        } else if (a.out_mode == kOutAtomic) {
            const uint32_t shf = (uint32_t)(bitpos & 31);
            uint32_t *wp = a.out_words + (bitpos >> 5);
            atomicOr(wp, cw << shf);
            if (shf && (cw >> (32 - shf))) atomicOr(wp + 1, cw >> (32 - shf));
        } else {
            uint8_t *ob = a.out + (bitpos >> 3);
            for (int bb = 0; bb < ((nb + 7) >> 3); ++bb) ob[bb] = (uint8_t)(cw >> (8 * bb));
        }
    };

    // rows of survivor dwords, a ring of RING dwords of stages ahead
    constexpr int RING = NC <= 4 ? 8 : 4;
    uint32_t ring[RING][NC];
    const int m_top = (max_len - 1) / SPD;
    const int m_bot = k_bot / SPD;
    auto load_row = [&](uint32_t (&dst)[NC], int m) PBVD_INLINE_LAMBDA {
        m = m < m_bot ? m_bot : m;
        const uint32_t *p = sp_tile + ((int64_t)m * kTilePbs + lane) * NC;
#pragma unroll
        for (int g = 0; g < NC; ++g) dst[g] = p[g];
    };
    static_for<0, RING - 1>([&](auto dc) PBVD_INLINE_LAMBDA {
        load_row(ring[decltype(dc)::value], m_top - decltype(dc)::value);
        return true;
    });
    int m = m_top;
    for (;;) {
        const bool more = static_for<0, RING>([&](auto dc) PBVD_INLINE_LAMBDA {
            constexpr int d = decltype(dc)::value;
            load_row(ring[(d + RING - 1) % RING], m - (RING - 1));
            const uint32_t(&row)[NC] = ring[d];
            static_for<0, SPD>([&](auto ic) PBVD_INLINE_LAMBDA {
                constexpr int i = SPD - 1 - decltype(ic)::value;   // stage i of the dword, top down
                const int k = m * SPD + i;
                if (k < max_len && k >= k_lo) {
                    const uint32_t bp = tt[S];
                    const uint32_t g = bp / WB, pos = bp % WB;
                    // the bit at that position of every group's word, then
                    // group g's (no select of a register by a lane's index)
                    const uint32_t sh = 31u - ((uint32_t)(i * WB) + pos);
                    uint32_t cand = 0;
#pragma unroll
                    for (int gg = 0; gg < NC; ++gg) cand |= ((row[gg] >> sh) & 1u) << gg;
                    const uint32_t dec = (cand >> g) & 1u;
                    if (k < k_out) {
                        const int rel = k - start - store0;
                        cw |= (S >> (V - 1)) << (rel & 31);
                        if ((rel & 31) == 0) {
                            flush(rel >> 5);
                            cw = 0;
                        }
                    }
                    S = ((S & (HALF - 1)) << 1) | dec;
                }
                return true;
            });
            if (m <= m_bot) return false;
            --m;
            return true;
        });
        if (!more) break;
    }
}

}  // namespace group
}  // namespace pbvd
