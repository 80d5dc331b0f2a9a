// Forward add-compare-select, survivor packing and traceback of the parallel
// block-based Viterbi decoder (arXiv 1608.00066, Sec. III-A), written for
// gfx950 wave64.
//
// Mapping: one lane decodes one parallel block (PB); one wave decodes 64 PBs
// that share a geometry, so every loop bound, phase and branch below is
// wave-uniform.  All N = 2^(K-1) path metrics of a lane live in VGPRs as
// N/2 packed pairs; the butterfly of Sec. III-B is done in place, which
// rotates the state <-> register assignment by one bit per stage and brings
// it back to the identity after K-1 stages (the unroll length).
//
// State <-> register map at phase ph (ph = stage index mod (K-1)):
//   u = rotl_{K-1}(state, ph); register = u mod N/2; half = u >> (K-2).
// A stage at phase ph < K-2 pairs register X (bit ph clear) with
// Y = X | 2^ph: X holds the even predecessors S_2j, Y the odd ones S_2j+1;
// the two new metrics for input 0 go back into X, those for input 1 into Y.
// At phase K-2 a register holds S_2j and S_2j+1 itself and is updated with
// half-broadcast operands.
//
// Branch metrics: only the 2^R distinct code-word metrics of a stage are
// computed (Sec. III-B, Eq. 3-6: every branch of a butterfly is alpha,
// beta, gamma or theta).  They are taken as sum_{r: c_r = 1} q_r, which
// differs from the mismatch distance by a constant shared by all code words
// of the stage; decisions and metric differences are therefore unchanged.
//
// Survivors: one bit per state and stage, 1 = lower branch (Sec. IV-B);
// bit position = register slot (+16 for the upper half of the pair).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

// Lambdas on the hot path are forced inline so that the arrays they capture
// stay in registers.
#define PBVD_INLINE_LAMBDA __attribute__((always_inline))

namespace pbvd {

constexpr int kWave = 64;

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E), until
// f returns false.  Returns false if it stopped early.
template <int B, int E, class F>
__device__ __forceinline__ bool static_for(F &&f) {
    if constexpr (B < E) {
        if (!f(std::integral_constant<int, B>{})) return false;
        return static_for<B + 1, E>(f);
    } else {
        return true;
    }
}

// Traceback row blocks kept in flight (a ring; all but one are loaded ahead).
#ifndef PBVD_TRACEBACK_BLOCKS
#define PBVD_TRACEBACK_BLOCKS 3
#endif
// VGPRs per lane for the row ring of the phase-aligned traceback (waves with
// one geometry): its steps are a few dependent ALU operations, so the ring is
// made as deep as this allows (the path metrics are dead by then).
#ifndef PBVD_TRACEBACK_RING_VGPRS
#define PBVD_TRACEBACK_RING_VGPRS 48
#endif

struct KernelArgs {
    const uint8_t *syms;    // T*R received symbols, stage-major
    uint8_t *out;           // packed decoded bits (direct path)
    uint32_t *out_words;    // zeroed word buffer (atomic path) or null
    int32_t *final_pm;      // [pb_count][N] normalized final metrics or null
    uint32_t *sp;           // survivor scratch, sp_wave_dwords per wave slot
    int64_t n;              // information bits of the stream
    int64_t T;              // trellis stages (n + K-1 when terminated)
    int64_t pb_first;       // first PB of this call
    int64_t b_lo, b_hi;     // interior PBs (full geometry) of this call
    int64_t n_head;         // edge PBs [pb_first, pb_first + n_head) precede b_lo
    int64_t n_fold;         // edge PBs placed in the first wave's leading slots
    int64_t n_int_waves;    // waves covering n_fold + (b_hi - b_lo) slots, 64 >> LB PBs each
    int64_t wave_begin;     // first wave (interior waves first, then edge waves)
    int64_t n_waves;        // waves in this launch
    int64_t out_bytes;      // bytes of `out`
    int64_t sp_wave_dwords; // survivor dwords per wave slot
    int32_t D, L;
    int32_t terminated;
    int32_t direct_out;     // 1: plain stores into out, 0: atomic OR into out_words
    int32_t fold_i_safe;    // first wave with folded PBs: last trip start whose wide fetch is in bounds
    int32_t fold_wide;      // first wave with folded PBs: every wide fetch is in bounds
};

// Place of PB b in the stream kernel's waves.  Edge PBs (clipped geometry at
// the stream ends) are numbered stream-start PBs first, then stream-end PBs;
// the first n_fold of them take the leading slots of wave 0, the interior PBs
// fill the slots after them 64 >> LB to a wave, and every other edge PB gets
// a wave of its own after the interior waves (slot 0).
struct WavePlace {
    int64_t wave;
    int slot;
};
__host__ __device__ inline WavePlace wave_place(int64_t b, int64_t pb_first, int64_t b_lo, int64_t b_hi,
                                                int64_t n_head, int64_t n_fold, int64_t n_int_waves, int pw) {
    if (b >= b_lo && b < b_hi) {
        const int64_t s = n_fold + (b - b_lo);
        return {s / pw, (int)(s % pw)};
    }
    const int64_t e = b < b_lo ? b - pb_first : n_head + (b - b_hi);
    if (e < n_fold) return {0, (int)e};
    return {n_int_waves + (e - n_fold), 0};
}

// ---------------------------------------------------------------------------
// Code description (compile-time generators)
// ---------------------------------------------------------------------------
template <int K_, int R_, uint32_t G0, uint32_t G1, uint32_t G2 = 0, uint32_t G3 = 0>
struct FixedCode {
    static constexpr int K = K_;
    static constexpr int R = R_;
    static constexpr int V = K - 1;       // memory cells
    static constexpr int N = 1 << V;      // states
    static constexpr int NR = N / 2;      // packed registers
    static constexpr int NC = 1 << R;     // code words
    static constexpr uint32_t gen(int r) { return r == 0 ? G0 : r == 1 ? G1 : r == 2 ? G2 : G3; }
    // Code word (c^(1) as MSB) contributed by register bit k (k = K-1: input).
    static constexpr int gcol(int k) {
        int c = 0;
        for (int r = 0; r < R; ++r) c = (c << 1) | (int)((gen(r) >> k) & 1u);
        return c;
    }
    // Encoder output c(S_d, 0) of Eq. 2.
    static constexpr int out0(int d) {
        int c = 0;
        for (int k = 0; k < V; ++k)
            if ((d >> k) & 1) c ^= gcol(k);
        return c;
    }
};

template <int V>
__host__ __device__ constexpr int rotr_v(int u, int s) {
    return s == 0 ? u : (((u >> s) | (u << (V - s))) & ((1 << V) - 1));
}
template <int V>
__host__ __device__ constexpr int rotl_v(int u, int s) {
    return rotr_v<V>(u, (V - s) % V);
}

// Survivor bit layout of one stage.  The decision of the state whose
// rotated index is u (register r = u mod N/2, half h = u >> (K-2)) sits at a
// bit position obtained by moving each bit t of u to ubit_pos(t):
//   shift layout (BP = false): dword r >> 4, bit (r & 15) + 16 h;
//   byte-permute layout (BP = true, 16-bit metrics, N >= 32): dword r >> 4,
//     bit 16 (r & 1) + 8 h + ((r & 15) >> 1) -- the sign bytes of two
//     registers' differences are gathered with one v_perm_b32 and eight
//     such words are merged per dword.
// Several stages share a dword when N < 32 (shift layout only).
template <int V, bool BP>
__host__ __device__ constexpr int ubit_pos(int t) {
    if (BP) return t == 0 ? 4 : (t < 4 ? t - 1 : (t == V - 1 ? 3 : t + 1));
    return t == V - 1 ? 4 : (t < 4 ? t : t + 1);
}
template <int V, bool BP>
__device__ __forceinline__ uint32_t u_to_idx(uint32_t u) {
    uint32_t idx = 0;
#pragma unroll
    for (int t = 0; t < V; ++t) idx |= ((u >> t) & 1u) << ubit_pos<V, BP>(t);
    return idx;
}

// ---------------------------------------------------------------------------
// Packed path-metric pairs
// on-lanes of a wave-constant lane pattern take b, the others a: one
// v_cndmask_b32 with the pattern in a scalar register pair
__device__ __forceinline__ int select_lanes(int a, int b, uint64_t pattern) {
    int r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(pattern));
    return r;
}

// Value of v in another lane of the same quad (DPP quad_perm control CTRL).
template <int CTRL>
__device__ __forceinline__ int dpp_int(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}

// ---------------------------------------------------------------------------
struct PM16 {
    typedef short v2 __attribute__((ext_vector_type(2)));
    typedef unsigned short v2u __attribute__((ext_vector_type(2)));
    using T = v2;
    static constexpr int kLimit = 32767;
    static __device__ __forceinline__ T make(int lo, int hi) { return T{(short)lo, (short)hi}; }
    static __device__ __forceinline__ T add(T a, T b) {
        return __builtin_bit_cast(T, __builtin_bit_cast(v2u, a) + __builtin_bit_cast(v2u, b));
    }
    static __device__ __forceinline__ T sub(T a, T b) {
        return __builtin_bit_cast(T, __builtin_bit_cast(v2u, a) - __builtin_bit_cast(v2u, b));
    }
    static __device__ __forceinline__ T vmin(T a, T b) { return __builtin_elementwise_min(a, b); }
    static __device__ __forceinline__ T bcast_lo(T a) { return a.xx; }
    static __device__ __forceinline__ T bcast_hi(T a) { return a.yy; }
    // sign of (b - a) of each half at bits 0 and 16: 1 = b strictly smaller
    static __device__ __forceinline__ uint32_t dec(T a, T b) {
        v2u d = __builtin_bit_cast(v2u, sub(b, a));
        d = d >> (v2u){15, 15};
        return __builtin_bit_cast(uint32_t, d);
    }
    // raw b - a of both halves: their sign bits are bits 15 and 31
    static __device__ __forceinline__ uint32_t diff(T a, T b) {
        return __builtin_bit_cast(uint32_t, sub(b, a));
    }
    static __device__ __forceinline__ int lo(T a) { return a.x; }
    static __device__ __forceinline__ int hi(T a) { return a.y; }
    template <int CTRL>
    static __device__ __forceinline__ T dpp(T a) {
        return __builtin_bit_cast(T, dpp_int<CTRL>(__builtin_bit_cast(int, a)));
    }
    template <class F>
    static __device__ __forceinline__ T each(T a, F f) {
        return __builtin_bit_cast(T, f(__builtin_bit_cast(int, a)));
    }
};

struct PM32 {
    struct T { int x, y; };
    static constexpr int kLimit = 0x7fffffff;
    static __device__ __forceinline__ T make(int lo, int hi) { return T{lo, hi}; }
    static __device__ __forceinline__ T add(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
    static __device__ __forceinline__ T sub(T a, T b) { return T{a.x - b.x, a.y - b.y}; }
    static __device__ __forceinline__ T vmin(T a, T b) { return T{a.x < b.x ? a.x : b.x, a.y < b.y ? a.y : b.y}; }
    static __device__ __forceinline__ T bcast_lo(T a) { return T{a.x, a.x}; }
    static __device__ __forceinline__ T bcast_hi(T a) { return T{a.y, a.y}; }
    static __device__ __forceinline__ uint32_t dec(T a, T b) {
        return ((uint32_t)(b.x - a.x) >> 31) | (((uint32_t)(b.y - a.y) >> 31) << 16);
    }
    static __device__ __forceinline__ int lo(T a) { return a.x; }
    static __device__ __forceinline__ int hi(T a) { return a.y; }
    template <int CTRL>
    static __device__ __forceinline__ T dpp(T a) { return T{dpp_int<CTRL>(a.x), dpp_int<CTRL>(a.y)}; }
    template <class F>
    static __device__ __forceinline__ T each(T a, F f) { return T{f(a.x), f(a.y)}; }
};

// acc | (x << SH) as one v_lshl_or_b32.  Written out so that the compiler
// keeps one instruction per inserted decision pair instead of rebuilding the
// OR chain as a shift-and-or tree.
template <int SH>
__device__ __forceinline__ uint32_t shl_or(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_lshl_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "n"(SH), "v"(acc));
    return r;
}

// acc | (x & mask) as one v_and_or_b32 (mask in an SGPR).
__device__ __forceinline__ uint32_t and_or(uint32_t x, uint32_t mask, uint32_t acc) {
    uint32_t r;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "s"(mask), "v"(acc));
    return r;
}

// Survivor rows of one wave slot, addressed through a buffer resource: the
// row offset is wave-uniform (SGPR), the lane offset a loop-invariant VGPR,
// so no per-stage address arithmetic runs on the vector unit.
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBufferFlags = 0x00020000;  // raw 32-bit data format (gfx9 family)
// Cache policy of survivor rows: non-temporal.  A row is written once and
// read once by the traceback, long after it has left the L2, so it should not
// evict the input symbols that the next loop trips of the same lanes read
// again (measured: 2.47 -> 1.93 GB fetched per 2^27-bit K=7 launch).
constexpr int kRowPolicy = 2;  // nt

// A lane moves NDW dwords of a row; consecutive rows are ROW_DW dwords apart
// (64 lanes x their own dwords when every lane stores its part).  Stores move
// at most 8 bytes per lane: the vector memory unit reads the data registers
// of a wider store over several cycles after it issues, and an instruction
// that overwrites them too soon (which the compiler does not always prevent)
// changes what the last lanes store.  8-byte stores have no such window.
template <int NDW, int ROW_DW = kWave * NDW>
struct RowStore {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t lane_off;  // bytes
    static constexpr int kRowBytes = ROW_DW * 4;
    __device__ __forceinline__ void store(int row, const uint32_t (&v)[NDW]) const {
        const int so = row * kRowBytes;
        if constexpr (NDW == 1) {
            __builtin_amdgcn_raw_buffer_store_b32(v[0], rsrc, lane_off, so, kRowPolicy);
        } else {
#pragma unroll
            for (int w = 0; w < NDW; w += 2)
                __builtin_amdgcn_raw_buffer_store_b64(u32x2{v[w], v[w + 1]}, rsrc, lane_off + 4 * w, so,
                                                      kRowPolicy);
        }
    }
    __device__ __forceinline__ void load(int row, uint32_t (&v)[NDW]) const {
        const int so = row * kRowBytes;
        if constexpr (NDW == 1) {
            v[0] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, lane_off, so, kRowPolicy);
        } else if constexpr (NDW == 2) {
            const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(rsrc, lane_off, so, kRowPolicy);
            v[0] = t.x;
            v[1] = t.y;
        } else {
#pragma unroll
            for (int w = 0; w < NDW; w += 4) {
                const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(rsrc, lane_off + 4 * w, so, kRowPolicy);
                v[w] = t.x;
                v[w + 1] = t.y;
                v[w + 2] = t.z;
                v[w + 3] = t.w;
            }
        }
    }
};

enum { kSoftI8 = 0, kHardU8 = 1 };

template <int KIND>
__device__ __forceinline__ int rx_value(const uint8_t *p) {
    if constexpr (KIND == kHardU8) return 1 - 2 * (int)(*p & 1u);
    else return (int)(int8_t)*p;
}

// The 2^R distinct branch metrics of one stage (Sec. III-B: every branch
// carries one of the 2^R code words): metric(c) = sum over r with c^(r) = 1
// of q_r.  The Sec. II distance sum_r [c^(r) != (q_r < 0)] |q_r| equals this
// plus sum_r max(-q_r, 0), which is the same for every c.
template <int R>
__device__ __forceinline__ void code_word_metrics(const int (&q)[R], int (&bm)[1 << R], int base = 0) {
#pragma unroll
    for (int c = 0; c < (1 << R); ++c) {
        int s = base;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if ((c >> (R - 1 - r)) & 1) s += q[r];
        bm[c] = s;
    }
}

// ---------------------------------------------------------------------------
// Lanes per PB.  With 2^LB lanes per PB (LB = 1 or 2) the registers of a PB
// are spread over a group of consecutive lanes: lane l of the group holds the
// states whose register index has l in its top LB bits.  Stages whose
// butterfly pairs registers of different lanes read the partner's metrics
// with a DPP quad permute; every lane keeps its own half of each pair.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int quad_sel(int a, int b, int c, int d) { return a | (b << 2) | (c << 4) | (d << 6); }
// quad-permute controls: read the lane of the group with lane bit B cleared /
// set, flip lane bit 0 / 1, or read the group's first lane
template <int B> __host__ __device__ constexpr int quad_lo() { return B == 0 ? quad_sel(0, 0, 2, 2) : quad_sel(0, 1, 0, 1); }
template <int B> __host__ __device__ constexpr int quad_hi() { return B == 0 ? quad_sel(1, 1, 3, 3) : quad_sel(2, 3, 2, 3); }
template <int B> __host__ __device__ constexpr int quad_flip() { return B == 0 ? quad_sel(1, 0, 3, 2) : quad_sel(2, 3, 0, 1); }
template <int LB> __host__ __device__ constexpr int quad_first() { return LB == 1 ? quad_sel(0, 0, 2, 2) : quad_sel(0, 0, 0, 0); }
// Lane bit 2 (groups of 8) crosses quads: DPP row shifts by 4 inside a row of
// 16 lanes, written only to the banks (groups of 4 lanes) that need them.
constexpr int kRowShl4 = 0x104;  // lane l reads lane l + 4 of its row
constexpr int kRowShr4 = 0x114;  // lane l reads lane l - 4 of its row
// v of the lane with bit 2 cleared / set (lanes that are that lane keep v)
__device__ __forceinline__ int bit2_lo(int v) { return __builtin_amdgcn_update_dpp(v, v, kRowShr4, 0xf, 0xa, false); }
__device__ __forceinline__ int bit2_hi(int v) { return __builtin_amdgcn_update_dpp(v, v, kRowShl4, 0xf, 0x5, false); }
// v of the lane whose bit 2 differs
__device__ __forceinline__ int bit2_flip(int v) {
    const int t = __builtin_amdgcn_update_dpp(v, v, kRowShl4, 0xf, 0x5, false);
    return __builtin_amdgcn_update_dpp(t, v, kRowShr4, 0xf, 0xa, false);
}

// ---------------------------------------------------------------------------
// One trellis stage at compile-time phase PH on the NR >> LB registers of a
// lane, with the stage's branch metrics bm[] already relabeled for the lane
// (see lane_code_mask).  Writes the stage's decision bits into dw[] at slot
// offset SLOT0 (in units of packed registers) in the shift layout, or in the
// byte-permute layout when BP.
// ---------------------------------------------------------------------------
template <class C, class P, int PH, int SLOT0, int NDW, bool BP, int LB>
__device__ __forceinline__ void acs_stage(typename P::T (&pm)[C::NR >> LB], const int (&bm)[C::NC],
                                          uint32_t (&dw)[NDW]) {
    using T = typename P::T;
    constexpr int V = C::V, NR = C::NR >> LB, NC = C::NC;
    constexpr int G0 = C::gcol(0), GK = C::gcol(C::K - 1);
    constexpr int kCross = V - 1 - LB;  // first phase whose pair bit is a lane bit

    // decisions of register X (two per register: lower and upper half)
    uint32_t dd[NR];
    auto record = [&](auto xc, T a, T b) PBVD_INLINE_LAMBDA {
        constexpr int X = decltype(xc)::value;
        if constexpr (!BP) {
            constexpr int sx = SLOT0 + X;
            dw[sx >> 4] = shl_or<(sx & 15)>(P::dec(a, b), dw[sx >> 4]);
        } else {
            dd[X] = P::diff(a, b);
            if constexpr (X & 1) {
                // selectors 8..11 of v_perm_b32 replicate bits 15, 31, 47, 63
                // of {dd[X], dd[X-1]} over a byte: the four signs
                // [lo(X-1), hi(X-1), lo(X), hi(X)] as 0x00 / 0xff bytes, so
                // any bit of a byte can take the decision without a shift
                const uint32_t p = __builtin_amdgcn_perm(dd[X], dd[X - 1], 0x0b0a0908u);
                constexpr int kk = (X & 15) >> 1;
                dw[X >> 4] = and_or(p, 0x01010101u << kk, dw[X >> 4]);
            }
        }
    };

    if constexpr (PH < kCross) {
        // pairs (X, Y = X | 2^PH) inside the lane; halves differ in state bit V-1-PH
        constexpr int GP = C::gcol(V - 1 - PH);
        T pair[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) pair[c] = P::make(bm[c], bm[c ^ GP]);
        static_for<0, NR / 2>([&](auto kc) PBVD_INLINE_LAMBDA {
            constexpr int k = decltype(kc)::value;
            constexpr int X = ((k >> PH) << (PH + 1)) | (k & ((1 << PH) - 1));
            constexpr int Y = X | (1 << PH);
            constexpr int alpha = C::out0(rotr_v<V>(X, PH));  // c(S_2j, 0) of the lower half
            const T a0 = P::add(pm[X], pair[alpha]);
            const T b0 = P::add(pm[Y], pair[alpha ^ G0]);
            const T a1 = P::add(pm[X], pair[alpha ^ GK]);
            const T b1 = P::add(pm[Y], pair[alpha ^ G0 ^ GK]);
            pm[X] = P::vmin(a0, b0);
            pm[Y] = P::vmin(a1, b1);
            record(std::integral_constant<int, X>{}, a0, b0);
            record(std::integral_constant<int, Y>{}, a1, b1);
            return true;
        });
    } else if constexpr (PH < V - 1) {
        // the pair bit is lane bit B: register X of the group's lane with B
        // clear holds S_2j, the same register of the lane with B set holds
        // S_2j+1; each lane computes the new metrics it keeps (input 0 for B
        // clear, input 1 for B set, folded into its relabeled metrics)
        constexpr int B = PH - kCross;
        constexpr int GP = C::gcol(V - 1 - PH);
        T pair[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) pair[c] = P::make(bm[c], bm[c ^ GP]);
        static_for<0, NR>([&](auto xc) PBVD_INLINE_LAMBDA {
            constexpr int X = decltype(xc)::value;
            constexpr int alpha = C::out0(rotr_v<V>(X, PH));
            T xv, yv;
            if constexpr (B < 2) {
                xv = P::template dpp<quad_lo<B>()>(pm[X]);
                yv = P::template dpp<quad_hi<B>()>(pm[X]);
            } else {
                xv = P::each(pm[X], bit2_lo);
                yv = P::each(pm[X], bit2_hi);
            }
            const T a = P::add(xv, pair[alpha]);
            const T b = P::add(yv, pair[alpha ^ G0]);
            pm[X] = P::vmin(a, b);
            record(xc, a, b);
            return true;
        });
    } else {
        // each register holds (S_2j, S_2j+1): broadcast operands
        T pair[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) pair[c] = P::make(bm[c], bm[c ^ GK]);
        static_for<0, NR>([&](auto xc) PBVD_INLINE_LAMBDA {
            constexpr int X = decltype(xc)::value;
            constexpr int alpha = C::out0(2 * X);
            const T a = P::add(P::bcast_lo(pm[X]), pair[alpha]);
            const T b = P::add(P::bcast_hi(pm[X]), pair[alpha ^ G0]);
            pm[X] = P::vmin(a, b);
            record(xc, a, b);
            return true;
        });
    }
}

// Relabeling of the code words for lane bit j at phase PH.  The code word of
// a branch is linear (over GF(2)) in the state bits, so the lane bits add the
// same mask to every branch of a lane: the lane uses metric[c ^ mask] where
// the stage code above uses metric[c].  In a stage whose pair bit is lane
// bit j, the lane with that bit set computes the input-1 outputs, whose code
// words differ by g_{K-1} (Eq. 4, Eq. 6).
template <class C, int LB>
__host__ __device__ constexpr int lane_code_mask(int PH, int j) {
    constexpr int V = C::V;
    const int kCross = V - 1 - LB;
    if (PH >= kCross && PH < V - 1 && PH - kCross == j) return C::gcol(C::K - 1);
    return C::out0(rotr_v<V>(1 << (kCross + j), PH));
}

// ---------------------------------------------------------------------------
// Compile-time layout constants of one code
// ---------------------------------------------------------------------------
template <class C, class P, int LB = 0>
struct Layout {
    static constexpr int V = C::V;
    static constexpr int NR = C::NR >> LB;                // packed registers per lane
    static constexpr int GL = 1 << LB;                    // lanes per PB
    static constexpr int PW = kWave >> LB;                // PBs per wave
    static constexpr int NDW = NR >= 16 ? NR / 16 : 1;    // survivor dwords a lane stores per row
    static constexpr int NDW_F = NDW * GL;                // survivor dwords of one PB's row
    static constexpr int S = NR >= 16 ? 1 : 16 / NR;      // stages per stored row
    static constexpr int gcd(int a, int b) { return b == 0 ? a : gcd(b, a % b); }
    static constexpr int U = V / gcd(V, S) * S;           // unrolled stages per loop trip
    static constexpr bool kBytePerm = std::is_same<P, PM16>::value && NR >= 16;
    // a second, check-free copy of the loop trip only where it is small
    static constexpr bool kFastLoop = NR <= 32;
    // Largest metric spread: the known-state start (8192) plus K-1 stages of
    // the widest branch-metric difference (128 per symbol).  Between two
    // renormalizations every metric moves by at most 128*R per stage.
    static constexpr int kSpread = 8192 + V * 128 * C::R;
    static constexpr long long kMaxStages = ((long long)P::kLimit - kSpread) / (128LL * C::R);
    static constexpr int kRenormTrips =
        kMaxStages / U > (1 << 30) ? (1 << 30) : (int)(kMaxStages / U);
    static_assert(kRenormTrips >= 1, "metric range too small for this code");
    // a lane group must fill whole survivor dwords with the byte-permute
    // layout, so that a PB's row is the same bits as with one lane per PB
    static_assert(LB == 0 || (LB <= 3 && NR >= 16 && std::is_same<P, PM16>::value),
                  "lane groups need 16-bit metrics and at least 16 registers per lane");
};

// Lane groups a code supports (compile-time mirror of lanes_allowed on the host).
template <class C, class P, int LB>
__host__ __device__ constexpr bool lanes_supported() {
    return LB == 0 || (LB <= 3 && (C::NR >> LB) >= 16 && std::is_same<P, PM16>::value);
}

template <int V>
__device__ __forceinline__ int rotr_rt(int u, int s) {
    return ((u >> s) | (u << (V - s))) & ((1 << V) - 1);
}

// ---------------------------------------------------------------------------
// Decode body shared by the stream kernel and the batch (tile) kernel:
// forward ACS with survivor-row stores, final metrics, then traceback with
// packed output, for the 64 PBs of one wave.
// ---------------------------------------------------------------------------
enum { kOutDirect = 0, kOutAtomic = 1, kOutBytes = 2 };

struct WaveJob {
    // wave-uniform
    int len;             // forward stages the wave runs (the longest lane's)
    int store0_min;      // lowest first-traced stage over the lanes
    int i_safe;          // last trip start whose wide fetch is in bounds (-1: none)
    bool fetch_safe;     // every wide fetch of the wave stays in bounds
    bool need_final;     // some lane needs its final metrics
    int out_mode;        // kOutDirect / kOutAtomic / kOutBytes
    const uint8_t *in_end;
    uint8_t *out;
    int64_t out_bytes;   // kOutDirect bound
    uint32_t *out_words; // kOutAtomic staging
    // per lane
    const uint8_t *in;   // symbols of the lane's first forward stage
    int my_len, my_store0, my_dec_end;
    bool known;          // start from encoder state 0
    bool argmin;         // trace back from the least-metric state
    bool active;
    bool store0_uniform; // VARLEN: every lane's first traced stage is store0_min
    int64_t out_bit0;    // output bit position of the lane's first decoded bit
    int32_t *pm_out;     // final-metric row or null
};

// VARLEN: lanes may run fewer stages than the wave (batch tiles).  All lanes
// start at stage 0 with their own initial metrics; a lane's stages past its
// own end compute values nobody reads, and its traceback starts at its own
// last stage.
template <class C, class P, int KIND, bool VARLEN, int LB>
__device__ __forceinline__ void decode_body(const WaveJob &j, const RowStore<Layout<C, P, LB>::NDW> &rows) {
    using T = typename P::T;
    using LY = Layout<C, P, LB>;
    constexpr int V = C::V, N = C::N, NR = LY::NR, R = C::R, NC = C::NC;
    constexpr int NDW = LY::NDW, NDW_F = LY::NDW_F, S = LY::S, U = LY::U;
    const int len = j.len;
    const uint8_t *const in = j.in;
    // lane within the PB's group; its bits are the top register-index bits
    const int ell = LB ? (int)(threadIdx.x & ((1u << LB) - 1)) : 0;

    // ---- initial metrics ----
    T pm[NR];
    {
        // known start state 0 when the lane's forward range starts at stage 0
        const int big = j.known ? 8192 : 0;
        const int zero = ell == 0 ? 0 : big;
#pragma unroll
        for (int r = 0; r < NR; ++r) pm[r] = P::make(r == 0 ? zero : big, big);
    }
    // branch metrics of stage phase PH for this lane: metric[c ^ mask], the
    // mask being the XOR of the masks of the lane's set group bits; lane
    // bit j of the group is set in the wave-constant lane pattern kBit[j]
    constexpr uint64_t kBit[3] = {0xaaaaaaaaaaaaaaaaull, 0xccccccccccccccccull, 0xf0f0f0f0f0f0f0f0ull};
    auto stage_metrics = [&](auto phc, int (&q)[R], int (&bm)[NC]) PBVD_INLINE_LAMBDA {
        constexpr int PH = decltype(phc)::value;
        code_word_metrics<R>(q, bm);
        auto relabel = [&](auto mc, auto jc) PBVD_INLINE_LAMBDA {
            constexpr int M = decltype(mc)::value;
            if constexpr (M != 0) {
                int t[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) t[c] = select_lanes(bm[c], bm[c ^ M], kBit[decltype(jc)::value]);
#pragma unroll
                for (int c = 0; c < NC; ++c) bm[c] = t[c];
            }
        };
        if constexpr (LB >= 1)
            relabel(std::integral_constant<int, lane_code_mask<C, LB>(PH, 0)>{}, std::integral_constant<int, 0>{});
        if constexpr (LB >= 2)
            relabel(std::integral_constant<int, lane_code_mask<C, LB>(PH, 1)>{}, std::integral_constant<int, 1>{});
        if constexpr (LB >= 3)
            relabel(std::integral_constant<int, lane_code_mask<C, LB>(PH, 2)>{}, std::integral_constant<int, 2>{});
    };
    // renormalization reference: the group's first lane's metric of register 0
    auto renorm = [&]() PBVD_INLINE_LAMBDA {
        T ref = P::bcast_lo(pm[0]);
        if constexpr (LB > 0) ref = P::template dpp<quad_first<LB>()>(ref);
        if constexpr (LB > 2) ref = P::each(ref, bit2_lo);
#pragma unroll
        for (int r = 0; r < NR; ++r) pm[r] = P::sub(pm[r], ref);
    };

    // ---- forward procedure ----
    // Received symbols of one loop trip (U stages, NB bytes) are fetched with
    // one wide dword-aligned load per lane a trip ahead of their use, then
    // shifted into place (each lane's block starts at its own byte offset).
    // Only a window that would run past the end of the input falls back to
    // byte loads.
    constexpr int NB = U * R;
    constexpr int NW = (NB + 3) / 4;   // dwords holding the trip's symbols
    constexpr int ND = NW + 1;         // dwords fetched (unaligned start)
    const uint8_t *const in_end = j.in_end;
    // a lane never fetches past its own last trip
    const int my_last_trip = VARLEN ? ((j.my_len - 1) / U) * U : 0;
    // when a trip spans whole dwords the lane's misalignment never changes
    const uint32_t mis0 = (uint32_t)((uintptr_t)in & 3u);
    const uint8_t *const in_aligned = in - mis0;  // keeps the global address space
    auto fetch = [&](uint32_t (&raw)[ND], uint32_t &sh, int i0, bool wide) PBVD_INLINE_LAMBDA {
        if constexpr (VARLEN) i0 = i0 < my_last_trip ? i0 : my_last_trip;
        const uint8_t *p = in + (int64_t)i0 * R;
        uint32_t mis;
        const uint8_t *pa;
        if constexpr (NB % 4 == 0) {
            mis = mis0;
            pa = in_aligned + (int64_t)i0 * R;
        } else {
            mis = (uint32_t)((uintptr_t)p & 3u);
            pa = p - mis;
        }
        sh = mis * 8u;
        if (wide) {
            const uint32_t *q = reinterpret_cast<const uint32_t *>(pa);
#pragma unroll
            for (int jj = 0; jj < ND; ++jj) raw[jj] = q[jj];
        } else {
#pragma unroll
            for (int jj = 0; jj < ND; ++jj) {
                uint32_t v = 0;
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) {
                    const uint8_t *c = pa + 4 * jj + bb;
                    if (c >= p && c < in_end) v |= (uint32_t)*c << (8 * bb);
                }
                raw[jj] = v;
            }
        }
    };
    auto align_trip = [&](const uint32_t (&raw)[ND], uint32_t sh, uint32_t (&w)[NW]) PBVD_INLINE_LAMBDA {
#pragma unroll
        for (int jj = 0; jj < NW; ++jj)
            w[jj] = (uint32_t)(((uint64_t)raw[jj + 1] << 32 | raw[jj]) >> sh);
    };
    auto symbols = [&](const uint32_t (&w)[NW], int k, int (&q)[R]) PBVD_INLINE_LAMBDA {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int t = k * R + r;
            const uint32_t byte = (w[t >> 2] >> (8 * (t & 3))) & 0xffu;
            if constexpr (KIND == kHardU8) q[r] = 1 - 2 * (int)(byte & 1u);
            else q[r] = (int)(int8_t)byte;
        }
    };
    uint32_t raw_next[ND], sh_next, wsym[NW];
    {
        uint32_t raw0[ND], sh0;
        fetch(raw0, sh0, 0, j.fetch_safe);
        align_trip(raw0, sh0, wsym);
    }
    uint32_t dw[NDW];
#pragma unroll
    for (int w = 0; w < NDW; ++w) dw[w] = 0;
    int trips_since_renorm = 0;
    int i0 = 0;
    // Straight-line trips: whole trips whose next fetch is in bounds need no
    // per-stage checks; the generic loop below finishes the block.
    const int fast_end = len - U < j.i_safe - U ? len - U : j.i_safe - U;
    // Trips that lie wholly before the lowest traced stage (the L warm-up
    // stages of Sec. III-A) store no rows: the traceback never reads them,
    // so their decision bits are not even formed.
    const int warm_end = j.store0_min / U * U < fast_end ? j.store0_min / U * U : fast_end;
    for (; i0 < warm_end; i0 += U) {
        fetch(raw_next, sh_next, i0 + U, true);
        if (++trips_since_renorm == LY::kRenormTrips) {
            trips_since_renorm = 0;
            renorm();
        }
        static_for<0, U>([&](auto kc) PBVD_INLINE_LAMBDA {
            constexpr int k = decltype(kc)::value;
            int q[R], bm[NC];
            symbols(wsym, k, q);
            stage_metrics(std::integral_constant<int, k % V>{}, q, bm);
            acs_stage<C, P, k % V, (k % S) * NR, NDW, LY::kBytePerm, LB>(pm, bm, dw);
            if constexpr ((k % S) == S - 1) {
#pragma unroll
                for (int w = 0; w < NDW; ++w) dw[w] = 0;
            }
            return true;
        });
        align_trip(raw_next, sh_next, wsym);
    }
    if constexpr (LY::kFastLoop) {
        for (; i0 < fast_end; i0 += U) {
            fetch(raw_next, sh_next, i0 + U, true);
            if (++trips_since_renorm == LY::kRenormTrips) {
                trips_since_renorm = 0;
                renorm();
            }
            static_for<0, U>([&](auto kc) PBVD_INLINE_LAMBDA {
                constexpr int k = decltype(kc)::value;
                int q[R], bm[NC];
                symbols(wsym, k, q);
                stage_metrics(std::integral_constant<int, k % V>{}, q, bm);
                acs_stage<C, P, k % V, (k % S) * NR, NDW, LY::kBytePerm, LB>(pm, bm, dw);
                if constexpr ((k % S) == S - 1) {
                    rows.store((i0 + k) / S, dw);
#pragma unroll
                    for (int w = 0; w < NDW; ++w) dw[w] = 0;
                }
                return true;
            });
            align_trip(raw_next, sh_next, wsym);
        }
    }
    for (;; i0 += U) {
        const bool last_trip = i0 + U >= len;
        if (!last_trip) fetch(raw_next, sh_next, i0 + U, j.fetch_safe);
        if (++trips_since_renorm == LY::kRenormTrips) {
            trips_since_renorm = 0;
            renorm();
        }
        const bool more = static_for<0, U>([&](auto kc) PBVD_INLINE_LAMBDA {
            constexpr int k = decltype(kc)::value;
            if (i0 + k >= len) return false;
            int q[R], bm[NC];
            symbols(wsym, k, q);
            stage_metrics(std::integral_constant<int, k % V>{}, q, bm);
            acs_stage<C, P, k % V, (k % S) * NR, NDW, LY::kBytePerm, LB>(pm, bm, dw);
            if ((k % S) == S - 1 || i0 + k + 1 == len) {
                rows.store((i0 + k) / S, dw);
#pragma unroll
                for (int w = 0; w < NDW; ++w) dw[w] = 0;
            }
            return true;
        });
        if (!more || last_trip) break;
        align_trip(raw_next, sh_next, wsym);
    }

    // ---- final metrics and traceback start (Sec. III-A; Sec. II at an
    //      unterminated stream end) ----
    const int ph_end = len % V;
    uint32_t idx = 0;  // rotated index of state 0 is 0
    if (j.need_final) {
        // rotated index of this lane's register r: u = r | ell << (K-2-LB),
        // plus 2^(K-2) for the upper half
        const int ubase = ell << (V - 1 - LB);
        int m = 0x7fffffff;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            m = min(m, P::lo(pm[r]));
            m = min(m, P::hi(pm[r]));
        }
        if constexpr (LB >= 1) m = min(m, dpp_int<quad_flip<0>()>(m));
        if constexpr (LB >= 2) m = min(m, dpp_int<quad_flip<1>()>(m));
        if constexpr (LB >= 3) m = min(m, bit2_flip(m));
        if (j.argmin) {
            int best = N;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int s_lo = rotr_rt<V>(ubase | r, ph_end);
                const int s_hi = rotr_rt<V>(ubase | r | (1 << (V - 1)), ph_end);
                if (P::lo(pm[r]) == m && s_lo < best) best = s_lo;
                if (P::hi(pm[r]) == m && s_hi < best) best = s_hi;
            }
            if constexpr (LB >= 1) best = min(best, dpp_int<quad_flip<0>()>(best));
            if constexpr (LB >= 2) best = min(best, dpp_int<quad_flip<1>()>(best));
            if constexpr (LB >= 3) best = min(best, bit2_flip(best));
            idx = u_to_idx<V, LY::kBytePerm>((uint32_t)rotr_rt<V>(best, (V - ph_end) % V));
        }
        if (j.pm_out && j.active) {
            int32_t *fp = j.pm_out;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                fp[rotr_rt<V>(ubase | r, ph_end)] = P::lo(pm[r]) - m;
                fp[rotr_rt<V>(ubase | r | (1 << (V - 1)), ph_end)] = P::hi(pm[r]) - m;
            }
        }
    }

    // ---- traceback (Sec. III-A, Alg. 1) ----
    // The survivor rows of a PB do not depend on the state being traced, so
    // they are loaded in blocks of TBR rows, kDepth - 1 blocks ahead of their
    // use (a ring of kDepth blocks); only the bit selection inside a row
    // follows the state.  Each lane loads the part of the row it stored (a
    // lane group's parts make up the PB's row); every lane of a group traces
    // the same state, takes the word it needs from the lane that holds it,
    // and the group's first lane writes the bits.
    // Rows of 4 or more dwords per PB are split: each lane of a group loads
    // its own part (W = NDW dwords); smaller rows are loaded whole by every
    // lane of the group (W = NDW_F).
    constexpr bool kSplit = LB > 0 && NDW_F >= 4;
    constexpr int W = kSplit ? NDW : NDW_F;
    constexpr int TBR = W >= 4 ? 4 : (W == 2 ? 8 : (16 / S));  // <= 16 stages, <= 16 dwords per block
    constexpr int kDepth = PBVD_TRACEBACK_BLOCKS;
    RowStore<W, kWave * NDW> tb_rows;
    tb_rows.rsrc = rows.rsrc;
    tb_rows.lane_off = kSplit || LB == 0 ? rows.lane_off
                                         : (uint32_t)(threadIdx.x & (kWave - 1)) / (1u << LB) * (NDW_F * 4);
    const bool writer = j.active && ell == 0;
    const int i_lo = j.store0_min;
    const int row_lo = i_lo / S;
    const int row_hi = (len - 1) / S;
    const int n_dec = j.my_dec_end - j.my_store0;
    uint32_t word = 0;
    int ph = (len - 1) % V;  // input phase of the stage being traced

    auto load_block = [&](uint32_t (&dst)[TBR][W], int top) PBVD_INLINE_LAMBDA {
#pragma unroll
        for (int t = 0; t < TBR; ++t) {
            const int row = top - t < row_lo ? row_lo : top - t;
            tb_rows.load(row, dst[t]);
        }
    };

    auto put_word = [&](int rel, int m) PBVD_INLINE_LAMBDA {
        const int64_t bitpos = j.out_bit0 + rel;
        if (j.out_mode == kOutDirect) {
            const int64_t byte = bitpos >> 3;
            if (m == 32 && byte + 4 <= j.out_bytes) {
                *reinterpret_cast<uint32_t *>(j.out + byte) = word;
            } else {
                for (int bb = 0; bb < ((m + 7) >> 3); ++bb)
                    if (byte + bb < j.out_bytes) j.out[byte + bb] = (uint8_t)(word >> (8 * bb));
            }
        } else if (j.out_mode == kOutAtomic) {
            const uint32_t sh = (uint32_t)(bitpos & 31);
            uint32_t *wp = j.out_words + (bitpos >> 5);
            atomicOr(wp, word << sh);
            if (sh && (word >> (32 - sh))) atomicOr(wp + 1, word >> (32 - sh));
        } else {
            // the lane owns whole bytes: its first bit is byte aligned
            uint8_t *ob = j.out + (bitpos >> 3);
            if (m == 32 && (((uintptr_t)ob & 3u) == 0)) {
                *reinterpret_cast<uint32_t *>(ob) = word;
            } else {
                for (int bb = 0; bb < ((m + 7) >> 3); ++bb) ob[bb] = (uint8_t)(word >> (8 * bb));
            }
        }
    };

    // bit position of the traced state's input bit at each phase, 4 bits per
    // phase (V <= 8), so a step finds it with shifts instead of branches
    constexpr uint32_t kQpos = [] {
        uint32_t t = 0;
        for (int p = 0; p < V; ++p) t |= (uint32_t)ubit_pos<V, LY::kBytePerm>(p) << (4 * p);
        return t;
    }();

    // follow the survivor of the traced state through one stage: its
    // decision bit in the stage's row (slot idx, + sub * NR for the sub-th
    // stage of a row) becomes bit qpos of the rotated index
    auto follow = [&](const uint32_t (&row)[W], int sub, uint32_t qpos) PBVD_INLINE_LAMBDA {
        uint32_t dec;
        if constexpr (!kSplit && W == 1) {
            dec = row[0] >> ((idx + (uint32_t)(sub * NR)) & 31u);
        } else if constexpr (!kSplit && W == 2) {
            const uint64_t r64 = ((uint64_t)row[1] << 32) | row[0];
            dec = (uint32_t)(r64 >> (idx & 63u));
        } else {
            // the row's dword idx >> 5: select among this lane's W
            // dwords with a binary tree, most significant index bit first
            // (v[w + half] differs from v[w] in that bit) ...
            uint32_t v[W];
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] = row[w];
            constexpr int kLogNdw = W >= 8 ? 3 : W >= 4 ? 2 : W >= 2 ? 1 : 0;
#pragma unroll
            for (int half = W / 2, bit = 4 + kLogNdw; half >= 1; half /= 2, --bit) {
                const bool up = (idx >> bit) & 1u;
#pragma unroll
                for (int w = 0; w < half; ++w) v[w] = up ? v[w + half] : v[w];
            }
            uint32_t wsel = v[0];
            if constexpr (kSplit) {
                // ... from the group lane that stored it: lane idx >> (5 + log NDW)
                const uint32_t owner = (idx >> (5 + kLogNdw)) & ((1u << LB) - 1);
                if constexpr (LB == 1) {
                    const uint32_t b0 = (uint32_t)dpp_int<quad_sel(0, 0, 2, 2)>((int)wsel);
                    const uint32_t b1 = (uint32_t)dpp_int<quad_sel(1, 1, 3, 3)>((int)wsel);
                    wsel = owner ? b1 : b0;
                } else {
                    // lane owner & 3 of this quad, then for groups of 8
                    // the other quad's when owner bit 2 differs from ours
                    const uint32_t b0 = (uint32_t)dpp_int<quad_sel(0, 0, 0, 0)>((int)wsel);
                    const uint32_t b1 = (uint32_t)dpp_int<quad_sel(1, 1, 1, 1)>((int)wsel);
                    const uint32_t b2 = (uint32_t)dpp_int<quad_sel(2, 2, 2, 2)>((int)wsel);
                    const uint32_t b3 = (uint32_t)dpp_int<quad_sel(3, 3, 3, 3)>((int)wsel);
                    wsel = owner & 2u ? (owner & 1u ? b3 : b2) : (owner & 1u ? b1 : b0);
                    if constexpr (LB == 3) {
                        const uint32_t other = (uint32_t)bit2_flip((int)wsel);
                        wsel = ((owner >> 2) & 1u) != (uint32_t)((ell >> 2) & 1) ? other : wsel;
                    }
                }
            }
            dec = wsel >> (idx & 31u);
        }
        // only bit 0 of dec is the decision: the insert mask drops the rest
        const uint32_t m = 1u << qpos;
        idx = (idx & ~m) | ((dec << qpos) & m);
    };

    if constexpr (S == 1) {
        if (!VARLEN || j.store0_uniform) {
            // ---- one stage per row and one first traced stage for the whole
            //      wave: blocks of V rows whose top row is at phase V-1, so every
            //      step's bit position is a compile-time constant; only the first
            //      and the last block (and the one holding the decoded range's
            //      end) check stage bounds.  With VARLEN each lane holds its start
            //      state until the traceback reaches its own last stage and takes
            //      bits only below its own decoded range's end (selects, no
            //      branches), so tiles of PBs of different lengths trace back at
            //      the rate of one geometry. ----
            constexpr int TB = V;
            constexpr int kRing = PBVD_TRACEBACK_RING_VGPRS / (TB * W) < 2 ? 2
                                : PBVD_TRACEBACK_RING_VGPRS / (TB * W) > 12 ? 12
                                : PBVD_TRACEBACK_RING_VGPRS / (TB * W);
            const int i_top = len - 1;
            const int dec_end = j.my_dec_end;  // decoded stages are [i_lo, dec_end)
            // take the input bit of stage i (decoded range) into the output word;
            // a word is complete at a multiple of 32 from the range's start
            auto take_bit = [&](int i, uint32_t qpos, bool emit) PBVD_INLINE_LAMBDA {
                const uint32_t nw = (word << 1) | ((idx >> qpos) & 1u);
                if constexpr (VARLEN) word = i < dec_end ? nw : word;
                else word = nw;
                if (__builtin_expect(emit, 0)) {  // one step in 32: keep it off the straight path
                    const int rel = i - i_lo;
                    const int m = n_dec - rel < 32 ? n_dec - rel : 32;
                    if (writer && (!VARLEN || m > 0)) put_word(rel, m);
                    word = 0;
                }
            };
            // a lane follows the survivors only below its own last stage
            auto follow_row = [&](const uint32_t (&row)[W], int i, uint32_t qpos) PBVD_INLINE_LAMBDA {
                if constexpr (VARLEN) {
                    const uint32_t held = idx;
                    follow(row, 0, qpos);
                    idx = i < j.my_len ? idx : held;
                } else {
                    follow(row, 0, qpos);
                }
            };
            // KIND 0: every stage is traced and decoded; 1: none is decoded;
            // 2: bounds and the decoded range's end are checked stage by stage
            auto run = [&](auto kc, const uint32_t (&blk)[TB][W], int top) PBVD_INLINE_LAMBDA {
                constexpr int kind = decltype(kc)::value;
                const int e = (top - i_lo) & 31;  // step whose bit completes a word
                static_for<0, TB>([&](auto tc) PBVD_INLINE_LAMBDA {
                    constexpr int t = decltype(tc)::value;
                    constexpr uint32_t qpos = ubit_pos<V, LY::kBytePerm>(V - 1 - t);
                    const int i = top - t;
                    if constexpr (kind == 2) {
                        if (i > i_top || i < i_lo) return true;
                        if (VARLEN || i < dec_end) take_bit(i, qpos, e == t);
                    } else if constexpr (kind == 0) {
                        take_bit(i, qpos, e == t);
                    }
                    follow_row(blk[t], i, qpos);
                    return true;
                });
            };
            auto load_rows = [&](uint32_t (&dst)[TB][W], int top) PBVD_INLINE_LAMBDA {
    #pragma unroll
                for (int t = 0; t < TB; ++t) {
                    int row = top - t;
                    row = row > row_hi ? row_hi : (row < row_lo ? row_lo : row);
                    tb_rows.load(row, dst[t]);
                }
            };
            uint32_t ring[kRing][TB][W];
            int top = i_top + (V - 1) - i_top % V;  // the first block's top row (phase V-1)
            static_for<0, kRing - 1>([&](auto dc) PBVD_INLINE_LAMBDA {
                load_rows(ring[decltype(dc)::value], top - decltype(dc)::value * TB);
                return true;
            });
            for (;;) {
                const bool more = static_for<0, kRing>([&](auto dc) PBVD_INLINE_LAMBDA {
                    constexpr int d = decltype(dc)::value;
                    load_rows(ring[(d + kRing - 1) % kRing], top - (kRing - 1) * TB);
                    const int bot = top - TB + 1;
                    // (VARLEN: the decoded range's end is checked in every step)
                    if (top > i_top || bot < i_lo || (!VARLEN && top >= dec_end && bot < dec_end))
                        run(std::integral_constant<int, 2>{}, ring[d], top);
                    else if (VARLEN || top < dec_end)
                        run(std::integral_constant<int, 0>{}, ring[d], top);
                    else
                        run(std::integral_constant<int, 1>{}, ring[d], top);
                    if (bot <= i_lo) return false;
                    top -= TB;
                    return true;
                });
                if (!more) break;
            }
            return;
        }
    }

    // one traceback step at stage i with that stage's survivor row
    auto step = [&](int i, const uint32_t (&row)[W], int sub) PBVD_INLINE_LAMBDA {
        const int qpos = (int)((kQpos >> (4 * ph)) & 15u);
        bool live = true;
        if constexpr (VARLEN) live = i < j.my_len && i >= j.my_store0;
        if (live) {
            const uint32_t x = (idx >> qpos) & 1u;
            if (i < j.my_dec_end) {
                word = (word << 1) | x;
                const int rel = i - j.my_store0;
                if ((rel & 31) == 0) {
                    if (writer) put_word(rel, n_dec - rel < 32 ? n_dec - rel : 32);
                    word = 0;
                }
            }
            follow(row, sub, (uint32_t)qpos);
        }
        ph = ph == 0 ? V - 1 : ph - 1;
    };

    // trace rows top..top-TBR+1; false once the first traced stage is passed
    auto run_block = [&](const uint32_t (&blk)[TBR][W], int top) PBVD_INLINE_LAMBDA {
        return static_for<0, TBR>([&](auto tc) PBVD_INLINE_LAMBDA {
            constexpr int t = decltype(tc)::value;
            const int row = top - t;
            if (row < row_lo) return false;
            return static_for<0, S>([&](auto sc) PBVD_INLINE_LAMBDA {
                constexpr int sub = S - 1 - decltype(sc)::value;
                const int i = row * S + sub;
                if (i >= len) return true;
                if (i < i_lo) return false;
                step(i, blk[t], sub);
                return true;
            });
        });
    };

    // ring of kDepth blocks: kDepth - 1 loaded ahead, the slot consumed last
    // is refilled before the next block is traced
    uint32_t ring[kDepth][TBR][W];
    int top = row_hi;
    static_for<0, kDepth - 1>([&](auto dc) PBVD_INLINE_LAMBDA {
        load_block(ring[decltype(dc)::value], top - decltype(dc)::value * TBR);
        return true;
    });
    for (;;) {
        const bool more = static_for<0, kDepth>([&](auto dc) PBVD_INLINE_LAMBDA {
            constexpr int d = decltype(dc)::value;
            load_block(ring[(d + kDepth - 1) % kDepth], top - (kDepth - 1) * TBR);
            if (!run_block(ring[d], top)) return false;
            top -= TBR;
            return true;
        });
        if (!more) break;
    }
}

// Register target for the 256-state trellis (waves per SIMD the compiler
// must leave room for).  Two waves force scratch spills inside the stage
// loop, which measured 2x slower than one wave with accumulator-register
// spills.
#ifndef PBVD_BIG_TRELLIS_WAVES_PER_EU
#define PBVD_BIG_TRELLIS_WAVES_PER_EU 1
#endif
// Register target for 64 metric VGPRs per lane (a 256-state trellis on lane
// pairs or 128 states on one lane, 16-bit metrics): three waves fit without
// spills.
#ifndef PBVD_MID_TRELLIS_WAVES_PER_EU
#define PBVD_MID_TRELLIS_WAVES_PER_EU 3
#endif
// MW = VGPRs of path metrics per lane
template <int MW>
__host__ __device__ constexpr int waves_per_eu_target() {
    return MW >= 128 ? PBVD_BIG_TRELLIS_WAVES_PER_EU : (MW >= 64 ? PBVD_MID_TRELLIS_WAVES_PER_EU : 1);
}

// ---------------------------------------------------------------------------
// Stream kernel: the PBs of one stream (Sec. III-A, Fig. 2).  Interior PBs
// (full geometry) go 64 to a wave.  PBs at the stream ends take the free
// slots the interior leaves (moved to the front of wave 0), so that they add
// no wave of their own while there is room; the others get a wave each.
// Waves of one SIMD run nearly one after another (the oldest wave issues
// first), so a single extra wave lengthens the whole launch by its share.
// ---------------------------------------------------------------------------
template <class C, class P, int KIND, int LB>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(waves_per_eu_target<(C::NR >> LB) * (int)(sizeof(typename P::T) / 4)>())))
    decode_kernel(const KernelArgs a) {
    using LY = Layout<C, P, LB>;
    constexpr int R = C::R, N = C::N, PW = LY::PW;
    constexpr int ND = (LY::U * R + 3) / 4 + 1;

    const int lane = threadIdx.x & (kWave - 1);
    const int pl = lane >> LB;  // the lane's PB inside the wave
    // wave index made provably uniform so that all geometry stays scalar
    const int64_t wave_local = (int64_t)blockIdx.x * (blockDim.x / kWave) +
                               __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (wave_local >= a.n_waves) return;
    const int64_t wave = a.wave_begin + wave_local;
    const int64_t D = a.D, L = a.L;

    RowStore<LY::NDW> rows;
    rows.rsrc = __builtin_amdgcn_make_buffer_rsrc(a.sp + wave_local * a.sp_wave_dwords, (short)0,
                                                  (int)(a.sp_wave_dwords * 4), kBufferFlags);
    rows.lane_off = (uint32_t)lane * (LY::NDW * 4);
    WaveJob j;
    j.out_mode = a.direct_out ? kOutDirect : kOutAtomic;
    j.out = a.out;
    j.out_bytes = a.out_bytes;
    j.out_words = a.out_words;
    j.in_end = a.syms + a.T * R;

    if (wave == 0 && a.n_fold > 0) {
        // ---- wave 0 with folded edge PBs: every lane has its own geometry
        //      (Sec. III-A, clipped to the stream), decoded like a batch tile.
        //      A lane shorter than the wave runs on past its own end, so its
        //      metrics at the wave's end are not its final metrics: the host
        //      folds no PB that starts its traceback from the best state and
        //      folds nothing when final metrics are asked for. ----
        int64_t b;
        bool active = true;
        if (pl < a.n_fold) {
            b = pl < a.n_head ? a.pb_first + pl : a.b_hi + (pl - a.n_head);
        } else {
            b = a.b_lo + (pl - a.n_fold);
            if (b >= a.b_hi) {
                b = a.b_hi - 1;
                active = false;
            }
        }
        const int64_t d0 = b * D;
        const int64_t f0 = d0 - L < 0 ? 0 : d0 - L;
        const int64_t f1 = d0 + D + L > a.T ? a.T : d0 + D + L;
        const int64_t d1 = d0 + D > a.n ? a.n : d0 + D;
        j.len = (int)(D + 2 * L);
        j.store0_min = a.n_head > 0 ? (int)(a.pb_first * D) : (int)L;
        j.i_safe = a.fold_i_safe;
        j.fetch_safe = a.fold_wide != 0;
        j.need_final = false;
        j.in = a.syms + f0 * R;
        j.my_len = (int)(f1 - f0);
        j.my_store0 = (int)(d0 - f0);
        j.my_dec_end = (int)(d1 - f0);
        j.known = f0 == 0;
        j.argmin = false;
        j.active = active;
        j.store0_uniform = false;
        j.out_bit0 = (b - a.pb_first) * D;
        j.pm_out = nullptr;
        decode_body<C, P, KIND, true, LB>(j, rows);
        return;
    }

    // ---- block geometry (Sec. III-A with M = L, clipped to the stream) ----
    int64_t b, f0w, f1w, d0w, d1w;   // wave-uniform PB geometry (interior: lane 0's)
    bool active;
    int64_t lane_stage_off;           // this lane's stage offset from f0w
    int64_t far_lane;                 // the wave's last real lane
    if (wave < a.n_int_waves) {
        const int64_t bw = a.b_lo + wave * PW - a.n_fold;
        b = bw + pl;
        active = b < a.b_hi;
        lane_stage_off = (active ? (int64_t)pl : (a.b_hi - 1 - bw)) * D;
        if (!active) b = a.b_hi - 1;
        far_lane = a.b_hi - 1 - bw < PW - 1 ? a.b_hi - 1 - bw : PW - 1;
        d0w = bw * D;
        f0w = d0w - L;
        f1w = d0w + D + L;
        d1w = d0w + D;
    } else {
        const int64_t e = wave - a.n_int_waves + a.n_fold;
        b = e < a.n_head ? a.pb_first + e : a.b_hi + (e - a.n_head);
        active = pl == 0;
        lane_stage_off = 0;
        far_lane = 0;
        d0w = b * D;
        f0w = d0w - L < 0 ? 0 : d0w - L;
        f1w = d0w + D + L > a.T ? a.T : d0w + D + L;
        d1w = d0w + D > a.n ? a.n : d0w + D;
    }
    // stage counts fit in 32 bits (at most D + 2L), which keeps the loop
    // control on the scalar unit
    j.len = (int)(f1w - f0w);
    j.store0_min = (int)(d0w - f0w);
    j.my_len = j.len;
    j.my_store0 = j.store0_min;
    j.my_dec_end = (int)(d1w - f0w);
    j.in = a.syms + (f0w + lane_stage_off) * R;
    // wave-uniform: every wide fetch of every lane stays inside the input;
    // only the last wave(s) of a stream take the byte-load path
    j.fetch_safe = a.syms + (f0w + far_lane * D + (j.len - 1)) * R + 4 * ND <= j.in_end;
    const int64_t safe_bytes = (int64_t)(j.in_end - (a.syms + (f0w + far_lane * D) * R)) - 4 * ND;
    j.i_safe = safe_bytes < 0 ? -1 : (safe_bytes / R > j.len ? j.len : (int)(safe_bytes / R));
    j.known = f0w + lane_stage_off == 0;  // an interior PB can start at 0 when L is a multiple of D
    j.argmin = f1w == a.T && !a.terminated;
    j.need_final = j.argmin || a.final_pm != nullptr;
    j.active = active;
    j.store0_uniform = true;
    j.out_bit0 = (b - a.pb_first) * D;
    j.pm_out = a.final_pm ? a.final_pm + (b - a.pb_first) * N : nullptr;
    decode_body<C, P, KIND, false, LB>(j, rows);
}

// ---------------------------------------------------------------------------
// Batch kernel: one wave per tile of up to 64 >> LB PBs of one code taken
// from any frames (lengths may differ inside a tile).  With lane groups the
// descriptor of a PB is repeated for each lane of its group.
// ---------------------------------------------------------------------------
struct LaneDesc {
    int64_t sym;       // byte offset in syms of the PB's first forward stage
    int64_t out_bit;   // bit offset in out of the PB's first decoded bit (byte aligned)
    int32_t len;       // forward stages
    int32_t store0;    // first traced stage
    int32_t dec_end;   // end of the decoded range (stage index)
    int32_t flags;     // kLaneKnown | kLaneArgmin | kLaneActive
};
struct TileHead {
    int32_t len;        // longest lane
    int32_t store0_min; // lowest first-traced stage
    int32_t flags;      // kTileWide | kTileFinal | kTileUniform | kTileStore0 | kTileCode1
    int32_t i_safe;     // without kTileWide: last stage whose wide symbol fetch is
                        // in bounds for every lane (-1: none); later trips load bytes
};
enum { kLaneKnown = 1, kLaneArgmin = 2, kLaneActive = 4 };
// kTileUniform: every lane has the same len, store0 and dec_end, so the tile
// runs the uniform-wave decode body (phase-aligned traceback); kTileStore0:
// every lane has the same store0 (lengths may differ), so the tile's
// traceback is phase-aligned too, with a per-lane start and end; kTileCode1:
// in a launch of a pair of codes, the tile's PBs are of the second code
enum { kTileWide = 1, kTileFinal = 2, kTileUniform = 4, kTileStore0 = 8, kTileCode1 = 16 };

struct TileArgs {
    const uint8_t *syms;
    int64_t sym_bytes;
    uint8_t *out;
    const LaneDesc *lanes;   // [tiles][64]
    const TileHead *heads;   // [tiles]
    uint32_t *sp;
    int64_t sp_wave_dwords;
    int64_t tile_begin;
    int64_t n_tiles;
};

// One tile of a batch (the wave's PBs, their descriptors and survivor slot).
template <class C, class P, int KIND, int LB>
__device__ __forceinline__ void tile_body(const TileArgs &a, int64_t wave_local, int lane, const TileHead &h,
                                          int tflags) {
    using LY = Layout<C, P, LB>;
    const int64_t tile = a.tile_begin + wave_local;
    const LaneDesc d = a.lanes[tile * kWave + lane];

    WaveJob j;
    j.len = __builtin_amdgcn_readfirstlane(h.len);
    j.store0_min = __builtin_amdgcn_readfirstlane(h.store0_min);
    j.fetch_safe = (tflags & kTileWide) != 0;
    j.i_safe = j.fetch_safe ? j.len : __builtin_amdgcn_readfirstlane(h.i_safe);
    j.need_final = (tflags & kTileFinal) != 0;
    j.in_end = a.syms + a.sym_bytes;
    j.in = a.syms + d.sym;
    j.my_len = d.len;
    j.my_store0 = d.store0;
    j.my_dec_end = d.dec_end;
    j.known = (d.flags & kLaneKnown) != 0;
    j.argmin = (d.flags & kLaneArgmin) != 0;
    j.active = (d.flags & kLaneActive) != 0;
    j.store0_uniform = (tflags & kTileStore0) != 0;
    j.out_mode = kOutBytes;
    j.out = a.out;
    j.out_bytes = 0;
    j.out_words = nullptr;
    j.out_bit0 = d.out_bit;
    j.pm_out = nullptr;

    RowStore<LY::NDW> rows;
    rows.rsrc = __builtin_amdgcn_make_buffer_rsrc(a.sp + wave_local * a.sp_wave_dwords, (short)0,
                                                  (int)(a.sp_wave_dwords * 4), kBufferFlags);
    rows.lane_off = (uint32_t)lane * (LY::NDW * 4);
    if (tflags & kTileUniform) {
        j.my_len = j.len;
        j.my_store0 = j.store0_min;
        j.my_dec_end = __builtin_amdgcn_readfirstlane(d.dec_end);
        decode_body<C, P, KIND, false, LB>(j, rows);
    } else {
        decode_body<C, P, KIND, true, LB>(j, rows);
    }
}

template <class C, class P, int KIND, int LB>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(waves_per_eu_target<(C::NR >> LB) * (int)(sizeof(typename P::T) / 4)>())))
    decode_tiles_kernel(const TileArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave_local = (int64_t)blockIdx.x * (blockDim.x / kWave) +
                               __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (wave_local >= a.n_tiles) return;
    const TileHead h = a.heads[a.tile_begin + wave_local];
    tile_body<C, P, KIND, LB>(a, wave_local, lane, h, __builtin_amdgcn_readfirstlane(h.flags));
}

// Batch kernel for a pair of codes of one constraint length: the tiles of
// both in one launch (longest first over both), each tile decoded with the
// code its head names (kTileCode1: the second).  One launch instead of one
// per code: no fork and join of streams, and the waves of both codes share
// the compute units from the first to the last tile.
template <class C0, class C1, class P, int KIND, int LB>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(waves_per_eu_target<(C0::NR >> LB) * (int)(sizeof(typename P::T) / 4)>())))
    decode_tiles_pair_kernel(const TileArgs a) {
    static_assert(C0::K == C1::K, "a pair shares one trellis size");
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave_local = (int64_t)blockIdx.x * (blockDim.x / kWave) +
                               __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (wave_local >= a.n_tiles) return;
    const TileHead h = a.heads[a.tile_begin + wave_local];
    const int tflags = __builtin_amdgcn_readfirstlane(h.flags);
    if (tflags & kTileCode1) tile_body<C1, P, KIND, LB>(a, wave_local, lane, h, tflags);
    else tile_body<C0, P, KIND, LB>(a, wave_local, lane, h, tflags);
}

}  // namespace pbvd
