// Small helper kernels of the decoder library: output staging for block
// lengths that are not a multiple of 32 bits, and the two verification hooks
// (survivor expansion, branch metrics).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbvd_aux.hpp"
#include "pbvd_kernel.hpp"
#include "pbvd_wave_args.hpp"

namespace pbvd {
namespace {

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void words_to_bytes_kernel(const uint32_t *w, uint8_t *out, int64_t nbytes) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nbytes;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (uint8_t)(w[i >> 2] >> (8 * (i & 3)));
}

__device__ __forceinline__ int rotl_dyn(int u, int s, int V) {
    s %= V;
    return ((u << s) | (u >> (V - s))) & ((1 << V) - 1);
}

// One thread per (PB, stored row, state): the decision of `state` at stage
// b*D + row, read back from the packed layout the forward pass wrote.
__global__ void unpack_survivors_kernel(SurvivorView v, uint8_t *dec) {
    const int N = 1 << (v.K - 1), NR = N / 2, V = v.K - 1;
    const int64_t rows = (int64_t)v.D + v.L;
    const int64_t total = v.pb_count * rows * N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int state = (int)(t % N);
        const int64_t row = (t / N) % rows;
        const int64_t pbl = t / (N * rows);
        const int64_t b = v.pb_first + pbl;
        const int64_t d0 = b * v.D;
        const int64_t f0 = d0 - v.L < 0 ? 0 : d0 - v.L;
        const int64_t f1 = d0 + v.D + v.L > v.T ? v.T : d0 + v.D + v.L;
        uint8_t bit = 0;
        if (d0 + row < f1) {
            const int pw = kWave >> v.lb;  // PBs per wave
            const WavePlace wp = wave_place(b, v.pb_first, v.b_lo, v.b_hi, v.n_head, v.n_fold, v.n_int_waves, pw);
            const int64_t wave = wp.wave;
            const int slot = wp.slot;     // the PB's place in its wave
            const int i = (int)(d0 + row - f0);       // stage index inside the PB
            const int u = rotl_dyn(state, i + 1, V);  // register map after stage i
            const int r = u & (NR - 1), half = u >> (V - 1);
            const uint32_t *base = v.sp + wave * v.sp_wave_dwords;
            uint32_t w;
            int pos;
            if (NR >= 16) {
                // a row holds the PBs of the wave one after another, each
                // PB's NR/16 dwords in register order (a lane group stores
                // them lane by lane, which is the same order)
                const int ndw = NR / 16;
                w = base[(int64_t)i * pw * ndw + (int64_t)slot * ndw + (r >> 4)];
                pos = v.byte_perm ? 16 * (r & 1) + 8 * half + ((r & 15) >> 1) : (r & 15) + 16 * half;
            } else {
                const int S = 16 / NR;
                w = base[(int64_t)(i / S) * kWave + slot];
                pos = (i % S) * NR + r + 16 * half;
            }
            bit = (uint8_t)((w >> pos) & 1);
        }
        dec[t] = bit;
    }
}

// The same for the state-parallel kernel: PB p of the call in slot p; its
// trips are aligned to the end of its forward range; the decision of state
// j at stage i (k-th step of its trip, phase k mod V) sits at position
// rotl^(k+1)(j): lane u mod 64, slot u / 64, bit W-1-k of the trip's word.
__global__ void unpack_wave_survivors_kernel(SurvivorView v, uint8_t *dec) {
    const int V = v.K - 1, N = 1 << V;
    const int W = wave::trip_stages(V), SL = wave::slots(V);
    const int64_t rows = (int64_t)v.D + v.L;
    const int64_t total = v.pb_count * rows * N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int state = (int)(t % N);
        const int64_t row = (t / N) % rows;
        const int64_t pbl = t / (N * rows);
        const int64_t b = v.pb_first + pbl;
        const int64_t d0 = b * v.D;
        const int64_t f0 = d0 - v.L < 0 ? 0 : d0 - v.L;
        const int64_t f1 = d0 + v.D + v.L > v.T ? v.T : d0 + v.D + v.L;
        uint8_t bit = 0;
        if (d0 + row < f1) {
            const int64_t len = f1 - f0;
            const int64_t n_trips = (len + W - 1) / W;
            const int64_t kk = (d0 + row - f0) + (n_trips * W - len);
            const int64_t trip = kk / W;
            const int k = (int)(kk % W);
            const int u = rotl_dyn(state, k % V + 1, V);
            const int lane = u & 63, slot = u >> 6;
            const uint32_t w = v.sp[pbl * v.sp_wave_dwords + (trip * SL + slot) * kWave + lane];
            bit = (uint8_t)((w >> (W - 1 - k)) & 1u);
        }
        dec[t] = bit;
    }
}

template <int R, int KIND>
__global__ void branch_metrics_kernel(const uint8_t *syms, int64_t n_stages, int32_t *out) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_stages;
         s += (int64_t)gridDim.x * blockDim.x) {
        int q[R];
#pragma unroll
        for (int r = 0; r < R; ++r) q[r] = rx_value<KIND>(syms + s * R + r);
        int bm[1 << R];
        code_word_metrics<R>(q, bm);
#pragma unroll
        for (int c = 0; c < (1 << R); ++c) out[s * (1 << R) + c] = bm[c];
    }
}

unsigned grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

template <int R>
void launch_bm(int kind, const uint8_t *syms, int64_t n_stages, int32_t *out, hipStream_t s) {
    const unsigned g = grid_for(n_stages, 256);
    if (kind == kHardU8)
        hipLaunchKernelGGL((branch_metrics_kernel<R, kHardU8>), dim3(g), dim3(256), 0, s, syms, n_stages, out);
    else
        hipLaunchKernelGGL((branch_metrics_kernel<R, kSoftI8>), dim3(g), dim3(256), 0, s, syms, n_stages, out);
}

}  // namespace

hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t words_to_bytes(const uint32_t *w, uint8_t *out, int64_t nbytes, hipStream_t s) {
    if (nbytes <= 0) return hipSuccess;
    hipLaunchKernelGGL(words_to_bytes_kernel, dim3(grid_for(nbytes, 256)), dim3(256), 0, s, w, out, nbytes);
    return hipGetLastError();
}

hipError_t unpack_survivors(const SurvivorView &v, uint8_t *dec, hipStream_t s) {
    const int64_t total = v.pb_count * ((int64_t)v.D + v.L) * (1 << (v.K - 1));
    if (total <= 0) return hipSuccess;
    if (v.wave)
        hipLaunchKernelGGL(unpack_wave_survivors_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, v, dec);
    else
        hipLaunchKernelGGL(unpack_survivors_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, v, dec);
    return hipGetLastError();
}

hipError_t branch_metrics(int R, int kind, const uint8_t *syms, int64_t n_stages, int32_t *out,
                          hipStream_t s) {
    if (n_stages <= 0) return hipSuccess;
    switch (R) {
    case 2: launch_bm<2>(kind, syms, n_stages, out, s); break;
    case 3: launch_bm<3>(kind, syms, n_stages, out, s); break;
    case 4: launch_bm<4>(kind, syms, n_stages, out, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pbvd
