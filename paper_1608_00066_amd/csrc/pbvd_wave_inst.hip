// State-parallel (one wave per PB) decoder kernels for one constraint length,
// every rate and input kind.  Compiled once per K with -DPBVD_WAVE_K=<K>.
#include "pbvd_wave.hpp"
#include "pbvd_registry.hpp"

#ifndef PBVD_WAVE_K
#error "compile with -DPBVD_WAVE_K=<constraint length>"
#endif

namespace pbvd {

template <int K>
hipError_t launch_wave(const WaveLaunchRequest &req) {
    constexpr int V = K - 1;
    const int R = req.R;
    const bool hard = req.input_kind == kHardU8;
#define PBVD_WAVE_CASE(RR)                                                                           \
    if (R == RR) {                                                                                  \
        if (hard)                                                                                   \
            hipLaunchKernelGGL((wave::decode_wave_kernel<V, RR, kHardU8>), dim3(req.grid),          \
                               dim3(kBlockThreads), 0, req.stream, req.args, req.args.syms);                       \
        else                                                                                        \
            hipLaunchKernelGGL((wave::decode_wave_kernel<V, RR, kSoftI8>), dim3(req.grid),          \
                               dim3(kBlockThreads), 0, req.stream, req.args, req.args.syms);                       \
        return hipGetLastError();                                                                   \
    }
    PBVD_WAVE_CASE(2)
    PBVD_WAVE_CASE(3)
    PBVD_WAVE_CASE(4)
#undef PBVD_WAVE_CASE
    return hipErrorInvalidValue;
}

template hipError_t launch_wave<PBVD_WAVE_K>(const WaveLaunchRequest &req);

}  // namespace pbvd
