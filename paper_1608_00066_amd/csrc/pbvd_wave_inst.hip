// State-parallel (one wave per PB) decoder kernel for one constraint length
// (every rate and input kind: they are run-time arguments).  Compiled once
// per K with -DPBVD_WAVE_K=<K>.
#include "pbvd_wave.hpp"
#include "pbvd_registry.hpp"

#ifndef PBVD_WAVE_K
#error "compile with -DPBVD_WAVE_K=<constraint length>"
#endif

namespace pbvd {

template <int K>
hipError_t launch_wave(const WaveLaunchRequest &req) {
    if (req.args.counter)
        hipLaunchKernelGGL((wave::decode_wave_kernel<K - 1, wave::kModePersist>), dim3(req.grid),
                           dim3(kBlockThreads), 0, req.stream, req.args, req.args.syms);
    else if (req.args.dec_sp)
        hipLaunchKernelGGL((wave::decode_wave_kernel<K - 1, wave::kModeDecisions>), dim3(req.grid),
                           dim3(kBlockThreads), 0, req.stream, req.args, req.args.syms);
    else
        hipLaunchKernelGGL((wave::decode_wave_kernel<K - 1, wave::kModeList>), dim3(req.grid),
                           dim3(kBlockThreads), 0, req.stream, req.args, req.args.syms);
    return hipGetLastError();
}

template <int K>
int wave_persistent_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wave::decode_wave_kernel<K - 1, wave::kModePersist>,
                                                     kBlockThreads, 0) != hipSuccess)
        return 0;
    return n;
}

template hipError_t launch_wave<PBVD_WAVE_K>(const WaveLaunchRequest &req);
template int wave_persistent_blocks_per_cu<PBVD_WAVE_K>();

}  // namespace pbvd
