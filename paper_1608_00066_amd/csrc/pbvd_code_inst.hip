// Decoder kernels of one registered code.  Compiled once per code with
// -DPBVD_CODE_IDX=<index>, so the per-code kernels build in parallel.
#include "pbvd_registry.hpp"

#ifndef PBVD_CODE_IDX
#error "compile with -DPBVD_CODE_IDX=<registry index>"
#endif

namespace pbvd {
namespace {

template <int IDX>
struct CodeAt;
#define PBVD_CODE_AT(i, K, R, g0, g1, g2, g3) \
    template <>                               \
    struct CodeAt<i> {                        \
        using type = FixedCode<K, R, g0, g1, g2, g3>; \
    };
PBVD_CODE_LIST(PBVD_CODE_AT)
#undef PBVD_CODE_AT

template <class C, class P, int KIND, int LB>
hipError_t launch_lb(const LaunchRequest &req) {
    if constexpr (lanes_supported<C, P, LB>()) {
        hipLaunchKernelGGL((decode_kernel<C, P, KIND, LB>), dim3(req.grid), dim3(kBlockThreads), 0,
                           req.stream, req.args);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <class C, class P, int KIND>
hipError_t launch_one(const LaunchRequest &req) {
    switch (req.lb) {
    case 0: return launch_lb<C, P, KIND, 0>(req);
    case 1: return launch_lb<C, P, KIND, 1>(req);
    case 2: return launch_lb<C, P, KIND, 2>(req);
    case 3: return launch_lb<C, P, KIND, 3>(req);
    }
    return hipErrorInvalidValue;
}

template <class C, class P, int KIND, int LB>
hipError_t launch_tiles_lb(const TileLaunchRequest &req) {
    if constexpr (lanes_supported<C, P, LB>()) {
        hipLaunchKernelGGL((decode_tiles_kernel<C, P, KIND, LB>), dim3(req.grid), dim3(req.block_threads), 0,
                           req.stream, req.args);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <class C, class P, int KIND>
hipError_t launch_tiles_one(const TileLaunchRequest &req) {
    switch (req.lb) {
    case 0: return launch_tiles_lb<C, P, KIND, 0>(req);
    case 1: return launch_tiles_lb<C, P, KIND, 1>(req);
    case 2: return launch_tiles_lb<C, P, KIND, 2>(req);
    case 3: return launch_tiles_lb<C, P, KIND, 3>(req);
    }
    return hipErrorInvalidValue;
}

}  // namespace

template <int IDX>
hipError_t launch_code(const LaunchRequest &req) {
    using C = typename CodeAt<IDX>::type;
    if (req.pm_bits == 16) {
        return req.input_kind == kHardU8 ? launch_one<C, PM16, kHardU8>(req)
                                         : launch_one<C, PM16, kSoftI8>(req);
    }
    if constexpr (C::K <= 8) {
        if (req.pm_bits == 32)
            return req.input_kind == kHardU8 ? launch_one<C, PM32, kHardU8>(req)
                                             : launch_one<C, PM32, kSoftI8>(req);
    }
    return hipErrorInvalidValue;
}

template <int IDX>
hipError_t launch_tiles(const TileLaunchRequest &req) {
    using C = typename CodeAt<IDX>::type;
    if (req.pm_bits == 16) {
        return req.input_kind == kHardU8 ? launch_tiles_one<C, PM16, kHardU8>(req)
                                         : launch_tiles_one<C, PM16, kSoftI8>(req);
    }
    if constexpr (C::K <= 8) {
        if (req.pm_bits == 32)
            return req.input_kind == kHardU8 ? launch_tiles_one<C, PM32, kHardU8>(req)
                                             : launch_tiles_one<C, PM32, kSoftI8>(req);
    }
    return hipErrorInvalidValue;
}

template hipError_t launch_code<PBVD_CODE_IDX>(const LaunchRequest &req);
template hipError_t launch_tiles<PBVD_CODE_IDX>(const TileLaunchRequest &req);

}  // namespace pbvd
