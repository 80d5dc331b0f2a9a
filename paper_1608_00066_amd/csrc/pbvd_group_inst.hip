// Group-mapped decoder kernels (pbvd_group.hpp) for one constraint length,
// every rate the mapping takes.  Compiled once per K with -DPBVD_GROUP_K=<K>.
#include "pbvd_group.hpp"
#include "pbvd_registry.hpp"

#ifndef PBVD_GROUP_K
#error "compile with -DPBVD_GROUP_K=<constraint length>"
#endif

namespace pbvd {

namespace {

template <int K, int R>
hipError_t launch_rate(const GroupLaunchRequest &req) {
    if constexpr (group::shape_ok(K, R)) {
        constexpr size_t lds = group::lds_bytes<K - 1, R>();
        if constexpr (lds > 65536) {
            // more than the default dynamic LDS of a launch
            static const hipError_t attr = hipFuncSetAttribute(
                reinterpret_cast<const void *>(&group::decode_group_kernel<K - 1, R>),
                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)attr;
        }
        hipLaunchKernelGGL((group::decode_group_kernel<K - 1, R>), dim3(req.grid), dim3(group::kTilePbs << R), lds,
                           req.stream, req.args);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace

template <int K>
hipError_t launch_group_kernel(const GroupLaunchRequest &req) {
    switch (req.R) {
    case 2: return launch_rate<K, 2>(req);
    case 3: return launch_rate<K, 3>(req);
    case 4: return launch_rate<K, 4>(req);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_group_kernel<PBVD_GROUP_K>(const GroupLaunchRequest &req);

}  // namespace pbvd
