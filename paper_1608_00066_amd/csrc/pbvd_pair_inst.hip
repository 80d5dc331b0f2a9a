// Batch tile kernels of one pair of registered codes (both codes' tiles in
// one launch).  Compiled once per pair and input kind with
// -DPBVD_PAIR_IDX=<index> -DPBVD_PAIR_KIND=<kSoftI8 or kHardU8>, so the
// units build in parallel.
#include "pbvd_registry.hpp"

#if !defined(PBVD_PAIR_IDX) || !defined(PBVD_PAIR_KIND)
#error "compile with -DPBVD_PAIR_IDX=<pair index> -DPBVD_PAIR_KIND=<input kind>"
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

template <int IDX>
struct PairAt;
#define PBVD_PAIR_AT(i, a, b)                       \
    template <>                                     \
    struct PairAt<i> {                              \
        using first = typename CodeAt<a>::type;     \
        using second = typename CodeAt<b>::type;    \
    };
PBVD_PAIR_LIST(PBVD_PAIR_AT)
#undef PBVD_PAIR_AT

template <class C0, class C1, int KIND, int LB>
hipError_t launch_pair_lb(const TileLaunchRequest &req) {
    if constexpr (lanes_supported<C0, PM16, LB>() && lanes_supported<C1, PM16, LB>()) {
        hipLaunchKernelGGL((decode_tiles_pair_kernel<C0, C1, PM16, KIND, LB>), dim3(req.grid),
                           dim3(req.block_threads), 0, req.stream, req.args);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <class C0, class C1, int KIND>
hipError_t launch_pair_kind(const TileLaunchRequest &req) {
    switch (req.lb) {
    case 0: return launch_pair_lb<C0, C1, KIND, 0>(req);
    case 1: return launch_pair_lb<C0, C1, KIND, 1>(req);
    case 2: return launch_pair_lb<C0, C1, KIND, 2>(req);
    case 3: return launch_pair_lb<C0, C1, KIND, 3>(req);
    }
    return hipErrorInvalidValue;
}

}  // namespace

template <int IDX, int KIND>
hipError_t launch_tiles_pair(const TileLaunchRequest &req) {
    using C0 = typename PairAt<IDX>::first;
    using C1 = typename PairAt<IDX>::second;
    static_assert(C0::K == C1::K, "a pair shares one trellis size");
    if (req.pm_bits != 16 || req.input_kind != KIND) return hipErrorInvalidValue;
    return launch_pair_kind<C0, C1, KIND>(req);
}

template hipError_t launch_tiles_pair<PBVD_PAIR_IDX, PBVD_PAIR_KIND>(const TileLaunchRequest &req);

}  // namespace pbvd
