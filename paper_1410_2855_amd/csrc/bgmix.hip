// Persistent round-trip kernels for mixed batches: N = 256 .. 1024, and
// N = 256 .. 2048 (256-thread shapes).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_small() {
    return group_info<S256, S384, S512, S768, S1024>(
        {GroupKernels<2, S256, S384, S512, S768, S1024>::variant()});
}
GroupInfo group_all256() {
    return group_info<S256, S384, S512, S768, S1024, S2048>(
        {GroupKernels<2, S256, S384, S512, S768, S1024, S2048>::variant()});
}
}  // namespace lsr
