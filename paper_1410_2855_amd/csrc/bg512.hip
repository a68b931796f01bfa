// Persistent round-trip kernels for batches of N = 512 cavities (two
// register budgets).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_512() {
    return group_info<S512>({GroupKernels<4, S512>::variant(), GroupKernels<2, S512>::variant()});
}
}  // namespace lsr
