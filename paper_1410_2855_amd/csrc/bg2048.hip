// Persistent round-trip kernels for batches of N = 2048 cavities (two
// register budgets).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_2048() {
    return group_info<S2048>({GroupKernels<4, S2048>::variant(), GroupKernels<2, S2048>::variant()});
}
}  // namespace lsr
