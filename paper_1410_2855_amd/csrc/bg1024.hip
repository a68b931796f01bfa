// Persistent round-trip kernels for batches of N = 1024 cavities (two
// register budgets).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_1024() {
    return group_info<S1024>({GroupKernels<4, S1024>::variant(), GroupKernels<2, S1024>::variant()});
}
}  // namespace lsr
