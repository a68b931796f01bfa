// Batch kernels for N = 2048 with the alternative radix order 16 16 8 (two
// register budgets).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_2048r() {
    return group_info<S2048r>({GroupKernels<4, S2048r>::variant(), GroupKernels<2, S2048r>::variant()}, 1);
}
}  // namespace lsr
