// Batch kernels for N = 512 with the alternative radix order 16 8 4 (two
// register budgets).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_512r() {
    return group_info<S512r>({GroupKernels<4, S512r>::variant(), GroupKernels<2, S512r>::variant()}, 1);
}
}  // namespace lsr
