// Persistent round-trip kernels for batches of N = 384 cavities (two
// register budgets).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_384() {
    return group_info<S384>({GroupKernels<4, S384>::variant(), GroupKernels<2, S384>::variant()});
}
}  // namespace lsr
