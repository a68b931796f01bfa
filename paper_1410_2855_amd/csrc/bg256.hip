// Persistent round-trip kernels for batches of N = 256 cavities (two
// register budgets).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_256() {
    return group_info<S256>({GroupKernels<4, S256>::variant(), GroupKernels<2, S256>::variant()});
}
}  // namespace lsr
