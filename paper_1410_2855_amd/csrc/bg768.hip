// Persistent round-trip kernels for batches of N = 768 cavities (two
// register budgets).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_768() {
    return group_info<S768>({GroupKernels<4, S768>::variant(), GroupKernels<2, S768>::variant()});
}
}  // namespace lsr
