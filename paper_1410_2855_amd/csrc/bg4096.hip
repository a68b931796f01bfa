// Persistent round-trip kernels for batches of N = 4096 cavities.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_4096() { return group_info<S4096>({GroupKernels<1, S4096>::variant()}); }
}  // namespace lsr
