// Batch kernels for N = 1024 cavities of which some have a rough mirror: each
// cavity's local-step code (model and roughness) is read per cavity.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_anyr_1024() { return group_info<S1024>({GroupKernelsT<2, 2, S1024>::variant()}, 0, 2); }
}  // namespace lsr
