// Batch kernels for N = 2048 cavities of which some have a rough mirror: each
// cavity's local-step code (model and roughness) is read per cavity.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_anyr_2048() { return group_info<S2048>({GroupKernelsT<2, 2, S2048>::variant()}, 0, 2); }
}  // namespace lsr
