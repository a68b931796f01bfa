// Batch kernels for N = 512 cavities of which some have a rough mirror: each
// cavity's local-step code (model and roughness) is read per cavity.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_anyr_512() { return group_info<S512>({GroupKernelsT<2, 2, S512>::variant()}, 0, 2); }
}  // namespace lsr
