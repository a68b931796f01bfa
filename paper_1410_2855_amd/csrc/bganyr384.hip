// Batch kernels for N = 384 cavities of which some have a rough mirror: each
// cavity's local-step code (model and roughness) is read per cavity.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_anyr_384() { return group_info<S384>({GroupKernelsT<2, 2, S384>::variant()}, 0, 2); }
}  // namespace lsr
