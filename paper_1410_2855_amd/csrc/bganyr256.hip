// Batch kernels for N = 256 cavities of which some have a rough mirror: each
// cavity's local-step code (model and roughness) is read per cavity.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_anyr_256() { return group_info<S256>({GroupKernelsT<2, 2, S256>::variant()}, 0, 2); }
}  // namespace lsr
