// Batch kernels for N = 4096 cavities of which some have a rough mirror: each
// cavity's local-step code (model and roughness) is read per cavity.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_anyr_4096() { return group_info<S4096>({GroupKernelsT<1, 2, S4096>::variant()}, 0, 2); }
}  // namespace lsr
