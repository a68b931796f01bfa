// Batch kernels for N = 768 cavities of which some have a rough mirror: each
// cavity's local-step code (model and roughness) is read per cavity.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_anyr_768() { return group_info<S768>({GroupKernelsT<2, 2, S768>::variant()}, 0, 2); }
}  // namespace lsr
