// Batch kernels for N = 4096 cavities that all have the same non-default
// local-step model (exact B-class update or class A) and a smooth mirror:
// that model alone is compiled in.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_fix1_4096() { return group_info<S4096>({GroupKernelsT<1, ANY_FIXED + 1, S4096>::variant()}, 0, ANY_FIXED + 1); }
GroupInfo group_fix2_4096() { return group_info<S4096>({GroupKernelsT<1, ANY_FIXED + 2, S4096>::variant()}, 0, ANY_FIXED + 2); }
}  // namespace lsr
