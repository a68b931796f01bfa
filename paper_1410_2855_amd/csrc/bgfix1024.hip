// Batch kernels for N = 1024 cavities that all have the same non-default
// local-step model (exact B-class update or class A) and a smooth mirror:
// that model alone is compiled in.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_fix1_1024() { return group_info<S1024>({GroupKernelsT<4, ANY_FIXED + 1, S1024>::variant(), GroupKernelsT<2, ANY_FIXED + 1, S1024>::variant()}, 0, ANY_FIXED + 1); }
GroupInfo group_fix2_1024() { return group_info<S1024>({GroupKernelsT<4, ANY_FIXED + 2, S1024>::variant(), GroupKernelsT<2, ANY_FIXED + 2, S1024>::variant()}, 0, ANY_FIXED + 2); }
}  // namespace lsr
