// Batch kernels for N = 384 cavities whose local-step model is any of the
// three (the model is read per cavity; batches of the default model use the
// kernels compiled for it alone).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_any_384() { return group_info<S384>({GroupKernelsT<2, 1, S384>::variant()}, 0, 1); }
}  // namespace lsr
