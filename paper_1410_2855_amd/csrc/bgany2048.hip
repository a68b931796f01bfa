// Batch kernels for N = 2048 cavities whose local-step model is any of the
// three (the model is read per cavity; batches of the default model use the
// kernels compiled for it alone).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_any_2048() { return group_info<S2048>({GroupKernelsT<2, 1, S2048>::variant()}, 0, 1); }
}  // namespace lsr
