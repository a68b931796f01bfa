// Batch kernels for N = 4096 cavities whose local-step model is any of the
// three (the model is read per cavity; batches of the default model use the
// kernels compiled for it alone).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_any_4096() { return group_info<S4096>({GroupKernelsT<1, 1, S4096>::variant()}, 0, 1); }
}  // namespace lsr
