// Batch kernels for N = 1024 cavities whose local-step model is any of the
// three (the model is read per cavity; batches of the default model use the
// kernels compiled for it alone).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_any_1024() { return group_info<S1024>({GroupKernelsT<2, 1, S1024>::variant()}, 0, 1); }
}  // namespace lsr
