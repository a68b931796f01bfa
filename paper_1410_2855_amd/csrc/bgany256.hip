// Batch kernels for N = 256 cavities whose local-step model is any of the
// three (the model is read per cavity; batches of the default model use the
// kernels compiled for it alone).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_any_256() { return group_info<S256>({GroupKernelsT<2, 1, S256>::variant()}, 0, 1); }
}  // namespace lsr
