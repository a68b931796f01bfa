// Batch kernels for N = 4096 with 128 lanes per line (512 threads, 32
// points per lane), the alternative plan 1 of this size.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_4096w() { return group_info<S4096w>({GroupKernels<1, S4096w>::variant()}, 1); }
}  // namespace lsr
