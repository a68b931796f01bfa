// Batch kernels for N = 256 with 8 points per lane (32 lanes x 8 lines,
// radices 8 8 4), the alternative plan 1 of this size: the shape a lone
// small cavity runs fastest with, for a batch of one replayed from graphs.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_256l() { return group_info<L256>({GroupKernels<4, L256>::variant(), GroupKernels<2, L256>::variant()}, 1); }
}  // namespace lsr
