// Round-trip kernels shared by cavities of uneven grid size (N = 256 .. 1024,
// the 256-thread shapes): one launch advances all of them.
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_small() {
    return group_info<S256, S384, S512, S768, S1024>(
        {GroupKernels<2, S256, S384, S512, S768, S1024>::variant()});
}
}  // namespace lsr
