// Batch kernels for N = 1024 with the alternative plans: radix order 16 16 4,
// and 8 x 8 tiles (eight lines per workgroup of 512 threads, held to four
// waves per SIMD so that two workgroups share a CU).
#include "batch_impl.hpp"

namespace lsr {
GroupInfo group_1024r() {
    return group_info<S1024r>({GroupKernels<4, S1024r>::variant(), GroupKernels<2, S1024r>::variant()}, 1);
}
GroupInfo group_1024t() { return group_info<S1024t>({GroupKernels<4, S1024t>::variant()}, 2); }
}  // namespace lsr
