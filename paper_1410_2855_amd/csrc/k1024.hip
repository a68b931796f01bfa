// Kernels for N = 1024 (FP32 and FP64 forms, and the one-cavity shape with
// 8 points per lane).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_1024f() { return make_launchers<S1024, float>(); }
const Launchers* launchers_1024d() { return make_launchers<D1024, double>(); }
const Launchers* launchers_1024l() { return make_launchers<L1024, float>(); }
}  // namespace lsr
