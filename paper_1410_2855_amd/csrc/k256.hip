// Kernels for N = 256 (FP32 and FP64 forms, and the one-cavity shape with
// 8 points per lane).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_256f() { return make_launchers<S256, float>(); }
const Launchers* launchers_256d() { return make_launchers<D256, double>(); }
const Launchers* launchers_256l() { return make_launchers<L256, float>(); }
}  // namespace lsr
