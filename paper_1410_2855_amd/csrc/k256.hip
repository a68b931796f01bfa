// Kernels for N = 256 (FP32 and FP64 forms, and the one-cavity shapes with
// 8 and 4 points per lane).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_256f() { return make_launchers<S256, float>(); }
const Launchers* launchers_256d() { return make_launchers<D256, double>(); }
const Launchers* launchers_256l() { return make_launchers<L256, float>(); }
const Launchers* launchers_256q() { return make_launchers<L256q, float>(); }
const Launchers* launchers_256p() { return make_launchers<L256p, float>(); }
}  // namespace lsr
