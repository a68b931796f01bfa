// Kernels for N = 256 (FP32 and FP64 forms).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_256f() { return make_launchers<S256, float>(); }
const Launchers* launchers_256d() { return make_launchers<D256, double>(); }
}  // namespace lsr
