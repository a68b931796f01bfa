// Kernels for N = 1024 (FP32 and FP64 forms).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_1024f() { return make_launchers<S1024, float>(); }
const Launchers* launchers_1024d() { return make_launchers<D1024, double>(); }
}  // namespace lsr
