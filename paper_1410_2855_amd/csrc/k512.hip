// Kernels for N = 512 (FP32 and FP64 forms).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_512f() { return make_launchers<S512, float>(); }
const Launchers* launchers_512d() { return make_launchers<D512, double>(); }
}  // namespace lsr
