// Kernels for N = 4096 (FP32 and FP64 forms).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_4096f() { return make_launchers<S4096, float>(); }
const Launchers* launchers_4096d() { return make_launchers<D4096, double>(); }
}  // namespace lsr
