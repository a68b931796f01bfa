// Kernels for N = 4096 (FP32 form only).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_4096f() { return make_launchers<S4096, float>(); }
}  // namespace lsr
