// Kernels for N = 384 (FP32 and FP64 forms).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_384f() { return make_launchers<S384, float>(); }
const Launchers* launchers_384d() { return make_launchers<D384, double>(); }
}  // namespace lsr
