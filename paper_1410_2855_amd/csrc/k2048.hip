// Kernels for N = 2048 (FP32 and FP64 forms).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_2048f() { return make_launchers<S2048, float>(); }
const Launchers* launchers_2048d() { return make_launchers<D2048, double>(); }
}  // namespace lsr
