// Kernels for N = 768 (FP32 and FP64 forms).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_768f() { return make_launchers<S768, float>(); }
const Launchers* launchers_768d() { return make_launchers<D768, double>(); }
}  // namespace lsr
