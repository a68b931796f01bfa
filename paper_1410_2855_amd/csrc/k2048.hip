// Kernels for N = 2048 (FP32 and FP64 forms, and the one-cavity shape with
// a wave per line).
#include "kernels_impl.hpp"

namespace lsr {
const Launchers* launchers_2048f() { return make_launchers<S2048, float>(); }
const Launchers* launchers_2048d() { return make_launchers<D2048, double>(); }
const Launchers* launchers_2048w() { return make_launchers<L2048w, float>(); }
}  // namespace lsr
