// registry.cpp -- grid size -> compiled kernels / shapes.
#include "launch.hpp"

namespace lsr {

#define LSR_DECL(n) const Launchers* launchers_##n##f(); const Launchers* launchers_##n##d();
LSR_DECL(256) LSR_DECL(384) LSR_DECL(512) LSR_DECL(768) LSR_DECL(1024) LSR_DECL(2048) LSR_DECL(4096)
#undef LSR_DECL
const Launchers* launchers_256l();
const Launchers* launchers_256q();
const Launchers* launchers_256p();
const Launchers* launchers_2048w();

const Launchers* launchers_alt(int N, int k) {
    if (N == 2048) return k == 1 ? launchers_2048w() : nullptr;
    if (N != 256) return nullptr;
    switch (k) {
    case 1:  return launchers_256l();
    case 2:  return launchers_256q();
    case 3:  return launchers_256p();
    default: return nullptr;
    }
}

const Launchers* launchers_for(int N, bool fp64) {
    switch (N) {
    case 256:  return fp64 ? launchers_256d() : launchers_256f();
    case 384:  return fp64 ? launchers_384d() : launchers_384f();
    case 512:  return fp64 ? launchers_512d() : launchers_512f();
    case 768:  return fp64 ? launchers_768d() : launchers_768f();
    case 1024: return fp64 ? launchers_1024d() : launchers_1024f();
    case 2048: return fp64 ? launchers_2048d() : launchers_2048f();
    case 4096: return fp64 ? launchers_4096d() : launchers_4096f();
    default:   return nullptr;
    }
}

bool shape_for(int N, bool fp64, ShapeInfo* out) {
    ShapeInfo s{};
    switch (N) {
    case 256:  s = fp64 ? shape_info<D256>() : shape_info<S256>(); break;
    case 384:  s = fp64 ? shape_info<D384>() : shape_info<S384>(); break;
    case 512:  s = fp64 ? shape_info<D512>() : shape_info<S512>(); break;
    case 768:  s = fp64 ? shape_info<D768>() : shape_info<S768>(); break;
    case 1024: s = fp64 ? shape_info<D1024>() : shape_info<S1024>(); break;
    case 2048: s = fp64 ? shape_info<D2048>() : shape_info<S2048>(); break;
    case 4096: s = fp64 ? shape_info<D4096>() : shape_info<S4096>(); break;
    default:   return false;
    }
    if (out) *out = s;
    return true;
}

}  // namespace lsr
