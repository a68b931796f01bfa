// launch.hpp -- host-side registry of the compiled grid sizes.
#pragma once

#include <hip/hip_runtime.h>

#include "desc.hpp"
#include "shapes.hpp"

namespace lsr {

struct Launchers {
    int (*row)(const CavDesc&, int mode, hipStream_t);
    int (*col)(const CavDesc&, int mode, hipStream_t);
    ShapeInfo shape;
};

// nullptr if grid size N is not compiled in for the precision class.
const Launchers* launchers_for(int N, bool fp64);

// One-cavity FFT plan k > 0 of the FP32 forms for size N (k = 1: 8 points
// per lane), or nullptr where none is compiled.
const Launchers* launchers_alt(int N, int k);

// Shape of N without touching HIP (table builders, introspection).
bool shape_for(int N, bool fp64, ShapeInfo* out);

}  // namespace lsr
