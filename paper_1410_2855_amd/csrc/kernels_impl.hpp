// kernels_impl.hpp -- one-cavity kernels (row pass, column pass, diagnostics)
// and their launchers, instantiated per grid size by the k*.hip units.
#pragma once

#include "launch.hpp"
#include "map.hpp"

namespace lsr {

// Waves per SIMD the register allocation of a one-cavity kernel must allow:
// those of the workgroups a launch places on one of the 256 CUs, as far as
// they fit in LDS (at most four waves).  A lone 2048^2 cavity launches two
// workgroups per CU, and its row kernel, wanting 130 registers, would
// otherwise run them one after the other (51.5 -> 43.5 us per trip); where a
// launch brings one workgroup per CU or fewer, the compiler keeps its choice
// (a tighter budget spills there for nothing).
template <class S, typename T>
constexpr int one_cavity_wpe() {
    constexpr int lds = S::LDS_ELEMS * (int)sizeof(cx<T>) + 4 * 16 * 8;
    constexpr int fit = 160 * 1024 / lds;
    constexpr int per_cu = S::N / S::LPW / 256;
    constexpr int wgs = per_cu < fit ? per_cu : fit;
    constexpr int waves = wgs * (S::THREADS / 64) / 4;
    return waves < 1 ? 1 : waves > 4 ? 4 : waves;
}

template <class S, typename T, int MODE, int MODEL = 0>
__global__ __launch_bounds__(S::THREADS) __attribute__((amdgpu_waves_per_eu(one_cavity_wpe<S, T>(), 8)))
void k_row(CavDesc d) {
    __shared__ cx<T> lds[S::LDS_ELEMS];
    __shared__ double red[4 * 16];
    row_task<S, T, MODE, MODEL>(d, blockIdx.x, lds, red);
}

template <class S, typename T, int MODE, int PROP>
__global__ __launch_bounds__(S::THREADS) __attribute__((amdgpu_waves_per_eu(one_cavity_wpe<S, T>(), 8)))
void k_col(CavDesc d) {
    __shared__ cx<T> lds[S::LDS_ELEMS];
    if constexpr (MODE == COL_PROP) {
        // the row pass of this trip is complete (stream order): fold its
        // per-block sums into the trace ring
        if (blockIdx.x == 0 && threadIdx.x < 64) finalize_sums(d);
    }
    col_task<S, T, MODE, PROP>(d, blockIdx.x, lds);
}

template <class S, typename T, int MODEL>
int launch_row_m(const CavDesc& d, int mode, hipStream_t st) {
    const dim3 g(S::N / S::LPW), b(S::THREADS);
    switch (mode) {
    case ROW_FIRST: hipLaunchKernelGGL((k_row<S, T, ROW_FIRST, MODEL>), g, b, 0, st, d); break;
    case ROW_MID:   hipLaunchKernelGGL((k_row<S, T, ROW_MID, MODEL>), g, b, 0, st, d); break;
    case ROW_LAST:  hipLaunchKernelGGL((k_row<S, T, ROW_LAST>), g, b, 0, st, d); break;   // no local step
    case ROW_DIAG:  hipLaunchKernelGGL((k_row<S, T, ROW_DIAG, MODEL>), g, b, 0, st, d); break;
    case ROW_FWD:   hipLaunchKernelGGL((k_row<S, T, ROW_FWD>), g, b, 0, st, d); break;     // no local step
    default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class S, typename T>
int launch_row_t(const CavDesc& d, int mode, hipStream_t st) {
    // the roughness kernels read d.rough without a check
    if (((d.model & MODEL_ROUGH) != 0) != (d.rough != nullptr)) return -1;
    switch (d.model) {
    case 0: return launch_row_m<S, T, 0>(d, mode, st);
    case 1: return launch_row_m<S, T, 1>(d, mode, st);
    case 2: return launch_row_m<S, T, 2>(d, mode, st);
    case MODEL_ROUGH + 0: return launch_row_m<S, T, MODEL_ROUGH + 0>(d, mode, st);
    case MODEL_ROUGH + 1: return launch_row_m<S, T, MODEL_ROUGH + 1>(d, mode, st);
    case MODEL_ROUGH + 2: return launch_row_m<S, T, MODEL_ROUGH + 2>(d, mode, st);
    default: return -1;
    }
}

template <class S, typename T>
int launch_col_t(const CavDesc& d, int mode, hipStream_t st) {
    const dim3 g(S::N / S::LPW), b(S::THREADS);
    switch (mode) {
    case COL_PROP:
        // the plain form evaluates the Fresnel phase on the device; a filter
        // (or any FP64-built propagator) comes from the table; a general
        // transfer function from its own N x N table
        if (d.prop_kind == 2) {
            if (!d.trans) return -1;
            hipLaunchKernelGGL((k_col<S, T, COL_PROP, PROP_TRANS>), g, b, 0, st, d);
        } else if (d.prec == PREC_PLAIN && d.prop_kind == 0) {
            hipLaunchKernelGGL((k_col<S, T, COL_PROP, PROP_PHASE>), g, b, 0, st, d);
        } else {
            hipLaunchKernelGGL((k_col<S, T, COL_PROP, PROP_TABLE>), g, b, 0, st, d);
        }
        break;
    case COL_DIAG: hipLaunchKernelGGL((k_col<S, T, COL_DIAG, PROP_TABLE>), g, b, 0, st, d); break;
    case COL_FREE:
        if (d.prec == PREC_PLAIN && d.prop_kind == 0) hipLaunchKernelGGL((k_col<S, T, COL_FREE, PROP_PHASE>), g, b, 0, st, d);
        else hipLaunchKernelGGL((k_col<S, T, COL_FREE, PROP_TABLE>), g, b, 0, st, d);
        break;
    default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class S, typename T>
const Launchers* make_launchers() {
    static const Launchers L{&launch_row_t<S, T>, &launch_col_t<S, T>, shape_info<S>()};
    return &L;
}

}  // namespace lsr
