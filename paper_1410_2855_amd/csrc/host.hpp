// host.hpp -- host-side plan object, error reporting and table builders.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lsr.h"
#include "desc.hpp"
#include "launch.hpp"

namespace lsr {

int set_err(int code, const char* fmt, ...);

// hipMalloc for every device allocation of the library, so that a test can
// force a failure from the host (lsr_test_fail_alloc).
hipError_t dev_malloc(void** p, size_t bytes);

#define LSR_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::lsr::set_err(LSR_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Keeps the caller's current device and restores it on scope exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// FP64 (or FP32-emulating) table builders; pure host arithmetic.
// interleaved re, im; pairs: layout of complex FP32 tables (tw_index)
std::vector<double> build_twiddles(const ShapeInfo& s, bool fp32_arith, bool pairs);
std::vector<double> build_hx(int N, double dx, double lambda, double L);
std::vector<double> build_filter(int N, double dx, double delta);   // interleaved, 1/N folded
std::vector<double> build_pump_cos(int N, double dx, double period);
std::vector<double> build_focal(int N, double dx, double lambda, double F); // interleaved

struct lsr_plan_impl;

}  // namespace lsr

struct lsr_plan_s {
    int device = 0;
    int N = 0;
    int prec = 0;
    double dx = 0, lambda = 0, L = 0, F = 0, R = 1;
    lsr_aperture ap{};
    double N0 = 0, T1 = 1, mod_amp = 0, mod_period = 0;
    double filter = 0;                 // > 0: width of the real filter replacing the propagator
    int model = 0;                     // lsr_model
    int slices = 1;                    // thin gain sheets per round trip
    int fft_plan = 0;                  // one-cavity FFT plan (0 default shape, 1 eight points per lane)
    unsigned version = 0;              // bumped whenever the descriptor d changes
    hipStream_t stream = nullptr;
    const lsr::Launchers* kern = nullptr;
    lsr::ShapeInfo shape{};
    lsr::CavDesc d{};          // template descriptor; E/Ninv filled per call
    // owned device memory
    void* d_tw = nullptr;
    void* d_hx = nullptr;
    void* d_pump = nullptr;
    void* d_foc = nullptr;
    void* d_hz = nullptr;            // propagator table of the last lsr_propagate distance
    void* d_hs = nullptr;            // nonlocal step between two of several gain sheets
    void* d_rough = nullptr;         // exp(i psi) of the mirror roughness, N*N complex, or null
    void* d_trans = nullptr;         // general transfer function, N*N complex by column, or null
    double* d_partials = nullptr;
    double* d_trace = nullptr;
    unsigned* d_counters = nullptr;
    void* d_scratch = nullptr;       // lazily, for lsr_diag
    double* d_radial_part = nullptr; // lazily
    double* d_diag_out = nullptr;    // lazily
    int trace_cap = 0;
    unsigned long long trips_done = 0;   // host shadow of counters[CNT_TRIPS]
    int last_n = 0;
    size_t real_bytes() const { return prec == lsr::PREC_FP64 ? 8 : 4; }
};

namespace lsr {
// Descriptor of gain sheet k (of the plan's m) for a call on (E, Ninv): the
// sheet's inversion, pump N0/m and step table; the mirror, aperture and
// roughness on sheet 0 only (plan.hip).
CavDesc plan_sheet_desc(const lsr_plan_s* p, void* E, void* Ninv, int k);
}  // namespace lsr
