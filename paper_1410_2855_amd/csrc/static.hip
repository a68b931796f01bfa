// static.hip -- the round trips of one cavity without a plan and without any
// allocation: the FP64-built tables, the per-row-block partial sums and the
// counters live in a file-scope device array, set up by a kernel at the start
// of every call.  For callers that cannot allocate device memory.
#include <cmath>
#include <mutex>

#include "host.hpp"

namespace lsr {

// The scratch array: each device the library runs on holds one copy until
// the process ends.  Host code never passes the array's name to a kernel or a
// copy: it passes the device address hipGetSymbolAddress returned for the
// current device (scratch_ptr).
static constexpr size_t kScratchBytes = 512 * 1024;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of the scratch array (looked up once
// per device, with that device current).
static int scratch_ptr(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return set_err(LSR_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_err(LSR_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch[dev]);
    return LSR_OK;
}

static constexpr double kTwoPiD = 6.283185307179586476925286766559;

// Where the tables sit inside the scratch array (byte offsets, 256-aligned).
struct StaticLayout {
    size_t counters, trace, partials, tw, hx, pump, foc, total;
};

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

static StaticLayout static_layout(const ShapeInfo& s, int N) {
    StaticLayout l{};
    l.counters = 0;
    l.trace = up256(l.counters + sizeof(unsigned) * CNT_WORDS);
    l.partials = up256(l.trace + 4 * sizeof(double));
    l.tw = up256(l.partials + 4 * sizeof(double) * (size_t)(N / s.LPW));
    l.hx = up256(l.tw + 2 * sizeof(float) * (size_t)s.tw_total);
    l.pump = up256(l.hx + 2 * sizeof(float) * (size_t)N);
    l.foc = up256(l.pump + sizeof(float) * (size_t)N);
    l.total = up256(l.foc + 2 * sizeof(float) * (size_t)N);
    return l;
}

// The tables of one call, built in FP64 and rounded to FP32 exactly as the
// plan's host builders do (the same formulas, angles reduced in turns), and
// the counters cleared.  Thread g covers twiddle entry g and axis index g.
struct StaticArgs {
    ShapeInfo s;
    int N;
    double dx, lambda, L, F, period;
    int modulated, curved;
    unsigned char* base;
    StaticLayout lay;
};

__global__ __launch_bounds__(256) void k_static_setup(StaticArgs a) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    unsigned* counters = reinterpret_cast<unsigned*>(a.base + a.lay.counters);
    if (g < CNT_WORDS) counters[g] = 0u;
    if (g < a.s.tw_total) {
        // the segment of twiddle entry g: forward passes, then inverse passes
        int at = g, dir = FWD, ns = 1, R = 0;
        bool found = false;
        for (int d = 0; d < 2 && !found; ++d) {
            dir = d == 0 ? FWD : INV;
            ns = 1;
            for (int p = 0; p < a.s.NP && !found; ++p) {
                R = dir == FWD ? a.s.rad[p] : a.s.rad[a.s.NP - 1 - p];
                if (ns > 1) {
                    if (at < ns * R) found = true;
                    else at -= ns * R;
                }
                if (!found) ns *= R;
            }
        }
        int k, r;
        if (R % 2 == 0) {
            // pair layout: (r/2) 2 ns + 2k + r%2
            const int rem = at % (2 * ns);
            r = 2 * (at / (2 * ns)) + rem % 2;
            k = rem / 2;
        } else {
            r = at / ns;
            k = at % ns;
        }
        const double th = kTwoPiD * (double)((long)r * k) / (double)((long)ns * R);
        float* tw = reinterpret_cast<float*>(a.base + a.lay.tw);
        tw[2 * g] = (float)cos(th);
        tw[2 * g + 1] = (float)(dir * sin(th));
    }
    if (g < a.N) {
        const int N = a.N;
        const double q = (double)(2 * g < N ? g : g - N);
        const double W = (double)N * a.dx;
        const double t = a.lambda * a.L * q * q / (2.0 * W * W);
        const double f = t - floor(t);
        float* hx = reinterpret_cast<float*>(a.base + a.lay.hx);
        hx[2 * g] = (float)(cos(kTwoPiD * f) / N);
        hx[2 * g + 1] = (float)(-sin(kTwoPiD * f) / N);
        const double x = (g - 0.5 * N) * a.dx;
        if (a.modulated) {
            const double u = x / a.period;
            reinterpret_cast<float*>(a.base + a.lay.pump)[g] = (float)cos(kTwoPiD * (u - floor(u)));
        }
        if (a.curved) {
            const double v = x * x / (2.0 * a.lambda * a.F);
            const double fv = v - floor(v);
            float* foc = reinterpret_cast<float*>(a.base + a.lay.foc);
            foc[2 * g] = (float)cos(kTwoPiD * fv);
            foc[2 * g + 1] = (float)sin(kTwoPiD * fv);
        }
    }
}

}  // namespace lsr

using namespace lsr;

extern "C" int lsr_roundtrips_static(int N, double dx, double lambda, double L, double F, double R,
                                     const lsr_aperture* ap, double N0, double T1, double mod_amp,
                                     double mod_period, int model, void* E, void* Ninv, int n_trips,
                                     double* trace, void* stream) {
    if (!(dx > 0) || !std::isfinite(dx) || !(lambda > 0) || !std::isfinite(lambda) || !(L >= 0) ||
        !std::isfinite(L) || !(R > 0) || !(R <= 1) || std::isnan(F))
        return set_err(LSR_EINVAL, "bad cavity parameters");
    if (!std::isfinite(N0) || !(T1 > 0) || !std::isfinite(T1) || !std::isfinite(mod_amp) || !(mod_period >= 0) ||
        !std::isfinite(mod_period))
        return set_err(LSR_EINVAL, "bad gain parameters");
    if (model < LSR_MODEL_B_EULER || model > LSR_MODEL_CLASS_A) return set_err(LSR_EINVAL, "model %d out of range", model);
    if (n_trips < 0) return set_err(LSR_EINVAL, "n_trips < 0");
    if (!E || !Ninv || ((uintptr_t)E & 15u) || ((uintptr_t)Ninv & 15u))
        return set_err(LSR_EINVAL, "E and Ninv must be 16-byte aligned device pointers");
    if (trace && ((uintptr_t)trace & 7u)) return set_err(LSR_EINVAL, "trace must be 8-byte aligned");
    lsr_aperture a{};
    if (ap) a = *ap;
    if (a.kind < 0 || a.kind > 3) return set_err(LSR_EINVAL, "aperture kind %d", a.kind);
    if ((a.kind == 1 || a.kind == 2) && !(a.radius > 0 && std::isfinite(a.radius)))
        return set_err(LSR_EINVAL, "aperture radius must be > 0");
    if (a.kind == 1 && (a.order < 2 || a.order % 2 != 0 || a.order > 64))
        return set_err(LSR_EINVAL, "super-Gaussian order must be even in [2, 64]");
    if (a.kind == 3 && (!a.mask || ((uintptr_t)a.mask & 15u)))
        return set_err(LSR_EINVAL, "mask must be a 16-byte aligned device pointer");
    const Launchers* k = launchers_for(N, false);
    ShapeInfo s;
    if (!k || !shape_for(N, false, &s)) return set_err(LSR_EUNSUPPORTED, "N=%d is not compiled in", N);
    const StaticLayout lay = static_layout(s, N);
    if (lay.total > kScratchBytes)
        return set_err(LSR_EINVAL, "N=%d needs %zu bytes of scratch, more than the %zu the library holds", N,
                       lay.total, kScratchBytes);
    if (n_trips == 0) return LSR_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_err(LSR_EDEVICE, "no HIP device");
    unsigned char* base = nullptr;
    int rc = scratch_ptr(dev, &base);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);

    const bool modulated = mod_amp != 0.0 && mod_period > 0.0;
    const bool curved = F != 0.0 && std::isfinite(F);
    StaticArgs sa{};
    sa.s = s;
    sa.N = N;
    sa.dx = dx;
    sa.lambda = lambda;
    sa.L = L;
    sa.F = F;
    sa.period = mod_period;
    sa.modulated = modulated;
    sa.curved = curved;
    sa.base = base;
    sa.lay = lay;
    const int threads = s.tw_total > N ? s.tw_total : N;
    hipLaunchKernelGGL(k_static_setup, dim3((threads + 255) / 256), dim3(256), 0, st, sa);
    if (hipGetLastError() != hipSuccess) return set_err(LSR_EDEVICE, "setup kernel launch failed");

    // the descriptor of a plan of the same parameters, its tables and
    // scratch in the array
    CavDesc d{};
    d.E = E;
    d.Ninv = Ninv;
    d.tw = base + lay.tw;
    d.hx = base + lay.hx;
    d.pump_c = modulated ? base + lay.pump : nullptr;
    d.foc = curved ? base + lay.foc : nullptr;
    d.mask = a.kind == 3 ? a.mask : nullptr;
    d.rough = nullptr;
    d.scratch = nullptr;
    d.partials = reinterpret_cast<double*>(base + lay.partials);
    d.radial_part = nullptr;
    d.trace = trace ? trace : reinterpret_cast<double*>(base + lay.trace);
    d.counters = reinterpret_cast<unsigned*>(base + lay.counters);
    d.N = N;
    d.prec = PREC_FP64TAB;
    d.ap_kind = a.kind;
    d.ap_half_order = a.kind == 1 ? a.order / 2 : 1;
    d.trace_cap = trace ? n_trips : 1;
    d.nrb = N / s.LPW;
    d.nbins = (int)floor(N / sqrt(2.0) + 0.5) + 1;
    d.prop_kind = 0;
    d.model = model;
    d.sqrtR = sqrt(R);
    d.N0 = N0;
    d.inv_T1 = 1.0 / T1;
    d.mod_amp = modulated ? mod_amp : 0.0;
    d.dx = dx;
    d.ap_step = aperture_step(a.kind, a.radius, d.ap_half_order, dx);
    d.phase_c = kTwoPiD * 0.5 * lambda * L / ((N * dx) * (N * dx));
    d.inv_nn = 1.0 / ((double)N * (double)N);

    // the launch sequence of lsr_roundtrips for one gain sheet
    rc = k->row(d, ROW_FIRST, st);
    for (int t = 0; t < n_trips && rc == 0; ++t) {
        rc = k->col(d, COL_PROP, st);
        if (rc == 0) rc = k->row(d, t + 1 == n_trips ? ROW_LAST : ROW_MID, st);
    }
    if (rc != 0) return set_err(LSR_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    return LSR_OK;
}
