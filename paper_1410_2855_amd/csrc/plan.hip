// plan.hip -- one-cavity plans: FP64 table building on the host, the
// launch sequence of a run of round trips, diagnostics, error reporting.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <vector>

#include "host.hpp"

namespace lsr {

static thread_local char g_err[512] = "";

int set_err(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

// Allocations left before a forced failure (-1: none forced).
static std::atomic<int> g_fail_after{-1};

hipError_t dev_malloc(void** p, size_t bytes) {
    int left = g_fail_after.load();
    while (left >= 0 && !g_fail_after.compare_exchange_weak(left, left - 1)) {
    }
    if (left == 0) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

static constexpr double kTwoPi = 6.283185307179586476925286766559;

static int sidx(int q, int n) { return (2 * q < n) ? q : q - n; }

// Stockham twiddles, forward passes then inverse passes; for a pass of radix
// R and sub-length Ns > 1: entry k*R + r = exp(dir 2 pi i r k / (Ns R)).
// The angle's integer part r*k < Ns*R is exact, so no further reduction is
// needed; fp32_arith evaluates the angle and cos/sin in single precision.
std::vector<double> build_twiddles(const ShapeInfo& s, bool fp32_arith, bool pairs) {
    std::vector<double> out;
    for (int dir : {FWD, INV}) {
        int ns = 1;
        for (int p = 0; p < s.NP; ++p) {
            const int R = (dir == FWD) ? s.rad[p] : s.rad[s.NP - 1 - p];
            if (ns > 1) {
                const size_t seg = out.size();
                out.resize(seg + 2 * (size_t)ns * R);
                for (int k = 0; k < ns; ++k)
                    for (int r = 0; r < R; ++r) {
                        const long m = (long)r * k;
                        const long n = (long)ns * R;
                        double c, sn;
                        if (fp32_arith) {
                            const float th = 6.28318530717958647692f * (float)m / (float)n;
                            c = (double)cosf(th);
                            sn = (double)sinf(th);
                        } else {
                            const double th = kTwoPi * (double)m / (double)n;
                            c = cos(th);
                            sn = sin(th);
                        }
                        const size_t at = seg + 2 * (size_t)tw_index(ns, R, k, r, pairs);
                        out[at] = c;
                        out[at + 1] = dir * sn;
                    }
            }
            ns *= R;
        }
    }
    return out;
}

// hx(p) = exp(-i pi lambda L fx_p^2) / N with fx_p = p~/(N dx): the phase in
// turns t = lambda L p~^2 / (2 (N dx)^2) is reduced to [0, 1) in FP64 before
// cos/sin, so the table stays accurate where the phase reaches ~1e3 turns.
std::vector<double> build_hx(int N, double dx, double lambda, double L) {
    std::vector<double> out(2 * (size_t)N);
    const double W = (double)N * dx;
    for (int p = 0; p < N; ++p) {
        const double q = (double)sidx(p, N);
        const double t = lambda * L * q * q / (2.0 * W * W);
        const double f = t - floor(t);
        out[2 * p] = cos(kTwoPi * f) / N;
        out[2 * p + 1] = -sin(kTwoPi * f) / N;
    }
    return out;
}

// Real renormalization-group filter of deviation delta (Sec. 2.3, Eq. (18)),
// exp[(delta^2/2) d^2/dx^2] per axis: hf(p) = exp(-2 pi^2 delta^2 fx_p^2) / N,
// zero imaginary part; the same separable form and 1/N folding as hx.
std::vector<double> build_filter(int N, double dx, double delta) {
    std::vector<double> out(2 * (size_t)N, 0.0);
    const double W = (double)N * dx;
    for (int p = 0; p < N; ++p) {
        const double f = (double)sidx(p, N) / W;
        out[2 * p] = exp(-0.5 * kTwoPi * kTwoPi * delta * delta * f * f) / N;
    }
    return out;
}

// cos(2 pi x_i / d), x_i = (i - N/2) dx, argument reduced to [0, 1) turns.
std::vector<double> build_pump_cos(int N, double dx, double period) {
    std::vector<double> out((size_t)N);
    for (int i = 0; i < N; ++i) {
        const double t = (i - 0.5 * N) * dx / period;
        out[i] = cos(kTwoPi * (t - floor(t)));
    }
    return out;
}

// exp(i k x_i^2 / (2F)) = exp(2 pi i x_i^2/(2 lambda F)), reduced in turns;
// the 2D mirror phase exp(i k r^2/(2F)) is the product of the x and y factors.
std::vector<double> build_focal(int N, double dx, double lambda, double F) {
    std::vector<double> out(2 * (size_t)N);
    for (int i = 0; i < N; ++i) {
        const double x = (i - 0.5 * N) * dx;
        const double t = x * x / (2.0 * lambda * F);
        const double f = t - floor(t);
        out[2 * i] = cos(kTwoPi * f);
        out[2 * i + 1] = sin(kTwoPi * f);
    }
    return out;
}

static int upload(void** dst, const std::vector<double>& v, bool as_float) {
    const size_t n = v.size();
    if (n == 0) { *dst = nullptr; return LSR_OK; }
    const size_t bytes = n * (as_float ? sizeof(float) : sizeof(double));
    if (dev_malloc(dst, bytes) != hipSuccess) {
        *dst = nullptr;
        (void)hipGetLastError();
        return set_err(LSR_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    if (as_float) {
        std::vector<float> f(n);
        for (size_t i = 0; i < n; ++i) f[i] = (float)v[i];
        LSR_HIP(hipMemcpy(*dst, f.data(), bytes, hipMemcpyHostToDevice));
    } else {
        LSR_HIP(hipMemcpy(*dst, v.data(), bytes, hipMemcpyHostToDevice));
    }
    return LSR_OK;
}

template <typename P>
static int dalloc(P** dst, size_t bytes) {
    void* p = nullptr;
    if (dev_malloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return set_err(LSR_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    *dst = static_cast<P*>(p);
    return LSR_OK;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

static void free_plan_memory(lsr_plan_s* p) {
    void* bufs[] = {p->d_tw, p->d_hx, p->d_pump, p->d_foc, p->d_partials, p->d_trace,
                    p->d_counters, p->d_scratch, p->d_radial_part, p->d_diag_out, p->d_hz,
                    p->d_hs, p->d_rough, p->d_trans};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
}

// Records kept in a plan's trace ring ($LSR_TRACE_CAP, default 8192).
static int trace_capacity() {
    const char* s = getenv("LSR_TRACE_CAP");
    long v = s ? strtol(s, nullptr, 10) : 8192;
    if (v < 1) v = 1;
    if (v > (1L << 24)) v = 1L << 24;
    return (int)v;
}

// Ordered reduction of the diagnostics partials: out[0..3] the four sums,
// out[4 + k] radial bin k.
__global__ __launch_bounds__(256) void k_diag_reduce(const double* __restrict__ partials, int nrb,
                                                     const double* __restrict__ radial, int nbins,
                                                     double* __restrict__ out) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g < nbins) {
        double s = 0.0;
        for (int cb = 0; cb < nrb; ++cb) s += radial[(size_t)cb * nbins + g];
        out[4 + g] = s;
    }
    if (blockIdx.x == 0 && threadIdx.x < 4) {
        double s = 0.0;
        for (int rb = 0; rb < nrb; ++rb) s += partials[4 * rb + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

int launch_diag_reduce(const CavDesc& d, double* out, hipStream_t st) {
    const int blocks = (d.nbins + 255) / 256;
    hipLaunchKernelGGL(k_diag_reduce, dim3(blocks), dim3(256), 0, st, d.partials, d.nrb,
                       d.radial_part, d.nbins, out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Table of the nonlocal step between two of m > 1 gain sheets: the propagator
// over L/m (FP64TAB, FP64) or the filter of variance delta^2/m, whose m steps
// compose to the whole filter.  The plain Fresnel form evaluates its phase on
// the device and has no table.
static int build_sheet_table(const lsr_plan_s* p, int m, double filter, void** out) {
    *out = nullptr;
    if (m <= 1) return LSR_OK;
    if (filter > 0) return upload(out, build_filter(p->N, p->dx, filter / std::sqrt((double)m)), p->prec != PREC_FP64);
    if (p->prec == PREC_PLAIN) return LSR_OK;
    return upload(out, build_hx(p->N, p->dx, p->lambda, p->L / m), p->prec != PREC_FP64);
}

// Descriptor of gain sheet k of the plan's m for a call on (E, Ninv).  Sheet 0
// is the mirror plane (reflectivity, curvature, aperture); the others apply
// gain only and hold their inversion k N^2 elements further on.  Every sheet
// has pump N0/m and steps over L/m.
static CavDesc sheet_desc(const lsr_plan_s* p, void* E, void* Ninv, int k) {
    CavDesc d = p->d;
    d.E = E;
    d.Ninv = Ninv;
    const int m = p->slices;
    if (m == 1) return d;
    d.hx = p->d_hs;
    d.phase_c = p->d.phase_c / m;
    d.N0 = p->d.N0 / m;
    if (k > 0) {
        d.Ninv = static_cast<char*>(Ninv) + (size_t)k * (size_t)p->N * (size_t)p->N * p->real_bytes();
        d.sqrtR = 1.0;
        d.ap_kind = AP_NONE;
        d.mask = nullptr;
        d.foc = nullptr;
        d.rough = nullptr;
        d.model &= MODEL_MASK;
    }
    return d;
}

CavDesc plan_sheet_desc(const lsr_plan_s* p, void* E, void* Ninv, int k) { return sheet_desc(p, E, Ninv, k); }

// The launches of n >= 1 round trips, in order: the first row pass, then per
// trip and sheet the column pass and the row pass of the next sheet; the last
// row pass only finishes the inverse transform.  Sheet 0's column pass folds
// the trip's sums into the trace ring, the other sheets' passes do not.
// launch(desc, is_row, mode) returns 0 or a launcher error.
template <class F>
static int for_each_launch(const lsr_plan_s* p, void* E, void* Ninv, int n_trips, F&& launch) {
    const int m = p->slices;
    int rc = launch(sheet_desc(p, E, Ninv, 0), true, ROW_FIRST);
    for (int t = 0; t < n_trips && rc == 0; ++t)
        for (int k = 0; k < m && rc == 0; ++k) {
            rc = launch(sheet_desc(p, E, Ninv, k), false, k == 0 ? COL_PROP : COL_FREE);
            const bool last = t + 1 == n_trips && k + 1 == m;
            if (rc == 0) rc = launch(sheet_desc(p, E, Ninv, last ? 0 : (k + 1) % m), true, last ? ROW_LAST : ROW_MID);
        }
    return rc;
}

}  // namespace lsr

using namespace lsr;

extern "C" {

const char* lsr_last_error(void) { return g_err; }

int lsr_test_fail_alloc(int after) {
    if (after < -1) return set_err(LSR_EINVAL, "after must be >= -1");
    g_fail_after.store(after);
    return LSR_OK;
}

const char* lsr_version(void) { return "lsr 0.1.0 gfx950"; }

int lsr_supported(int N, int prec) {
    if (prec < 0 || prec > 2) return 0;
    return shape_for(N, prec == PREC_FP64, nullptr) ? 1 : 0;
}

int lsr_fft_shape(int N, int prec, int* radices, int max, int* lanes_per_line, int* lines_per_group) {
    ShapeInfo s;
    if (prec < 0 || prec > 2) return set_err(LSR_EINVAL, "prec %d out of range", prec);
    if (!shape_for(N, prec == PREC_FP64, &s)) return set_err(LSR_EUNSUPPORTED, "N=%d not compiled in", N);
    if (radices)
        for (int i = 0; i < s.NP && i < max; ++i) radices[i] = s.rad[i];
    if (lanes_per_line) *lanes_per_line = s.L;
    if (lines_per_group) *lines_per_group = s.LPW;
    return s.NP;
}

int lsr_propagator_table(int N, double dx, double lambda, double L, float* out) {
    if (N < 1 || !(dx > 0) || !(lambda > 0) || !(L >= 0) || !out)
        return set_err(LSR_EINVAL, "bad propagator-table arguments");
    std::vector<double> h = build_hx(N, dx, lambda, L);
    for (size_t i = 0; i < h.size(); ++i) out[i] = (float)h[i];
    return LSR_OK;
}

int lsr_twiddle_table(int N, int prec, float* out, int capacity) {
    ShapeInfo s;
    if (prec < 0 || prec > 2) return set_err(LSR_EINVAL, "prec %d out of range", prec);
    if (!shape_for(N, prec == PREC_FP64, &s)) return set_err(LSR_EUNSUPPORTED, "N=%d not compiled in", N);
    std::vector<double> t = build_twiddles(s, prec == PREC_PLAIN, prec != PREC_FP64);
    const int n = (int)(t.size() / 2);
    if (!out) return n;
    if (capacity < n) return set_err(LSR_EINVAL, "capacity %d < %d twiddles", capacity, n);
    for (size_t i = 0; i < t.size(); ++i) out[i] = (float)t[i];
    return n;
}

int lsr_plan_create(lsr_plan* out, int N, double dx, double lambda, double L, double F, double R,
                    const lsr_aperture* ap, lsr_prec prec) {
    if (!out) return set_err(LSR_EINVAL, "out is NULL");
    *out = nullptr;
    if ((int)prec < 0 || (int)prec > 2) return set_err(LSR_EINVAL, "prec %d out of range", (int)prec);
    if (!(dx > 0) || !std::isfinite(dx)) return set_err(LSR_EINVAL, "dx must be > 0");
    if (!(lambda > 0) || !std::isfinite(lambda)) return set_err(LSR_EINVAL, "lambda must be > 0");
    if (!(L >= 0) || !std::isfinite(L)) return set_err(LSR_EINVAL, "L must be >= 0");
    if (!(R > 0) || !(R <= 1)) return set_err(LSR_EINVAL, "R must lie in (0, 1]");
    if (std::isnan(F)) return set_err(LSR_EINVAL, "F is NaN");
    lsr_aperture a{};
    if (ap) a = *ap;
    if (a.kind < 0 || a.kind > 3) return set_err(LSR_EINVAL, "aperture kind %d", a.kind);
    if ((a.kind == 1 || a.kind == 2) && !(a.radius > 0 && std::isfinite(a.radius)))
        return set_err(LSR_EINVAL, "aperture radius must be > 0");
    if (a.kind == 1 && (a.order < 2 || a.order % 2 != 0 || a.order > 64))
        return set_err(LSR_EINVAL, "super-Gaussian order must be even in [2, 64]");
    if (a.kind == 3 && (!a.mask || !aligned16(a.mask))) return set_err(LSR_EINVAL, "mask must be a 16-byte aligned device pointer");
    const Launchers* k = launchers_for(N, prec == LSR_PREC_FP64);
    if (!k) return set_err(LSR_EUNSUPPORTED, "N=%d is not compiled in for prec %d", N, (int)prec);

    lsr_plan_s* p = new (std::nothrow) lsr_plan_s();
    if (!p) return set_err(LSR_ENOMEM, "host allocation failed");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete p;
        return set_err(LSR_EDEVICE, "no HIP device");
    }
    p->device = dev;
    p->N = N;
    p->prec = (int)prec;
    p->dx = dx;
    p->lambda = lambda;
    p->L = L;
    p->F = F;
    p->R = R;
    p->ap = a;
    p->kern = k;
    p->shape = k->shape;
    p->trace_cap = trace_capacity();
    const bool f32 = prec != LSR_PREC_FP64;
    const int nrb = N / p->shape.LPW;
    // row blocks of the narrowest shape a plan of this size can take (lines
    // per workgroup >= 2), so the partials and spectrum scratch fit any
    const int nrb_max = N / 2;
    int rc = LSR_OK;
    auto fail = [&](int code) {
        free_plan_memory(p);
        delete p;
        return code;
    };
    if ((rc = upload(&p->d_tw, build_twiddles(p->shape, prec == LSR_PREC_PLAIN, prec != LSR_PREC_FP64), f32))) return fail(rc);
    if (prec != LSR_PREC_PLAIN)
        if ((rc = upload(&p->d_hx, build_hx(N, dx, lambda, L), f32))) return fail(rc);
    const bool curved = F != 0.0 && std::isfinite(F);
    if (curved)
        if ((rc = upload(&p->d_foc, build_focal(N, dx, lambda, F), f32))) return fail(rc);
    if ((rc = dalloc(&p->d_partials, sizeof(double) * 4 * (size_t)nrb_max))) return fail(rc);
    if ((rc = dalloc(&p->d_trace, sizeof(double) * 4 * (size_t)p->trace_cap))) return fail(rc);
    if ((rc = dalloc(&p->d_counters, sizeof(unsigned) * CNT_WORDS))) return fail(rc);
    if (hipMemset(p->d_counters, 0, sizeof(unsigned) * CNT_WORDS) != hipSuccess ||
        hipMemset(p->d_trace, 0, sizeof(double) * 4 * (size_t)p->trace_cap) != hipSuccess)
        return fail(set_err(LSR_EDEVICE, "hipMemset failed"));

    CavDesc& d = p->d;
    d.tw = p->d_tw;
    d.hx = p->d_hx;
    d.pump_c = nullptr;
    d.foc = p->d_foc;
    d.mask = a.kind == 3 ? a.mask : nullptr;
    d.rough = nullptr;
    d.partials = p->d_partials;
    d.trace = p->d_trace;
    d.counters = p->d_counters;
    d.N = N;
    d.prec = (int)prec;
    d.ap_kind = a.kind;
    d.ap_half_order = a.kind == 1 ? a.order / 2 : 1;
    d.trace_cap = p->trace_cap;
    d.nrb = nrb;
    d.nbins = (int)floor(N / sqrt(2.0) + 0.5) + 1;
    d.sqrtR = sqrt(R);
    d.N0 = 0.0;
    d.inv_T1 = 1.0;
    d.mod_amp = 0.0;
    d.dx = dx;
    d.ap_step = aperture_step(a.kind, a.radius, d.ap_half_order, dx);
    d.phase_c = kTwoPi * 0.5 * lambda * L / ((N * dx) * (N * dx));
    d.inv_nn = 1.0 / ((double)N * (double)N);
    d.prop_kind = 0;
    d.model = 0;
    *out = p;
    return LSR_OK;
}

int lsr_plan_set_gain(lsr_plan p, double N0, double T1, double mod_amp, double mod_period) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    if (!std::isfinite(N0)) return set_err(LSR_EINVAL, "N0 must be finite");
    if (!(T1 > 0) || !std::isfinite(T1)) return set_err(LSR_EINVAL, "T1 must be > 0");
    if (!std::isfinite(mod_amp) || !(mod_period >= 0) || !std::isfinite(mod_period))
        return set_err(LSR_EINVAL, "bad pump modulation");
    DeviceGuard g(p->device);
    const bool modulated = mod_amp != 0.0 && mod_period > 0.0;
    if (modulated) {
        void* t = nullptr;
        int rc = upload(&t, build_pump_cos(p->N, p->dx, mod_period), p->prec != PREC_FP64);
        if (rc) return rc;
        if (p->d_pump) {
            // the old table may still be read by enqueued work
            const hipError_t e = hipStreamSynchronize(p->stream);
            if (e != hipSuccess) {
                (void)hipFree(t);
                return set_err(LSR_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
            }
            (void)hipFree(p->d_pump);
        }
        p->d_pump = t;
    }
    p->N0 = N0;
    p->T1 = T1;
    p->mod_amp = mod_amp;
    p->mod_period = mod_period;
    p->d.N0 = N0;
    p->d.inv_T1 = 1.0 / T1;
    p->d.mod_amp = modulated ? mod_amp : 0.0;
    p->d.pump_c = modulated ? p->d_pump : nullptr;
    ++p->version;
    return LSR_OK;
}

int lsr_plan_set_model(lsr_plan p, int model) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    if (model < LSR_MODEL_B_EULER || model > LSR_MODEL_CLASS_A) return set_err(LSR_EINVAL, "model %d out of range", model);
    p->model = model;
    p->d.model = model | (p->d_rough ? MODEL_ROUGH : 0);
    ++p->version;
    return LSR_OK;
}

int lsr_plan_set_filter(lsr_plan p, double delta) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    if (!(delta >= 0) || !std::isfinite(delta)) return set_err(LSR_EINVAL, "filter width must be >= 0");
    DeviceGuard g(p->device);
    void* t = nullptr;
    if (delta > 0) {
        int rc = upload(&t, build_filter(p->N, p->dx, delta), p->prec != PREC_FP64);
        if (rc) return rc;
    } else if (p->prec != PREC_PLAIN) {
        int rc = upload(&t, build_hx(p->N, p->dx, p->lambda, p->L), p->prec != PREC_FP64);
        if (rc) return rc;
    }
    void* ts = nullptr;
    int rc = build_sheet_table(p, p->slices, delta, &ts);
    if (rc == LSR_OK && hipStreamSynchronize(p->stream) != hipSuccess)
        rc = set_err(LSR_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(hipGetLastError()));
    if (rc != LSR_OK) {
        if (t) (void)hipFree(t);
        if (ts) (void)hipFree(ts);
        return rc;
    }
    // the old tables are no longer read by enqueued work
    if (p->d_hx) (void)hipFree(p->d_hx);
    if (p->d_hs) (void)hipFree(p->d_hs);
    p->d_hx = t;
    p->d_hs = ts;
    p->filter = delta;
    p->d.hx = t;
    p->d.prop_kind = p->d_trans ? 2 : delta > 0 ? 1 : 0;
    ++p->version;
    return LSR_OK;
}

int lsr_plan_set_fft_plan(lsr_plan p, int k) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    if (k < 0) return set_err(LSR_EINVAL, "FFT plan %d", k);
    const Launchers* kern = k == 0 ? launchers_for(p->N, p->prec == PREC_FP64)
                                   : (p->prec == PREC_FP64 ? nullptr : launchers_alt(p->N, k));
    if (!kern) return set_err(LSR_EUNSUPPORTED, "no one-cavity FFT plan %d for N=%d in this precision form", k, p->N);
    if (k == p->fft_plan) return LSR_OK;
    DeviceGuard g(p->device);
    void* t = nullptr;
    int rc = upload(&t, build_twiddles(kern->shape, p->prec == PREC_PLAIN, p->prec != PREC_FP64), p->prec != PREC_FP64);
    if (rc) return rc;
    if (hipStreamSynchronize(p->stream) != hipSuccess) {
        (void)hipFree(t);
        return set_err(LSR_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(hipGetLastError()));
    }
    // the old table is no longer read by enqueued work
    (void)hipFree(p->d_tw);
    p->d_tw = t;
    p->d.tw = t;
    p->kern = kern;
    p->shape = kern->shape;
    p->d.nrb = p->N / p->shape.LPW;
    p->fft_plan = k;
    ++p->version;
    return LSR_OK;
}

int lsr_plan_set_transfer(lsr_plan p, const double* T) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    const int N = p->N;
    const size_t nn = (size_t)N * (size_t)N;
    void* t = nullptr;
    if (T) {
        if (p->slices != 1) return set_err(LSR_EINVAL, "a general transfer function needs a single gain sheet");
        // by column (frequency p, q at p*N + q), 1/N^2 folded in
        std::vector<double> tab(2 * nn);
        const double inn = 1.0 / ((double)N * (double)N);
        for (int q = 0; q < N; ++q)
            for (int pp = 0; pp < N; ++pp) {
                const size_t src = 2 * ((size_t)q * N + pp), dst = 2 * ((size_t)pp * N + q);
                if (!std::isfinite(T[src]) || !std::isfinite(T[src + 1]))
                    return set_err(LSR_EINVAL, "transfer value (%d, %d) is not finite", q, pp);
                tab[dst] = T[src] * inn;
                tab[dst + 1] = T[src + 1] * inn;
            }
        DeviceGuard g(p->device);
        int rc = upload(&t, tab, p->prec != PREC_FP64);
        if (rc) return rc;
    }
    DeviceGuard g(p->device);
    if (hipStreamSynchronize(p->stream) != hipSuccess) {
        if (t) (void)hipFree(t);
        return set_err(LSR_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(hipGetLastError()));
    }
    // the old table is no longer read by enqueued work
    if (p->d_trans) (void)hipFree(p->d_trans);
    p->d_trans = t;
    p->d.trans = t;
    p->d.prop_kind = t ? 2 : p->filter > 0 ? 1 : 0;
    ++p->version;
    return LSR_OK;
}

int lsr_plan_set_roughness(lsr_plan p, const double* psi) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    const size_t nn = (size_t)p->N * (size_t)p->N;
    void* t = nullptr;
    if (psi) {
        // exp(i psi) in FP64, each angle reduced to one turn first
        std::vector<double> tab(2 * nn);
        for (size_t i = 0; i < nn; ++i) {
            if (!std::isfinite(psi[i])) return set_err(LSR_EINVAL, "roughness phase %zu is not finite", i);
            const double turns = psi[i] / kTwoPi;
            const double f = turns - floor(turns);
            tab[2 * i] = cos(kTwoPi * f);
            tab[2 * i + 1] = sin(kTwoPi * f);
        }
        DeviceGuard g(p->device);
        int rc = upload(&t, tab, p->prec != PREC_FP64);
        if (rc) return rc;
    }
    DeviceGuard g(p->device);
    if (hipStreamSynchronize(p->stream) != hipSuccess) {
        if (t) (void)hipFree(t);
        return set_err(LSR_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(hipGetLastError()));
    }
    // the old table is no longer read by enqueued work
    if (p->d_rough) (void)hipFree(p->d_rough);
    p->d_rough = t;
    p->d.rough = t;
    p->d.model = p->model | (t ? MODEL_ROUGH : 0);
    ++p->version;
    return LSR_OK;
}

int lsr_plan_set_slices(lsr_plan p, int m) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    if (m < 1 || m > LSR_MAX_SLICES) return set_err(LSR_EINVAL, "%d gain sheets: must be 1..%d", m, LSR_MAX_SLICES);
    if (m > 1 && p->d_trans) return set_err(LSR_EINVAL, "several gain sheets do not combine with a general transfer function");
    DeviceGuard g(p->device);
    void* ts = nullptr;
    int rc = build_sheet_table(p, m, p->filter, &ts);
    if (rc != LSR_OK) return rc;
    if (hipStreamSynchronize(p->stream) != hipSuccess) {
        if (ts) (void)hipFree(ts);
        return set_err(LSR_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(hipGetLastError()));
    }
    // the old table is no longer read by enqueued work
    if (p->d_hs) (void)hipFree(p->d_hs);
    p->d_hs = ts;
    p->slices = m;
    ++p->version;
    return LSR_OK;
}

int lsr_plan_set_stream(lsr_plan p, void* s) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    p->stream = static_cast<hipStream_t>(s);
    return LSR_OK;
}

int lsr_plan_nbins(lsr_plan p) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    return p->d.nbins;
}

int lsr_roundtrips(lsr_plan p, void* E, void* Ninv, int n_trips) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    if (n_trips < 0) return set_err(LSR_EINVAL, "n_trips < 0");
    if (!E || !Ninv) return set_err(LSR_EINVAL, "E or Ninv is NULL");
    if (!aligned16(E) || !aligned16(Ninv)) return set_err(LSR_EINVAL, "E and Ninv must be 16-byte aligned");
    if (n_trips == 0) return LSR_OK;
    DeviceGuard g(p->device);
    const Launchers* k = p->kern;
    const int rc = for_each_launch(p, E, Ninv, n_trips, [&](const CavDesc& d, bool row, int mode) {
        return row ? k->row(d, mode, p->stream) : k->col(d, mode, p->stream);
    });
    if (rc != 0) return set_err(LSR_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    p->trips_done += (unsigned long long)n_trips;
    p->last_n = n_trips;
    return LSR_OK;
}

int lsr_time_kernels(lsr_plan p, void* E, void* Ninv, int n_trips, double* ms) {
    if (!p || !ms) return set_err(LSR_EINVAL, "plan or ms is NULL");
    if (n_trips < 1) return set_err(LSR_EINVAL, "n_trips < 1");
    if (!E || !Ninv || !aligned16(E) || !aligned16(Ninv)) return set_err(LSR_EINVAL, "bad E/Ninv pointer");
    DeviceGuard g(p->device);
    const Launchers* k = p->kern;
    const int nl = 2 * n_trips * p->slices + 1;
    std::vector<hipEvent_t> ev(2 * (size_t)nl, nullptr);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& x : ev)
                if (x) (void)hipEventDestroy(x);
            return set_err(LSR_EDEVICE, "hipEventCreate failed");
        }
    int li = 0;
    int rc = for_each_launch(p, E, Ninv, n_trips, [&](const CavDesc& d, bool row, int mode) {
        (void)hipEventRecord(ev[2 * li], p->stream);
        const int r = row ? k->row(d, mode, p->stream) : k->col(d, mode, p->stream);
        (void)hipEventRecord(ev[2 * li + 1], p->stream);
        ++li;
        return r;
    });
    double row_ms = 0, col_ms = 0;
    int nrow = 0, ncol = 0;
    if (rc == 0 && li == nl && hipStreamSynchronize(p->stream) == hipSuccess) {
        // launch order: row, (col, row) * n * m; the first and last row
        // launches (FIRST / LAST forms) are excluded from the row mean unless
        // they are the only ones
        for (int i = 0; i < nl; ++i) {
            float t = 0;
            (void)hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
            const bool row = (i % 2) == 0;
            if (row) {
                if (nl > 3 && (i == 0 || i == nl - 1)) continue;
                row_ms += t;
                ++nrow;
            } else {
                col_ms += t;
                ++ncol;
            }
        }
    } else if (rc == 0) {
        rc = -3;
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (rc != 0) return set_err(LSR_EDEVICE, "timed launches failed: %s", hipGetErrorString(hipGetLastError()));
    ms[0] = nrow ? row_ms / nrow : 0.0;
    ms[1] = ncol ? col_ms / ncol : 0.0;
    p->trips_done += (unsigned long long)n_trips;
    p->last_n = n_trips;
    return LSR_OK;
}

int lsr_sync(lsr_plan p) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    DeviceGuard g(p->device);
    LSR_HIP(hipStreamSynchronize(p->stream));
    unsigned c[CNT_WORDS];
    LSR_HIP(hipMemcpy(c, p->d_counters, sizeof c, hipMemcpyDeviceToHost));
    if (c[CNT_HANG]) {
        LSR_HIP(hipMemset(p->d_counters + CNT_HANG, 0, sizeof(unsigned)));
        // the skipped column tasks recorded no trace: realign the host's
        // count with the device's, and the failed call has no trace
        p->trips_done = c[CNT_TRIPS];
        p->last_n = 0;
        return set_err(LSR_EDEVICE, "a batched round trip gave up waiting for its row pass (task table error)");
    }
    if (c[CNT_NONFINITE]) {
        const unsigned bad = c[CNT_NONFINITE];
        LSR_HIP(hipMemset(p->d_counters + CNT_NONFINITE, 0, sizeof(unsigned)));
        return set_err(LSR_ENONFINITE, "non-finite state at trip %u (counted since plan creation)", bad - 1);
    }
    return LSR_OK;
}

int lsr_trace(lsr_plan p, double* out, int capacity) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    if (capacity < 0 || (capacity > 0 && !out)) return set_err(LSR_EINVAL, "bad output buffer");
    DeviceGuard g(p->device);
    LSR_HIP(hipStreamSynchronize(p->stream));
    int n = p->last_n;
    if (n > p->trace_cap) n = p->trace_cap;
    if (n > capacity) n = capacity;
    if (n == 0) return 0;
    // newest n records of the last call, oldest first: one or two contiguous
    // runs of the ring
    const unsigned long long first = p->trips_done - (unsigned long long)n;
    const size_t slot = (size_t)(first % (unsigned long long)p->trace_cap);
    const size_t n1 = std::min((size_t)n, (size_t)p->trace_cap - slot);
    const size_t rec = 4 * sizeof(double);
    LSR_HIP(hipMemcpy(out, p->d_trace + 4 * slot, n1 * rec, hipMemcpyDeviceToHost));
    if (n1 < (size_t)n) LSR_HIP(hipMemcpy(out + 4 * n1, p->d_trace, ((size_t)n - n1) * rec, hipMemcpyDeviceToHost));
    return n;
}

int lsr_diag(lsr_plan p, const void* E, const void* Ninv, lsr_diag_out* out) {
    if (!p || !out) return set_err(LSR_EINVAL, "plan or out is NULL");
    if (!E || !Ninv || !aligned16(E) || !aligned16(Ninv)) return set_err(LSR_EINVAL, "bad E/Ninv pointer");
    DeviceGuard g(p->device);
    const int N = p->N, nb = p->d.nbins, nrb = N / 2;   // as many row blocks as any shape has
    const size_t elem = 2 * p->real_bytes();
    int rc;
    // the spectrum scratch, on first use; all three or none
    if (!p->d_scratch) {
        void* sc = nullptr;
        double *rp = nullptr, *dout = nullptr;
        if ((rc = dalloc(&sc, elem * (size_t)N * N)) || (rc = dalloc(&rp, sizeof(double) * (size_t)nrb * nb)) ||
            (rc = dalloc(&dout, sizeof(double) * (4 + (size_t)nb)))) {
            if (sc) (void)hipFree(sc);
            if (rp) (void)hipFree(rp);
            return rc;
        }
        p->d_scratch = sc;
        p->d_radial_part = rp;
        p->d_diag_out = dout;
    }
    CavDesc d = p->d;
    d.E = const_cast<void*>(E);
    d.Ninv = const_cast<void*>(Ninv);
    d.scratch = p->d_scratch;
    d.radial_part = p->d_radial_part;
    rc = p->kern->row(d, ROW_DIAG, p->stream);
    if (rc == 0) rc = p->kern->col(d, COL_DIAG, p->stream);
    if (rc != 0) return set_err(LSR_EDEVICE, "diag launch failed: %s", hipGetErrorString(hipGetLastError()));
    if (launch_diag_reduce(d, p->d_diag_out, p->stream)) return set_err(LSR_EDEVICE, "diag reduce launch failed");
    std::vector<double> h(4 + (size_t)nb);
    LSR_HIP(hipMemcpyAsync(h.data(), p->d_diag_out, h.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    LSR_HIP(hipStreamSynchronize(p->stream));
    const double dx2 = p->dx * p->dx;
    out->energy = h[0] * dx2;
    out->power_out = (1.0 - p->R) * h[2] * dx2;
    out->gain_sum = (h[2] - h[1]) * dx2;
    out->aperture_loss = (h[0] - h[1]) * dx2;
    out->inv_sum = h[3] * dx2;
    out->nbins = nb;
    int best = -1;
    double bv = -1.0;
    for (int k = 1; k < nb; ++k)
        if (h[4 + k] > bv) { bv = h[4 + k]; best = k; }
    out->dominant_bin = best;
    if (out->radial) memcpy(out->radial, h.data() + 4, sizeof(double) * (size_t)nb);
    if (!std::isfinite(h[0]) || !std::isfinite(h[3]))
        return set_err(LSR_ENONFINITE, "non-finite state passed to lsr_diag");
    return LSR_OK;
}

int lsr_propagate(lsr_plan p, const void* E_in, double z, void* E_out) {
    if (!p) return set_err(LSR_EINVAL, "plan is NULL");
    if (!(z >= 0) || !std::isfinite(z)) return set_err(LSR_EINVAL, "z must be >= 0 and finite");
    if (!E_in || !E_out || !aligned16(E_in) || !aligned16(E_out)) return set_err(LSR_EINVAL, "bad E_in/E_out pointer");
    DeviceGuard g(p->device);
    // the previous call's table may still be in use
    LSR_HIP(hipStreamSynchronize(p->stream));
    if (p->d_hz) (void)hipFree(p->d_hz);
    p->d_hz = nullptr;
    int rc = upload(&p->d_hz, build_hx(p->N, p->dx, p->lambda, z), p->prec != PREC_FP64);
    if (rc) return rc;
    CavDesc d = p->d;
    d.E = const_cast<void*>(E_in);
    d.scratch = E_out;
    rc = p->kern->row(d, ROW_FWD, p->stream);
    d.E = E_out;
    d.hx = p->d_hz;
    d.prop_kind = 1;   // table form in every precision
    if (rc == 0) rc = p->kern->col(d, COL_FREE, p->stream);
    if (rc == 0) rc = p->kern->row(d, ROW_LAST, p->stream);
    if (rc != 0) return set_err(LSR_EDEVICE, "propagate launch failed: %s", hipGetErrorString(hipGetLastError()));
    return LSR_OK;
}

void lsr_plan_destroy(lsr_plan p) {
    if (!p) return;
    DeviceGuard g(p->device);
    (void)hipStreamSynchronize(p->stream);
    free_plan_memory(p);
    delete p;
}

}  // extern "C"

