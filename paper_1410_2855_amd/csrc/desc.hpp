// desc.hpp -- per-cavity descriptor read by the kernels (host and device).
#pragma once

#include <cmath>
#include <cstdint>

namespace lsr {

enum Prec : int { PREC_PLAIN = 0, PREC_FP64TAB = 1, PREC_FP64 = 2 };
enum ApKind : int { AP_NONE = 0, AP_SUPERGAUSS = 1, AP_GAUSS = 2, AP_MASK = 3 };

// Row-pass modes.  FIRST reads the row-major state, MID the tiled transform
// of the previous trip, LAST finishes the inverse transform and writes the
// row-major state, DIAG evaluates the local step and forward row transform
// of a state into scratch without touching the state.
// ROW_FWD: forward row transform of a row-major field (E) into the tiled
// scratch, no local step (free propagation of a field copy).
enum RowMode : int { ROW_FIRST = 0, ROW_MID = 1, ROW_LAST = 2, ROW_DIAG = 3, ROW_FWD = 4 };
// COL_FREE: the propagator multiply without folding the trip's sums.
enum ColMode : int { COL_PROP = 0, COL_DIAG = 1, COL_FREE = 2 };

// Counters of a cavity (device, 16 words):
//  [0] trips completed (trace ring slot of the next trip)
//  [1] first trip (1-based) whose sums were non-finite, 0 if none
//  [2] set when a batched column task gave up waiting for its row pass
enum : int { CNT_TRIPS = 0, CNT_NONFINITE = 1, CNT_HANG = 2, CNT_WORDS = 16 };

// Bit of the local-step code selecting the kernels that apply the mirror
// roughness table (the others carry no code for it).
enum : int { MODEL_ROUGH = 4, MODEL_MASK = 3 };

struct CavDesc {
    void* E;                // field (row-major between calls, tiled inside)
    void* Ninv;             // inversion, row-major
    const void* tw;         // Stockham twiddles of this N (forward, then inverse passes)
    const void* hx;         // per-axis factor hx(p) of the nonlocal step, N entries: the
                            // propagator (FP64TAB / FP64) or the real filter (any form)
    const void* pump_c;     // cos(2 pi x_i / d), N entries, or null (uniform pump)
    const void* foc;        // exp(i pi x_i^2/(lambda F)), N complex entries, or null (flat mirror)
    const void* mask;       // N*N aperture amplitude (AP_MASK) or null
    const void* rough;      // N*N exp(i psi) of the mirror roughness psi, complex, or null
    const void* trans;      // N*N complex transfer function of a general nonlocal step
                            // (prop_kind 2), stored by column: frequency (p, q) at p*N + q,
                            // 1/N^2 folded in; or null
    void* scratch;          // DIAG: tiled forward row transform of G (N*N complex)
    double* partials;       // per row block: 4 sums
    double* radial_part;    // DIAG: per column block radial spectrum partials
    double* trace;          // ring of trace_cap records of 4 sums; null in the batch descriptors
                            // of gain sheets other than 0 (their column pass folds no sums)
    unsigned* counters;     // CNT_WORDS words
    int N;
    int prec;
    int ap_kind;
    int ap_half_order;      // super-Gaussian exponent / 2
    int trace_cap;
    int nrb;                // row blocks = column blocks = N / LPW
    int nbins;
    int prop_kind;          // 0 Fresnel propagator (hx), 1 real filter table (hx holds it),
                            // 2 general transfer function (trans)
    int model;              // local-step code: bits 0-1 the model, 0 B class (Euler
                            // update), 1 B class (exact update over a trip), 2 class A
                            // (saturable gain); MODEL_ROUGH set exactly when rough is
                            // non-null
    double sqrtR;
    double N0, inv_T1, mod_amp;
    double dx;
    double ap_step;         // grid step in aperture units: with X' = (x - N/2) ap_step and
                            // Y' likewise, u = X'^2 + Y'^2 and A = 2^(-u^h) (aperture_step)
    double phase_c;         // PLAIN: pi lambda L / (N dx)^2, rad per index^2
    double inv_nn;          // 1/N^2
};

// The aperture amplitude A = exp(-(r^2/r0^2)^h) (super-Gaussian of order 2h)
// or exp(-r^2/(2 r0^2)) (Gaussian, h = 1) written as A = 2^(-u^h) with
// u = c r^2, c = log2(e)^(1/h) / r0^2 (resp. log2(e) / (2 r0^2)): the base-2
// exponential and the scale by log2(e) then cost nothing per point, and the
// grid step is scaled by sqrt(c) so that u = X'^2 + Y'^2.  0 without a
// smooth aperture.
inline double aperture_step(int kind, double radius, int half_order, double dx) {
    const double log2e = 1.4426950408889634073599246810019;
    if (kind == AP_SUPERGAUSS) return dx * std::sqrt(std::pow(log2e, 1.0 / half_order) / (radius * radius));
    if (kind == AP_GAUSS) return dx * std::sqrt(log2e / (2.0 * radius * radius));
    return 0.0;
}

}  // namespace lsr
