/*
 * orc.h -- FP64 CPU oracle of the split-step round-trip map of a
 * microchip-laser cavity (Okulov, "Two-dimensional periodic and
 * quasiperiodic spatial structures in microchip laser resonator").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain, obviously
 * correct reference that the GPU path is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or constant with the GPU library.
 *
 * Complex arrays are interleaved (re, im) doubles.  N x N grids are
 * row-major: element (row y, column x) sits at index y*N + x.
 */
#ifndef ORC_H
#define ORC_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int    N;           /* grid points per side                               */
    double dx;          /* grid spacing (m)                                   */
    double lambda;      /* wavelength (m)                                     */
    double L;           /* propagation length of one map iterate (m)          */
    double focal;       /* mirror focal length (m), < 0 diverging; 0 or inf = flat */
    double R;           /* mirror (intensity) reflectivity, 0 < R <= 1         */
    int    ap_kind;     /* 0 none, 1 super-Gaussian, 2 Gaussian, 3 user mask   */
    double ap_radius;   /* aperture radius r0 (m)                             */
    int    ap_order;    /* super-Gaussian exponent m in exp(-(r/r0)^m)        */
    const double* ap_mask; /* kind 3: N*N real amplitude, row-major           */
    double N0;          /* pump level (round-trip log-gain units)             */
    double T1;          /* inversion relaxation time (round trips)            */
    double mod_amp;     /* pump modulation depth (0 = uniform pump)            */
    double mod_period;  /* pump modulation period d (m); 0 = uniform          */
    double filter_delta;/* > 0: the real renormalization-group filter
                           exp[(Delta^2/2) Laplacian] (Sec. 2.3, Eq. (18)) of
                           deviation Delta (m) replaces the Fresnel step;
                           0 = Fresnel propagation over L                       */
    int    model;       /* local step and inversion update, sigma = 1:
                           0 B-class laser, Eq. (1) (forward Euler, one trip)
                           1 B-class laser, Eq. (6) integrated exactly over one
                             trip with |E|^2 frozen
                           2 class-A laser, Eq. (8): saturable gain
                             N/(1 + T1|E|^2), inversion held at the pump     */
    int    slices;      /* thin gain sheets per iterate, m; 0 or 1 = the single
                           sheet of Eq. (1).  m > 1: the active medium cut
                           into m thin sheets spread along the cavity, each
                           holding its own inversion (the distributed-gain
                           variant noted in Sec. 2.2 after Eq. (12)); see
                           orc_run                                          */
    const double* rough;/* N*N phase psi (rad) of the mirror roughness, the
                           random term of the complex aperture of Eq. (12);
                           row-major; NULL = smooth mirror                  */
    const double* transfer; /* the nonlocal step as a general convolution,
                           the map with kernel K of Eq. (10):
                           E_{n+1} = IFFT2(T . FFT2(G)) with T given here as
                           N*N complex values (interleaved re, im), in FFT
                           frequency order, row-major (row = y frequency
                           index q, column = x frequency index p).  For the
                           kernel of Eq. (10) sampled on the grid,
                           E_{n+1}(x2) = dx^2 sum_{x1} K(x1 - x2) G(x1),
                           T(f) = dx^2 sum_u K(u) exp(+2 pi i f.u / N).
                           NULL = Fresnel propagation (or the filter);
                           not combined with the filter or several sheets */
} orc_params;

/* One-dimensional DFT of length n = 2^a 3^b, in place, unnormalized.
 * inverse = 0: X[k] = sum_j x[j] exp(-2 pi i jk/n); inverse = 1: exp(+...). */
int  orc_fft1d(double* x, int n, int inverse);

/* The same transform evaluated by the O(n^2) definition. */
int  orc_dft_brute1d(const double* in, double* out, int n, int inverse);

/* Two-dimensional transform of an n x n row-major array: all rows, then all
 * columns.  Unnormalized in both directions. */
int  orc_fft2(double* x, int n, int inverse);

/* The same 2D transform evaluated by the O(n^4) definition. */
int  orc_dft_brute2d(const double* in, double* out, int n, int inverse);

/* Advance (E, Ninv) by n_trips iterates of the round-trip map.
 * E: N*N complex field at the gain-sheet plane, before the local step.
 * Ninv: N*N inversion.  Both are updated in place.
 * With m = slices > 1 an iterate is m steps, k = 0..m-1: thin sheet k with
 * its own inversion (Ninv holds m*N*N values, sheet k at offset k*N*N),
 * then free propagation over L/m (filter: variance Delta^2/m).  Sheet 0
 * carries the mirror and aperture; every sheet has pump N0/m, so that the
 * small-signal gain of an iterate is that of the single sheet.  The trace
 * sums are those of sheet 0.
 * trace (nullable): 4*n_trips doubles; for trip t the raw sums
 *   [4t+0] S1 = sum |E_t|^2
 *   [4t+1] S2 = sum |A|^2 |E_t|^2
 *   [4t+2] S3 = sum |A|^2 exp(N_t) |E_t|^2
 *   [4t+3] S4 = sum N_t
 * taken over the grid in row-major order.
 * Returns 0, or -1 on invalid parameters / allocation failure. */
int  orc_run(const orc_params* p, double* E, double* Ninv, int n_trips,
             double* trace);

/* Free propagation over a distance z >= 0 (m), no local step: E is replaced
 * by IFFT2( exp(-i pi lambda z (fx^2 + fy^2)) FFT2(E) ) (the operator
 * exponent of Sec. 2.3, Eq. (25), for length z).  Uses N, dx and lambda of p.
 * Returns 0, or -1 for invalid arguments. */
int  orc_propagate(const orc_params* p, double* E, double z);

/* Number of radial bins of the far-field spectrum for an N-point grid. */
int  orc_nbins(int N);

/* Far-field radial spectrum of the field leaving the gain sheet:
 * radial[k] = sum over (p,q) with round(sqrt(p~^2 + q~^2)) = k of |FFT2(G)|^2,
 * G = sqrt(R) A exp(N/2) E.  radial has nbins >= orc_nbins(N) entries.
 * Returns the dominant bin (argmax over k >= 1, lowest on ties) or -1. */
int  orc_spectrum(const orc_params* p, const double* E, const double* Ninv,
                  double* radial, int nbins);

#ifdef __cplusplus
}
#endif
#endif
