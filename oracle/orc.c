/*
 * orc.c -- FP64 CPU oracle of the split-step round-trip map.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, plain reference the GPU library is
 * checked against.  Single-threaded, double precision throughout, no
 * blocking, fusion or reordering of the method's steps.  It shares no code
 * with the GPU path.  Build: gcc -O2 -fno-fast-math -ffp-contract=off.
 *
 * The method (paper, Introduction, Eq. (1) "conv_map", and Sec. 2.2,
 * Eq. (11) "complex_8F" with the aperture of Eq. (12)): one iterate of the
 * cavity map is a local step f (gain sheet with inversion frozen during the
 * pass, mirror reflectivity, aperture) followed by the nonlocal linear step,
 * Fresnel diffraction over the cavity length L.  The diffraction operator is
 * evaluated as the operator exponent exp[i L/(2k) Laplacian] of Sec. 2.3,
 * Eq. (25), i.e. by the split-step FFT method named in the abstract and in
 * Sec. 2.2: forward 2D DFT, multiplication by the free-space transfer
 * function, inverse 2D DFT.  The inversion is updated once per bounce as in
 * the second line of Eq. (1).
 *
 * Readings of points where the paper is silent or garbled (each is also
 * listed in the design notes):
 *  - inversion update: Eq. (1) prints N_{n+1} = -(N_n - N0)/T1 - sigma N_n|E_n|^2,
 *    which lacks the N_n on the right.  Read as the forward-Euler step, one
 *    round trip long, of the B-class rate equation Eq. (6):
 *        N_{n+1} = N_n + (N0 - N_n)/T1 - N_n |E_n|^2,   sigma = 1.
 *  - local map f: the inversion is frozen while the field passes (Intro), so
 *    f(E) = sqrt(R) A exp(N/2) E: amplitude gain exp(N/2) (intensity exp(N)),
 *    N being the round-trip log-gain; saturation enters through the update.
 *  - |E_n|^2 depleting the inversion is the field incident on the sheet.
 *  - transfer function: exp[i L/(2k) Laplacian] of Eq. (25) in Fourier space
 *    is H = exp(-i pi lambda L (fx^2 + fy^2)); no exp(ikL), no global sign.
 *  - order within the trip: local step first, then propagation; the state
 *    E_n is the field at the gain sheet before the local step.
 *  - grid: x_j = (j - N/2) dx; signed frequency index p~ = p (p < N/2) else
 *    p - N; fx = p~ / (N dx).  Forward DFT unnormalized, inverse scaled 1/N^2.
 *  - several gain sheets: the paper names, only by reference, the variant in
 *    which the active medium is spread along the cavity as thin sheets, each
 *    with its own inversion (Sec. 2.2, after Eq. (12)).  Read as m equally
 *    spaced sheets per iterate, free propagation over L/m after each; the
 *    mirror and aperture act at sheet 0, which holds the state; each sheet
 *    has pump N0/m, the same T1 and local-step model, and is depleted by the
 *    field incident on it.  m = 1 is Eq. (1) exactly.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* Textbook FFT: iterative radix-2 decimation in time, plus a radix-3  */
/* decimation-in-time split for lengths 3 * 2^m.                        */
/* ------------------------------------------------------------------ */

static int length_ok(int n)
{
    if (n < 1) return 0;
    while (n % 3 == 0) n /= 3;
    while (n % 2 == 0) n /= 2;
    return n == 1;
}

/* In-place radix-2 DIT on a power-of-two length: bit-reversal permutation,
 * then log2(n) butterfly stages.  Each stage's twiddles exp(sign 2 pi i k/len)
 * come straight from cos/sin, not from a recurrence. */
static void fft_pow2(double* x, int n, double sign)
{
    if (n < 2) return;
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double tr = x[2 * i], ti = x[2 * i + 1];
            x[2 * i] = x[2 * j];
            x[2 * i + 1] = x[2 * j + 1];
            x[2 * j] = tr;
            x[2 * j + 1] = ti;
        }
    }
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    for (int len = 2; len <= n; len <<= 1) {
        int half = len >> 1;
        for (int k = 0; k < half; k++) {
            double ang = 2.0 * M_PI * (double)k / (double)len;
            w[2 * k] = cos(ang);
            w[2 * k + 1] = sign * sin(ang);
        }
        for (int i = 0; i < n; i += len) {
            for (int k = 0; k < half; k++) {
                double* u = x + 2 * (i + k);
                double* v = x + 2 * (i + k + half);
                double vr = v[0] * w[2 * k] - v[1] * w[2 * k + 1];
                double vi = v[0] * w[2 * k + 1] + v[1] * w[2 * k];
                double ur = u[0], ui = u[1];
                u[0] = ur + vr;
                u[1] = ui + vi;
                v[0] = ur - vr;
                v[1] = ui - vi;
            }
        }
    }
    free(w);
}

static int fft_any(double* x, int n, double sign)
{
    if (n % 3 == 0) {
        /* X[k] = sum_{r=0..2} W_n^{rk} Y_r[k mod m],  Y_r = DFT_m(x[3j + r]),
         * W_n = exp(sign 2 pi i / n). */
        int m = n / 3;
        double* y = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        if (!y) return -1;
        for (int r = 0; r < 3; r++)
            for (int j = 0; j < m; j++) {
                y[2 * (r * m + j)] = x[2 * (3 * j + r)];
                y[2 * (r * m + j) + 1] = x[2 * (3 * j + r) + 1];
            }
        for (int r = 0; r < 3; r++)
            if (fft_any(y + 2 * r * m, m, sign)) { free(y); return -1; }
        for (int k = 0; k < n; k++) {
            double sr = 0.0, si = 0.0;
            for (int r = 0; r < 3; r++) {
                long e = ((long)r * k) % n;
                double ang = 2.0 * M_PI * (double)e / (double)n;
                double wr = cos(ang), wi = sign * sin(ang);
                double yr = y[2 * (r * m + k % m)], yi = y[2 * (r * m + k % m) + 1];
                sr += yr * wr - yi * wi;
                si += yr * wi + yi * wr;
            }
            x[2 * k] = sr;
            x[2 * k + 1] = si;
        }
        free(y);
        return 0;
    }
    fft_pow2(x, n, sign);
    return 0;
}

int orc_fft1d(double* x, int n, int inverse)
{
    if (!x || !length_ok(n)) return -1;
    return fft_any(x, n, inverse ? 1.0 : -1.0);
}

int orc_dft_brute1d(const double* in, double* out, int n, int inverse)
{
    if (!in || !out || n < 1) return -1;
    double sign = inverse ? 1.0 : -1.0;
    for (int k = 0; k < n; k++) {
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < n; j++) {
            long e = ((long)j * k) % n;     /* exact integer reduction of jk */
            double ang = 2.0 * M_PI * (double)e / (double)n;
            double wr = cos(ang), wi = sign * sin(ang);
            sr += in[2 * j] * wr - in[2 * j + 1] * wi;
            si += in[2 * j] * wi + in[2 * j + 1] * wr;
        }
        out[2 * k] = sr;
        out[2 * k + 1] = si;
    }
    return 0;
}

int orc_fft2(double* x, int n, int inverse)
{
    if (!x || !length_ok(n)) return -1;
    double sign = inverse ? 1.0 : -1.0;
    for (int y = 0; y < n; y++)
        if (fft_any(x + 2 * (size_t)y * n, n, sign)) return -1;
    double* col = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!col) return -1;
    for (int c = 0; c < n; c++) {
        for (int y = 0; y < n; y++) {
            col[2 * y] = x[2 * ((size_t)y * n + c)];
            col[2 * y + 1] = x[2 * ((size_t)y * n + c) + 1];
        }
        if (fft_any(col, n, sign)) { free(col); return -1; }
        for (int y = 0; y < n; y++) {
            x[2 * ((size_t)y * n + c)] = col[2 * y];
            x[2 * ((size_t)y * n + c) + 1] = col[2 * y + 1];
        }
    }
    free(col);
    return 0;
}

int orc_dft_brute2d(const double* in, double* out, int n, int inverse)
{
    if (!in || !out || n < 1) return -1;
    double sign = inverse ? 1.0 : -1.0;
    for (int ky = 0; ky < n; ky++)
        for (int kx = 0; kx < n; kx++) {
            double sr = 0.0, si = 0.0;
            for (int y = 0; y < n; y++)
                for (int x = 0; x < n; x++) {
                    long e = ((long)x * kx + (long)y * ky) % n;
                    double ang = 2.0 * M_PI * (double)e / (double)n;
                    double wr = cos(ang), wi = sign * sin(ang);
                    const double* v = in + 2 * ((size_t)y * n + x);
                    sr += v[0] * wr - v[1] * wi;
                    si += v[0] * wi + v[1] * wr;
                }
            out[2 * ((size_t)ky * n + kx)] = sr;
            out[2 * ((size_t)ky * n + kx) + 1] = si;
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* The cavity map                                                      */
/* ------------------------------------------------------------------ */

static int params_ok(const orc_params* p)
{
    if (!p || !length_ok(p->N) || p->N < 2) return 0;
    if (!(p->dx > 0.0) || !(p->lambda > 0.0) || !(p->L >= 0.0)) return 0;
    if (!(p->R > 0.0) || !(p->R <= 1.0)) return 0;
    if (!(p->T1 > 0.0)) return 0;
    if (p->ap_kind < 0 || p->ap_kind > 3) return 0;
    if ((p->ap_kind == 1 || p->ap_kind == 2) && !(p->ap_radius > 0.0)) return 0;
    if (p->ap_kind == 1 && p->ap_order < 1) return 0;
    if (p->ap_kind == 3 && !p->ap_mask) return 0;
    if (!(p->filter_delta >= 0.0) || !isfinite(p->filter_delta)) return 0;
    if (p->model < 0 || p->model > 2) return 0;
    if (p->slices < 0) return 0;
    if (p->transfer && (p->filter_delta > 0.0 || p->slices > 1)) return 0;
    return 1;
}

static double coord(int j, const orc_params* p)
{
    return ((double)j - 0.5 * (double)p->N) * p->dx;
}

static int signed_index(int q, int n)
{
    return (2 * q < n) ? q : q - n;
}

/* Complex aperture D of Eq. (12) at grid point (x, y): modulus D0 (finite
 * width of gain region / mirror) times the phase exp(i k r^2 / (2F) + i psi)
 * of a mirror of focal length F with surface roughness psi(x, y).  D0 is the
 * super-Gaussian exp(-(r/r0)^m), the Gaussian exp(-r^2/(2 r0^2)) of Eq. (26)
 * (exponent read as 2 D_a^2, as in Eq. (27)), 1, or a user mask. */
static void aperture(const orc_params* p, int y, int x, double* ar, double* ai)
{
    double xx = coord(x, p), yy = coord(y, p);
    double r2 = xx * xx + yy * yy;
    double amp, ph = 0.0;
    switch (p->ap_kind) {
    case 1: amp = exp(-pow(r2 / (p->ap_radius * p->ap_radius), 0.5 * p->ap_order)); break;
    case 2: amp = exp(-r2 / (2.0 * p->ap_radius * p->ap_radius)); break;
    case 3: amp = p->ap_mask[(size_t)y * p->N + x]; break;
    default: amp = 1.0; break;
    }
    if (p->focal != 0.0 && isfinite(p->focal)) {
        double k = 2.0 * M_PI / p->lambda;
        ph = k * r2 / (2.0 * p->focal);
    }
    if (p->rough) ph += p->rough[(size_t)y * p->N + x];
    *ar = amp * cos(ph);
    *ai = amp * sin(ph);
}

/* Pump N0(r): uniform, or the spatially periodic gain N0(r) = N0(r + p) of
 * Sec. 3 in the form N0 (1 + m cos(2 pi x/d) cos(2 pi y/d)). */
static double pump(const orc_params* p, int y, int x)
{
    if (p->mod_amp == 0.0 || !(p->mod_period > 0.0)) return p->N0;
    double cx = cos(2.0 * M_PI * coord(x, p) / p->mod_period);
    double cy = cos(2.0 * M_PI * coord(y, p) / p->mod_period);
    return p->N0 * (1.0 + p->mod_amp * cx * cy);
}

/* Amplitude factor of the gain sheet for inversion Nn and incident
 * intensity I.  B-class (models 0, 1): the inversion is frozen during the
 * pass (Intro), amplitude gain exp(N/2).  Class A (model 2, Sec. 2.1,
 * Eq. (8)): the gain term sigma N / (2 (1 + sigma T1 |E|^2)) integrated over
 * one round trip with |E|^2 frozen, i.e. amplitude gain
 * exp(N / (2 (1 + T1 I))). */
static double gain_amp(const orc_params* p, double Nn, double I)
{
    if (p->model == 2) return exp(0.5 * Nn / (1.0 + p->T1 * I));
    return exp(0.5 * Nn);
}

/* Inversion after one round trip, from Nn, the local pump level P and the
 * incident intensity I (sigma = 1, time in round trips).
 * Model 0: forward Euler of dN/dt = (P - N)/T1 - N I, the reading of the
 *          second line of Eq. (1).
 * Model 1: the same equation (Eq. (6)) solved exactly over one trip with I
 *          frozen: N relaxes to N_eq = P / (1 + T1 I) at rate 1/T1 + I.
 * Model 2: class A: the inversion follows the pump adiabatically; the state
 *          holds the pump level and saturation acts through gain_amp. */
static double inversion_next(const orc_params* p, double Nn, double P, double I)
{
    if (p->model == 1) {
        double rate = 1.0 / p->T1 + I;
        double neq = P / (1.0 + p->T1 * I);
        return neq + (Nn - neq) * exp(-rate);
    }
    if (p->model == 2) return P;
    return Nn + (P - Nn) / p->T1 - Nn * I;
}

int orc_run(const orc_params* p, double* E, double* Ninv, int n_trips,
            double* trace)
{
    if (!params_ok(p) || !E || !Ninv || n_trips < 0) return -1;
    const int N = p->N;
    const size_t NN = (size_t)N * N;
    /* m thin sheets per iterate (Sec. 2.2, after Eq. (12)); m = 1 is Eq. (1) */
    const int m = p->slices > 1 ? p->slices : 1;
    double* A = (double*)malloc(sizeof(double) * 2 * NN);   /* complex aperture */
    double* P0 = (double*)malloc(sizeof(double) * NN);      /* pump map of one sheet */
    double* H = (double*)malloc(sizeof(double) * 2 * NN);   /* transfer function */
    double* G = (double*)malloc(sizeof(double) * 2 * NN);
    if (!A || !P0 || !H || !G) { free(A); free(P0); free(H); free(G); return -1; }

    for (int y = 0; y < N; y++)
        for (int x = 0; x < N; x++) {
            size_t i = (size_t)y * N + x;
            aperture(p, y, x, &A[2 * i], &A[2 * i + 1]);
            /* each of the m sheets holds 1/m of the medium's pumped gain */
            P0[i] = pump(p, y, x) / (double)m;
        }
    /* Free-space transfer function of the operator exponent exp[iL/(2k) Lap]
     * (Sec. 2.3, Eq. (25)): the Laplacian is -4 pi^2 (fx^2 + fy^2) in Fourier
     * space and k = 2 pi / lambda, so H = exp(-i pi lambda L (fx^2 + fy^2)).
     * It is the Fourier transform of the Fresnel kernel of Eqs. (11), (13).
     * With m sheets it is taken for the distance L/m between two sheets. */
    /* With filter_delta > 0 the nonlocal step is instead the real kernel of
     * the renormalization-group fixed point (Sec. 2.3, Eq. (18)), the
     * operator exp[(Delta^2/2) d^2/dx^2] applied along both transverse axes:
     * in Fourier space d^2/dx^2 -> -4 pi^2 fx^2, so
     * H = exp(-2 pi^2 Delta^2 (fx^2 + fy^2)), real and at most 1.  With m
     * sheets each step applies variance Delta^2/m, so that m steps make the
     * whole filter (exponents add). */
    const double Ls = p->L / (double)m;
    const double d2 = p->filter_delta * p->filter_delta / (double)m;
    for (int q = 0; q < N; q++)
        for (int pp = 0; pp < N; pp++) {
            double fx = signed_index(pp, N) / (N * p->dx);
            double fy = signed_index(q, N) / (N * p->dx);
            size_t i = (size_t)q * N + pp;
            if (p->transfer) {
                /* a general nonlocal step: the convolution of Eq. (10) with
                 * the caller's kernel, as its transfer function */
                H[2 * i] = p->transfer[2 * i];
                H[2 * i + 1] = p->transfer[2 * i + 1];
            } else if (p->filter_delta > 0.0) {
                H[2 * i] = exp(-2.0 * M_PI * M_PI * d2 * (fx * fx + fy * fy));
                H[2 * i + 1] = 0.0;
            } else {
                double ph = M_PI * p->lambda * Ls * (fx * fx + fy * fy);
                H[2 * i] = cos(ph);
                H[2 * i + 1] = -sin(ph);
            }
        }
    const double sqR = sqrt(p->R);
    const double inv_nn = 1.0 / ((double)N * (double)N);

    for (int t = 0; t < n_trips; t++) {
        for (int k = 0; k < m; k++) {
            double* Nk = Ninv + (size_t)k * NN;      /* inversion of sheet k */
            double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
            for (size_t i = 0; i < NN; i++) {
                double er = E[2 * i], ei = E[2 * i + 1];
                double I = er * er + ei * ei;        /* |E|^2 incident on the sheet */
                double Nn = Nk[i];
                double g = gain_amp(p, Nn, I);       /* gain sheet, amplitude */
                if (k == 0) {
                    /* the sheet at the mirror: local step f of Eq. (1),
                     * G = sqrt(R) A g E_n (g = exp(N_n/2) for B class) */
                    double a2 = A[2 * i] * A[2 * i] + A[2 * i + 1] * A[2 * i + 1];
                    s1 += I;
                    s2 += a2 * I;
                    s3 += a2 * g * g * I;
                    s4 += Nn;
                    double fr = sqR * g * er, fi = sqR * g * ei;
                    G[2 * i] = A[2 * i] * fr - A[2 * i + 1] * fi;
                    G[2 * i + 1] = A[2 * i] * fi + A[2 * i + 1] * fr;
                } else {
                    /* a sheet away from the mirror: gain only */
                    G[2 * i] = g * er;
                    G[2 * i + 1] = g * ei;
                }
                /* inversion: relaxation toward the pump, depletion by |E|^2 */
                Nk[i] = inversion_next(p, Nn, P0[i], I);
            }
            if (k == 0 && trace) {
                trace[4 * (size_t)t + 0] = s1;
                trace[4 * (size_t)t + 1] = s2;
                trace[4 * (size_t)t + 2] = s3;
                trace[4 * (size_t)t + 3] = s4;
            }
            /* nonlocal step to the next sheet: E <- IFFT2(H . FFT2(G)) */
            if (orc_fft2(G, N, 0)) goto fail;
            for (size_t i = 0; i < NN; i++) {
                double gr = G[2 * i], gi = G[2 * i + 1];
                G[2 * i] = gr * H[2 * i] - gi * H[2 * i + 1];
                G[2 * i + 1] = gr * H[2 * i + 1] + gi * H[2 * i];
            }
            if (orc_fft2(G, N, 1)) goto fail;
            for (size_t i = 0; i < 2 * NN; i++) E[i] = G[i] * inv_nn;
        }
    }
    free(A); free(P0); free(H); free(G);
    return 0;
fail:
    free(A); free(P0); free(H); free(G);
    return -1;
}

int orc_propagate(const orc_params* p, double* E, double z)
{
    if (!params_ok(p) || !E || !(z >= 0.0) || !isfinite(z)) return -1;
    const int N = p->N;
    const size_t NN = (size_t)N * N;
    if (orc_fft2(E, N, 0)) return -1;
    for (int q = 0; q < N; q++)
        for (int pp = 0; pp < N; pp++) {
            double fx = signed_index(pp, N) / (N * p->dx);
            double fy = signed_index(q, N) / (N * p->dx);
            double ph = M_PI * p->lambda * z * (fx * fx + fy * fy);
            size_t i = (size_t)q * N + pp;
            double hr = cos(ph), hi = -sin(ph);
            double er = E[2 * i], ei = E[2 * i + 1];
            E[2 * i] = er * hr - ei * hi;
            E[2 * i + 1] = er * hi + ei * hr;
        }
    if (orc_fft2(E, N, 1)) return -1;
    const double inv_nn = 1.0 / ((double)N * (double)N);
    for (size_t i = 0; i < 2 * NN; i++) E[i] *= inv_nn;
    return 0;
}

int orc_nbins(int N)
{
    /* largest radius is |(N/2, N/2)| = N / sqrt(2) */
    return (int)floor((double)N / sqrt(2.0) + 0.5) + 1;
}

int orc_spectrum(const orc_params* p, const double* E, const double* Ninv,
                 double* radial, int nbins)
{
    if (!params_ok(p) || !E || !Ninv || !radial) return -1;
    const int N = p->N;
    if (nbins < orc_nbins(N)) return -1;
    const size_t NN = (size_t)N * N;
    double* G = (double*)malloc(sizeof(double) * 2 * NN);
    if (!G) return -1;
    const double sqR = sqrt(p->R);
    for (int y = 0; y < N; y++)
        for (int x = 0; x < N; x++) {
            size_t i = (size_t)y * N + x;
            double ar, ai;
            aperture(p, y, x, &ar, &ai);
            double I = E[2 * i] * E[2 * i] + E[2 * i + 1] * E[2 * i + 1];
            double g = sqR * gain_amp(p, Ninv[i], I);
            double fr = g * E[2 * i], fi = g * E[2 * i + 1];
            G[2 * i] = ar * fr - ai * fi;
            G[2 * i + 1] = ar * fi + ai * fr;
        }
    if (orc_fft2(G, N, 0)) { free(G); return -1; }
    for (int k = 0; k < nbins; k++) radial[k] = 0.0;
    for (int q = 0; q < N; q++)
        for (int pp = 0; pp < N; pp++) {
            long a = signed_index(pp, N), b = signed_index(q, N);
            long s = a * a + b * b;
            /* round(sqrt(s)); s is an integer, so sqrt(s) never sits on .5 */
            int k = (int)floor(sqrt((double)s) + 0.5);
            size_t i = (size_t)q * N + pp;
            radial[k] += G[2 * i] * G[2 * i] + G[2 * i + 1] * G[2 * i + 1];
        }
    free(G);
    int best = -1;
    double bv = -1.0;
    for (int k = 1; k < nbins; k++)
        if (radial[k] > bv) { bv = radial[k]; best = k; }
    return best;
}
