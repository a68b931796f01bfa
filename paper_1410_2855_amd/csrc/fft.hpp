// fft.hpp -- per-line Stockham FFT held in registers, exchanged through LDS.
//
// The nonlocal step of the cavity map (paper, Sec. 2.2, Eq. (11), evaluated
// as the operator exponent of Sec. 2.3, Eq. (25)) is diagonal in Fourier
// space; the split-step method (abstract; Sec. 2.2) reaches Fourier space
// with 2D DFTs.  Each 1D DFT of length N = R_0 R_1 ... R_{NP-1} runs as NP
// Stockham autosort passes.  Pass s (radix R, sub-length Ns = R_0...R_{s-1})
// takes butterfly j in [0, N/R):
//     x_r   = in[j + r N/R]                      r = 0..R-1
//     x_r  *= w^{r k},  k = j mod Ns,  w = exp(DIR 2 pi i/(Ns R))
//     X     = DFT_R(x)
//     out[(j div Ns) Ns R + k + r Ns] = X_r
// and the last pass leaves natural order.  A lane owns butterflies
// j = lane + b L (b < P/R); between passes the values go through the line's
// LDS buffer.  DFT_R runs in registers, composite R by one Cooley-Tukey step
// with compile-time twiddles.
#pragma once

#include "cx.hpp"
#include "shapes.hpp"

namespace lsr {

// a * exp(DIR 2 pi i M / R), constants folded at compile time.
template <int R, int M, int DIR, typename T>
__device__ __forceinline__ cx<T> twc(cx<T> a) {
    constexpr int m = ((M % R) + R) % R;
    if constexpr (m == 0) {
        return a;
    } else if constexpr (4 * m == R) {
        return rot_q<DIR>(a);
    } else if constexpr (2 * m == R) {
        return {-a.re, -a.im};
    } else if constexpr (4 * m == 3 * R) {
        return rot_q<-DIR>(a);
    } else if constexpr (8 * m == R || 8 * m == 3 * R || 8 * m == 5 * R || 8 * m == 7 * R) {
        // (+-1 +- i)/sqrt(2): two adds and two multiplies
        constexpr double th = 2.0 * kPi * m / R;
        constexpr T c = (T)ce_cos(th);
        constexpr T s = (T)(DIR * ce_sin(th));
        constexpr T h = (T)0.70710678118654752440084436210484904;
        constexpr T cs = c > 0 ? h : -h;
        constexpr T ss = s > 0 ? h : -h;
        if constexpr ((cs > 0) == (ss > 0)) {
            // c == s
            return {(a.re - a.im) * cs, (a.re + a.im) * cs};
        } else {
            // c == -s
            return {(a.re + a.im) * cs, (a.im - a.re) * cs};
        }
    } else {
        constexpr double th = 2.0 * kPi * m / R;
        constexpr T c = (T)ce_cos(th);
        constexpr T s = (T)(DIR * ce_sin(th));
        return {fma_(a.re, c, -(a.im * s)), fma_(a.re, s, a.im * c)};
    }
}

// For a twiddle exp(DIR 2 pi i M / R) of the form (+-1 +- i)/sqrt(2): the
// sign of its real part (twc scales the rotated value by that sign times
// 1/sqrt(2)); 0 for every other twiddle.
template <int R, int M, int DIR>
constexpr int half_sqrt2_sign() {
    constexpr int m = ((M % R) + R) % R;
    if constexpr (8 * m == R || 8 * m == 3 * R || 8 * m == 5 * R || 8 * m == 7 * R)
        return ce_cos(2.0 * kPi * m / R) > 0 ? 1 : -1;
    else
        return 0;
}

// twc for a (+-1 +- i)/sqrt(2) twiddle without its scale: the caller folds
// (sign) / sqrt(2) into the multiply-adds that consume the value.
template <int R, int M, int DIR, typename T>
__device__ __forceinline__ cx<T> twc_unscaled(cx<T> a) {
    constexpr int m = ((M % R) + R) % R;
    constexpr double th = 2.0 * kPi * m / R;
    constexpr bool same = (ce_cos(th) > 0) == (DIR * ce_sin(th) > 0);
    if constexpr (same) return {a.re - a.im, a.re + a.im};   // c == s
    else return {a.re + a.im, a.im - a.re};                  // c == -s
}

// a + c b, componentwise, as fused multiply-adds.
template <typename T>
__device__ __forceinline__ cx<T> fma_cx(cx<T> b, T c, cx<T> a) {
    return {fma_(b.re, c, a.re), fma_(b.im, c, a.im)};
}

// In-place DFT of length R in registers: X_k = sum_n x_n exp(DIR 2 pi i nk/R).
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* x) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        cx<T> a = x[0], b = x[1];
        x[0] = a + b;
        x[1] = a - b;
    } else if constexpr (R == 3) {
        constexpr T s3 = (T)0.86602540378443864676372317075293618;
        cx<T> t = x[1] + x[2];
        cx<T> d = scale(rot_q<DIR>(x[1] - x[2]), s3);
        cx<T> m = {fma_((T)-0.5, t.re, x[0].re), fma_((T)-0.5, t.im, x[0].im)};
        x[0] = x[0] + t;
        x[1] = m + d;
        x[2] = m - d;
    } else if constexpr (R == 4) {
        cx<T> t0 = x[0] + x[2], t1 = x[0] - x[2];
        cx<T> t2 = x[1] + x[3], t3 = rot_q<DIR>(x[1] - x[3]);
        x[0] = t0 + t2;
        x[2] = t0 - t2;
        x[1] = t1 + t3;
        x[3] = t1 - t3;
    } else {
        // R = A * B: A decimated sub-DFTs of length B, twiddles exp(DIR 2 pi i n1 k2/R),
        // then B DFTs of length A; X[k2 + B k1].
        constexpr int A = (R % 4 == 0) ? 4 : ((R % 3 == 0) ? 3 : 2);
        constexpr int B = R / A;
        // with A = 4 the (+-1 +- i)/sqrt(2) twiddles stay unscaled and their
        // scale is folded into the length-4 DFTs as fused multiply-adds
        constexpr bool FOLD = A == 4;
        cx<T> y[R];
        sfor<0, A>([&](auto n1c) {
            constexpr int n1 = decltype(n1c)::value;
            cx<T> s[B];
            sfor<0, B>([&](auto mc) { s[decltype(mc)::value] = x[n1 + A * decltype(mc)::value]; });
            dft<B, DIR>(s);
            sfor<0, B>([&](auto kc) {
                constexpr int k2 = decltype(kc)::value;
                if constexpr (FOLD && half_sqrt2_sign<R, n1 * k2, DIR>() != 0)
                    y[n1 * B + k2] = twc_unscaled<R, n1 * k2, DIR>(s[k2]);
                else
                    y[n1 * B + k2] = twc<R, n1 * k2, DIR>(s[k2]);
            });
        });
        sfor<0, B>([&](auto kc) {
            constexpr int k2 = decltype(kc)::value;
            if constexpr (FOLD) {
                constexpr T h = (T)0.70710678118654752440084436210484904;
                constexpr int g1 = half_sqrt2_sign<R, k2, DIR>();
                constexpr int g2 = half_sqrt2_sign<R, 2 * k2, DIR>();
                constexpr int g3 = half_sqrt2_sign<R, 3 * k2, DIR>();
                const cx<T> s0 = y[k2], s1 = y[B + k2], s2 = y[2 * B + k2], s3 = y[3 * B + k2];
                // t0, t1 = s0 +- g2 h s2
                cx<T> t0, t1;
                if constexpr (g2 != 0) {
                    t0 = fma_cx(s2, (T)g2 * h, s0);
                    t1 = fma_cx(s2, -(T)g2 * h, s0);
                } else {
                    t0 = s0 + s2;
                    t1 = s0 - s2;
                }
                // t2 = g1 h s1 + g3 h s3, t3 = rot(g1 h s1 - g3 h s3)
                if constexpr (g1 != 0 && g3 != 0) {
                    // common factor c = g1 h kept out: t2 = c u, t3 = c rot(v)
                    constexpr T c = (T)g1 * h;
                    const cx<T> u = g1 == g3 ? s1 + s3 : s1 - s3;
                    const cx<T> v = rot_q<DIR>(g1 == g3 ? s1 - s3 : s1 + s3);
                    x[k2] = fma_cx(u, c, t0);
                    x[k2 + 2 * B] = fma_cx(u, -c, t0);
                    x[k2 + B] = fma_cx(v, c, t1);
                    x[k2 + 3 * B] = fma_cx(v, -c, t1);
                } else {
                    cx<T> t2, d;
                    if constexpr (g1 != 0) {
                        t2 = fma_cx(s1, (T)g1 * h, s3);
                        d = fma_cx(s1, (T)g1 * h, cx<T>{-s3.re, -s3.im});
                    } else if constexpr (g3 != 0) {
                        t2 = fma_cx(s3, (T)g3 * h, s1);
                        d = fma_cx(s3, -(T)g3 * h, s1);
                    } else {
                        t2 = s1 + s3;
                        d = s1 - s3;
                    }
                    const cx<T> t3 = rot_q<DIR>(d);
                    x[k2] = t0 + t2;
                    x[k2 + 2 * B] = t0 - t2;
                    x[k2 + B] = t1 + t3;
                    x[k2 + 3 * B] = t1 - t3;
                }
            } else {
                cx<T> s[A];
                sfor<0, A>([&](auto n1c) { s[decltype(n1c)::value] = y[decltype(n1c)::value * B + k2]; });
                dft<A, DIR>(s);
                sfor<0, A>([&](auto k1c) { x[k2 + B * decltype(k1c)::value] = s[decltype(k1c)::value]; });
            }
        });
    }
}

// Synchronisation among the lanes of one line: a line inside one wavefront
// needs only a wave-level fence; a line spanning several waves a barrier.
template <class S>
__device__ __forceinline__ void line_sync() {
    if constexpr (S::L <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Load the R twiddles of sub-transform k of a pass (sub-length NS) whose
// table segment starts at entry SEG, in the tw_index layout: FP32 pairs with
// one 16-byte load per two twiddles, else one load per twiddle; either way
// the lanes of a wave (consecutive k) read contiguous memory.
template <int R, int NS, int SEG, typename T>
__device__ __forceinline__ void load_tw(cx<T>* w, const cx<T>* __restrict__ tw, int k) {
    constexpr int E = (int)sizeof(cx<T>);
    if constexpr (E == 8 && (R % 2 == 0)) {
        const unsigned off = (unsigned)k * 16u;
        sfor<0, R / 2>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            static_assert(tw_index(NS, R, 0, 2 * i, true) == 2 * i * NS, "pair layout");
            const float4 q = gld<float4, (SEG + 2 * i * NS) * E>(tw, off);
            w[2 * i] = {(T)q.x, (T)q.y};
            w[2 * i + 1] = {(T)q.z, (T)q.w};
        });
    } else {
        const unsigned off = (unsigned)k * (unsigned)E;
        sfor<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            w[i] = gld<cx<T>, (SEG + tw_index(NS, R, 0, i, false)) * E>(tw, off);
        });
    }
}

// Where the Stockham twiddles come from: TW_GLOBAL reads the plan's table
// (tw_index layout); TW_LDS reads a copy held in LDS in r-major order (entry
// r*Ns + k of a segment), so the lanes of a wave read consecutive entries.  Kernels that keep global loads in flight across the
// FFT use TW_LDS: on this ISA waiting for a later global load also waits for
// every earlier one.
enum : int { TW_GLOBAL = 0, TW_LDS = 1 };

// Butterflies of pass PASS in direction DIR on the lane's registers.
template <class S, int DIR, int PASS, int TWS = TW_GLOBAL, typename T>
__device__ __forceinline__ void pass_compute(cx<T>* v, int lane, const cx<T>* __restrict__ tw) {
    constexpr int R = S::rad(DIR, PASS);
    constexpr int Ns = S::ns(DIR, PASS);
    constexpr int B = S::P / R;
    sfor<0, B>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        cx<T>* x = v + b * R;
        if constexpr (Ns > 1) {
            const int j = lane + b * S::L;
            const int k = j % Ns;
            cx<T> w[R];
            if constexpr (TWS == TW_LDS) {
                sfor<1, R>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    w[r] = tw[S::tw_off(DIR, PASS) + r * Ns + k];
                });
            } else {
                load_tw<R, Ns, S::tw_off(DIR, PASS)>(w, tw, k);
            }
            sfor<1, R>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                x[r] = cmul(x[r], w[r]);
            });
        }
        dft<R, DIR>(x);
    });
}

// Copy a twiddle table from HBM (tw_index layout) into LDS (r-major).
template <class S, typename T>
__device__ __forceinline__ void twiddles_to_lds(const cx<T>* __restrict__ tw, cx<T>* ltw, int tid) {
    sfor<0, 2 * S::NP>([&](auto pc) {
        constexpr int dir = decltype(pc)::value < S::NP ? FWD : INV;
        constexpr int pass = decltype(pc)::value % S::NP;
        constexpr int Ns = S::ns(dir, pass);
        constexpr int R = S::rad(dir, pass);
        constexpr int off = S::tw_off(dir, pass);
        if constexpr (Ns > 1) {
            for (int i = tid; i < Ns * R; i += S::THREADS) {
                const int k = i % Ns, r = i / Ns;
                const int src = tw_index(Ns, R, k, r, sizeof(T) == 4);
                ltw[off + r * Ns + k] = gld<cx<T>>(tw, (unsigned)(sizeof(cx<T>) * (off + src)));
            }
        }
    });
}

// LDS slot of line position base + r*stride, r < R.  The padding is linear
// in r -- pad(base + r s) = pad(base) + r s + (r s)/16 -- whenever no two
// terms of the walk straddle a 16-block boundary differently: for strides
// that are multiples of 16, and for the Stockham scatter when s divides 16
// and s*R divides or is a multiple of 16 (base mod 16 < s there, or the whole
// walk stays inside one block).  Then every slot is the base slot plus a
// compile-time offset, an immediate of the LDS instruction.
template <int STRIDE, int R>
constexpr bool linear_walk() {
    return STRIDE % 16 == 0 ||
           (16 % STRIDE == 0 && ((STRIDE * R) % 16 == 0 || 16 % (STRIDE * R) == 0));
}

template <class S, int STRIDE, int R>
__device__ __forceinline__ int slot(int padded_base, int base, int r) {
    if constexpr (linear_walk<STRIDE, R>()) return padded_base + r * STRIDE + ((r * STRIDE) >> 4);
    else return S::pad(base + r * STRIDE);
}

// Write the outputs of pass PASS to their Stockham positions in the line.
template <class S, int DIR, int PASS, typename T>
__device__ __forceinline__ void pass_scatter(const cx<T>* v, cx<T>* line, int lane) {
    constexpr int R = S::rad(DIR, PASS);
    constexpr int Ns = S::ns(DIR, PASS);
    constexpr int B = S::P / R;
    sfor<0, B>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        const int j = lane + b * S::L;
        const int k = j % Ns;
        const int base = (j / Ns) * Ns * R + k;
        const int pb = S::pad(base);
        sfor<0, R>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            line[slot<S, Ns, R>(pb, base, r)] = v[b * R + r];
        });
    });
}

// Read the inputs of a pass with radix R: v[b R + r] = line[j + r N/R].
template <class S, int R, typename T>
__device__ __forceinline__ void gather_in(cx<T>* v, const cx<T>* line, int lane) {
    constexpr int B = S::P / R;
    sfor<0, B>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        const int j = lane + b * S::L;
        const int pb = S::pad(j);
        sfor<0, R>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            v[b * R + r] = line[slot<S, S::N / R, R>(pb, j, r)];
        });
    });
}

// Inverse of gather_in: line[j + r N/R] = v[b R + r] (natural order out).
template <class S, int R, typename T>
__device__ __forceinline__ void scatter_out(const cx<T>* v, cx<T>* line, int lane) {
    constexpr int B = S::P / R;
    sfor<0, B>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        const int j = lane + b * S::L;
        const int pb = S::pad(j);
        sfor<0, R>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            line[slot<S, S::N / R, R>(pb, j, r)] = v[b * R + r];
        });
    });
}

// Grid index of register v[b R + r] in the layout gather_in/scatter_out use.
template <class S, int R>
__device__ __forceinline__ int reg_pos(int lane, int b, int r) {
    return lane + b * S::L + r * (S::N / R);
}

// Radix of the first forward pass (= last inverse pass) and of the last
// forward pass (= first inverse pass).
template <class S> constexpr int R_FIRST = S::rad_fwd(0);
template <class S> constexpr int R_LAST = S::rad_fwd(S::NP - 1);

// Full 1D transform of one line.  On entry v holds the pass-0 inputs
// (gather_in order for the first radix of DIR); on exit the natural-order
// outputs in the gather_in order of the last radix of DIR.  The line buffer
// is scratch; the caller synchronises before reusing it.
template <class S, int DIR, int TWS = TW_GLOBAL, typename T>
__device__ __forceinline__ void fft_line(cx<T>* v, cx<T>* line, int lane, const cx<T>* __restrict__ tw) {
    sfor<0, S::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        pass_compute<S, DIR, p, TWS>(v, lane, tw);
        if constexpr (p + 1 < S::NP) {
            pass_scatter<S, DIR, p>(v, line, lane);
            line_sync<S>();
            gather_in<S, S::rad(DIR, p + 1)>(v, line, lane);
            line_sync<S>();
        }
    });
}

}  // namespace lsr
