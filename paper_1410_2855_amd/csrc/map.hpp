// map.hpp -- the round trip as workgroup tasks: row blocks and column blocks.
//
// One round trip of the cavity map (paper, Intro Eq. (1); Sec. 2.2 Eqs.
// (11)-(12); diffraction as the operator exponent of Sec. 2.3 Eq. (25)):
//     G       = sqrt(R) A exp(N_n/2) E_n              local step
//     N_{n+1} = N_n + (N0 - N_n)/T1 - N_n |E_n|^2      inversion update
//     E_{n+1} = IFFT2( H FFT2(G) )                    diffraction
// is carried by two streaming passes over the field:
//   row task (LPW rows):  [inverse row DFT of trip n-1] -> E_n -> local step,
//                         inversion update, diagnostics sums -> forward row DFT
//   column task (LPW columns): forward column DFT -> x H -> inverse column DFT
// so trip n's inverse row DFT is fused with trip n+1's local step and
// forward row DFT.  Each pass reads and writes the field once: 24 B/point for
// the row pass (field and inversion), 16 B/point for the column pass.
//
// Internal field layout between passes ("tiled"): the N x N array is cut into
// LPW x LPW tiles stored contiguously, tiles ordered row-block-major, and
// elements row-major inside a tile.  Row block rb (rows rb*LPW..) is then one
// contiguous span, exactly the span rows rb*LPW.. occupy in row-major order,
// so the first and last row passes convert in place; column block cb is N/LPW
// tiles, each contiguous, one row block apart.  Every global access covers
// whole tiles (>= 128 B for the FP32 shapes), independent of N.
#pragma once

#include "desc.hpp"
#include "fft.hpp"

namespace lsr {

template <typename T> struct V16;
template <> struct V16<float> { using type = float4; };
template <> struct V16<double> { using type = double2; };

template <typename T> constexpr int EPC = 16 / (int)sizeof(cx<T>);  // elements per 16-byte chunk

template <typename T>
__device__ __forceinline__ void unpack16(const typename V16<T>::type& q, cx<T>* e) {
    if constexpr (sizeof(T) == 4) {
        e[0] = {q.x, q.y};
        e[1] = {q.z, q.w};
    } else {
        e[0] = {q.x, q.y};
    }
}
template <typename T>
__device__ __forceinline__ typename V16<T>::type pack16(const cx<T>* e) {
    if constexpr (sizeof(T) == 4) return float4{e[0].re, e[0].im, e[1].re, e[1].im};
    else return double2{e[0].re, e[0].im};
}

// exp(x) as 2^(x log2 e): one v_exp_f32 (1-ulp hardware 2^x) for FP32, the
// library exp for FP64.  The FP32 form feeds only the gain and aperture
// factors, whose arguments are O(1) where the factors matter.
__device__ __forceinline__ float ex(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896340736f); }
__device__ __forceinline__ double ex(double x) { return exp(x); }
// 2^x: v_exp_f32 for FP32, the library exp2 for FP64
__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double ex2(double x) { return exp2(x); }
// log2(e) / 2: exp(n/2) = 2^(n log2(e)/2), one multiply
template <typename T> constexpr T HALF_LOG2E = (T)0.72134752044448170367996234050095;
__device__ __forceinline__ void sc(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sc(double x, double* s, double* c) { sincos(x, s, c); }

__device__ __forceinline__ int signed_idx(int q, int n) { return (2 * q < n) ? q : q - n; }

// threadIdx.x hidden from loop-invariant code motion: in the persistent
// kernel every lane-dependent address would otherwise be hoisted out of the
// task loop and held in registers across all tasks.
// RANGE: tell the compiler the value is still a thread index (non-negative,
// below the largest workgroup), so lane, line and Stockham index arithmetic
// by constants becomes unsigned shifts and masks: 12% fewer vector
// instructions in the 1024-point column pass.  The row pass goes without:
// there the compiler then keeps 4 more registers, over the budget of four
// waves per SIMD.
template <bool RANGE = true>
__device__ __forceinline__ int opaque_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    if constexpr (RANGE) __builtin_assume(t >= 0 && t < 1024);
    return t;
}

// round(sqrt(s)) for an integer s >= 0, exactly: k with k^2 - k < s <= k^2 + k.
__device__ __forceinline__ int round_sqrt(int s) {
    int k = (int)(sqrtf((float)s) + 0.5f);
    while ((long long)k * k + k < s) ++k;
    while (k > 0 && (long long)k * k - k >= s) --k;
    return k;
}

// ---------------------------------------------------------------------------
// Staging between HBM and the LDS line buffers (16-byte chunks).
// Row spans: LAYOUT 0 = row-major rows, 1 = tiled row block.
template <class S, typename T, int LAYOUT>
__device__ __forceinline__ void row_chunk_pos(int c, int& l, int& x) {
    const int o = c * EPC<T>;
    if constexpr (LAYOUT == 0) {
        l = o / S::N;
        x = o % S::N;
    } else {
        constexpr int TT = S::LPW * S::LPW;
        const int t = o / TT, rem = o % TT;
        l = rem / S::LPW;
        x = t * S::LPW + rem % S::LPW;
    }
}

// A thread stages chunks c = tid + i THREADS.  Chunk i then lies a fixed
// distance after chunk 0 on every lane: in a tiled row span i EPC THREADS/TT
// whole tiles later (same line, RSTEP i positions further on), in row-major
// rows i EPC THREADS elements later.  The advances are multiples of 16, so
// the padded LDS slot is chunk 0's plus a compile-time offset (an immediate
// of the LDS instruction) rather than recomputed for every chunk.
template <class S, typename T> constexpr int RSTEP = EPC<T> * S::THREADS / S::LPW;
// whether chunk i's slot is chunk 0's plus a constant (row-major spans: when
// the staging stride and N divide one another)
template <class S, typename T, int LAYOUT>
constexpr bool row_slots_shift() {
    constexpr int ST = EPC<T> * S::THREADS;
    if constexpr (LAYOUT == 1) return ST % (S::LPW * S::LPW) == 0 && RSTEP<S, T> % 16 == 0;
    else return ST % 16 == 0 && (ST % S::N == 0 || S::N % ST == 0);
}
template <class S, typename T, int LAYOUT>
constexpr int row_slot_delta(int i) {
    constexpr int ST = EPC<T> * S::THREADS;
    if constexpr (LAYOUT == 1) {
        return i * (RSTEP<S, T> + RSTEP<S, T> / 16);
    } else {
        // whole rows (i ST)/N further on, and within the row (i ST) mod N
        // positions further on (0 when ST is a multiple of N)
        return (i * ST / S::N) * S::LINE + (i * ST % S::N) + (i * ST % S::N) / 16;
    }
}

// Chunks of a row span a workgroup thread stages.
template <class S, typename T> constexpr int ROW_IT = S::LPW * S::N / EPC<T> / S::THREADS;

template <class S, typename T>
__device__ __forceinline__ void load_rows(const cx<T>* __restrict__ blk, typename V16<T>::type* q, int tid) {
    using V = typename V16<T>::type;
    static_assert((S::LPW * S::N / EPC<T>) % S::THREADS == 0, "row staging must tile the workgroup");
    sfor<0, ROW_IT<S, T>>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        q[i] = gld_nt<V, 16 * i * S::THREADS>(blk, 16u * (unsigned)tid);
    });
}

template <class S, typename T, int LAYOUT>
__device__ __forceinline__ void commit_rows(const typename V16<T>::type* q, cx<T>* lds, int tid) {
    if constexpr (row_slots_shift<S, T, LAYOUT>()) {
        int l, x;
        row_chunk_pos<S, T, LAYOUT>(tid, l, x);
        cx<T>* base = lds + l * S::LINE + S::pad(x);   // x is a multiple of EPC: the chunk stays in a 16-block
        sfor<0, ROW_IT<S, T>>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            cx<T> e[EPC<T>];
            unpack16<T>(q[i], e);
            sfor<0, EPC<T>>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                base[row_slot_delta<S, T, LAYOUT>(i) + k] = e[k];
            });
        });
    } else {
        sfor<0, ROW_IT<S, T>>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            int l, x;
            row_chunk_pos<S, T, LAYOUT>(tid + i * S::THREADS, l, x);
            cx<T> e[EPC<T>];
            unpack16<T>(q[i], e);
            sfor<0, EPC<T>>([&](auto kc) { lds[l * S::LINE + S::pad(x + decltype(kc)::value)] = e[decltype(kc)::value]; });
        });
    }
}

template <class S, typename T, int LAYOUT>
__device__ __forceinline__ void stage_out_rows(cx<T>* __restrict__ blk, const cx<T>* lds, int tid) {
    using V = typename V16<T>::type;
    constexpr int NCH = S::LPW * S::N / EPC<T>;
    constexpr int IT = NCH / S::THREADS;
    if constexpr (row_slots_shift<S, T, LAYOUT>()) {
        int l, x;
        row_chunk_pos<S, T, LAYOUT>(tid, l, x);
        const cx<T>* base = lds + l * S::LINE + S::pad(x);
        sfor<0, IT>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            cx<T> e[EPC<T>];
            sfor<0, EPC<T>>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                e[k] = base[row_slot_delta<S, T, LAYOUT>(i) + k];
            });
            gst_nt<V, 16 * i * S::THREADS>(blk, 16u * (unsigned)tid, pack16<T>(e));
        });
    } else {
        sfor<0, IT>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            int l, x;
            row_chunk_pos<S, T, LAYOUT>(tid + i * S::THREADS, l, x);
            cx<T> e[EPC<T>];
            sfor<0, EPC<T>>([&](auto kc) { e[decltype(kc)::value] = lds[l * S::LINE + S::pad(x + decltype(kc)::value)]; });
            gst_nt<V, 16 * i * S::THREADS>(blk, 16u * (unsigned)tid, pack16<T>(e));
        });
    }
}

// Column block cb of the tiled layout: tiles (i, cb), i = 0..N/LPW-1.
// Returns the chunk index relative to the block's first tile (32 bits: a
// cavity's field is below 4 GiB).
template <class S, typename T>
__device__ __forceinline__ unsigned col_chunk(int c, int& line, int& y) {
    constexpr int TT = S::LPW * S::LPW;
    constexpr int CPT = TT / EPC<T>;
    const int i = c / CPT;
    const int o = (c % CPT) * EPC<T>;
    line = o % S::LPW;
    y = i * S::LPW + o / S::LPW;
    return (unsigned)(i * S::LPW * S::N + o) / EPC<T>;
}

template <class S, typename T> constexpr int COL_IT = S::N * S::LPW / EPC<T> / S::THREADS;

template <class S, typename T>
__device__ __forceinline__ void load_cols(const cx<T>* __restrict__ E, int cb, typename V16<T>::type* q, int tid) {
    using V = typename V16<T>::type;
    static_assert(S::LPW % EPC<T> == 0, "a chunk must stay inside one tile row");
    static_assert((S::N * S::LPW / EPC<T>) % S::THREADS == 0, "column staging must tile the workgroup");
    const cx<T>* src = E + (size_t)cb * S::LPW * S::LPW;
    sfor<0, COL_IT<S, T>>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        int ln, yy;
        q[i] = gld_nt<V>(src, 16u * col_chunk<S, T>(tid + i * S::THREADS, ln, yy));
    });
}

template <class S, typename T>
__device__ __forceinline__ void commit_cols(const typename V16<T>::type* q, cx<T>* lds, int tid) {
    sfor<0, COL_IT<S, T>>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        int ln, yy;
        (void)col_chunk<S, T>(tid + i * S::THREADS, ln, yy);
        cx<T> e[EPC<T>];
        unpack16<T>(q[i], e);
        sfor<0, EPC<T>>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            lds[(ln + k) * S::LINE + S::pad(yy)] = e[k];
        });
    });
}

template <class S, typename T>
__device__ __forceinline__ void stage_out_cols(cx<T>* __restrict__ E, int cb, const cx<T>* lds, int tid) {
    using V = typename V16<T>::type;
    constexpr int NCH = S::N * S::LPW / EPC<T>;
    constexpr int IT = NCH / S::THREADS;
    cx<T>* dst = E + (size_t)cb * S::LPW * S::LPW;
    sfor<0, IT>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        int line, y;
        const unsigned off = col_chunk<S, T>(tid + i * S::THREADS, line, y);
        cx<T> e[EPC<T>];
        sfor<0, EPC<T>>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            e[k] = lds[(line + k) * S::LINE + S::pad(y)];
        });
        gst_nt<V>(dst, 16u * off, pack16<T>(e));
    });
}

// ---------------------------------------------------------------------------
// Reductions (wave64 butterflies, then LDS across waves, fixed order).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

template <class S>
__device__ __forceinline__ void block_sums_store(double* acc, double* red, double* out, int tid) {
    constexpr int NW = S::THREADS / 64;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = wave_sum(acc[q]);
    if ((tid & 63) == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[(tid >> 6) * 4 + q] = acc[q];
    }
    __syncthreads();
    if (tid < 4) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += red[w * 4 + tid];
        out[tid] = s;
    }
}

// Ordered reduction of a cavity's row-block partials into its trace ring;
// run by one full wavefront.  Flags the first non-finite trip.
__device__ __forceinline__ void finalize_sums(const CavDesc& d) {
    const int lane = threadIdx.x & 63;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int rb = lane; rb < d.nrb; rb += 64) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q] += d.partials[4 * rb + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = wave_sum(s[q]);
    if (lane == 0) {
        const unsigned t = d.counters[CNT_TRIPS];
        const unsigned slot = t % (unsigned)d.trace_cap;
#pragma unroll
        for (int q = 0; q < 4; ++q) d.trace[4 * (size_t)slot + q] = s[q];
        const bool bad = !isfinite(s[0]) || !isfinite(s[1]) || !isfinite(s[2]) || !isfinite(s[3]);
        if (bad && d.counters[CNT_NONFINITE] == 0u) d.counters[CNT_NONFINITE] = t + 1u;
        d.counters[CNT_TRIPS] = t + 1u;
    }
}

// ---------------------------------------------------------------------------
// Local step, inversion update and diagnostics sums on the lane's points of
// row y (register order of the first forward radix = natural x order), in
// chunks of points: the aperture power of a chunk runs as one loop uniform
// across lanes.
// MODEL is the local-step code: its low bits select the local step (0 B class
// with the Euler update, 1 B class with the update exact over a trip, 2 class
// A), MODEL_ROUGH adds the roughness factor.  A compile-time choice, so the
// default kernels carry no code or registers of the others.
template <class S, typename T, int MODE, int MODEL = 0>
__device__ __forceinline__ void local_step(cx<T>* v, const T* nv, const CavDesc& d, int y, int lane,
                                           double* acc) {
    constexpr int R = R_FIRST<S>;
    constexpr int P = S::P;
    constexpr int LS = MODEL & MODEL_MASK;
    constexpr bool ROUGH = (MODEL & MODEL_ROUGH) != 0;
    const T half = (T)(0.5 * S::N);
    const T sqR = (T)d.sqrtR, N0 = (T)d.N0, iT1 = (T)d.inv_T1;
    const int kind = d.ap_kind;
    const T* pc = static_cast<const T*>(d.pump_c);
    const cx<T>* foc = static_cast<const cx<T>*>(d.foc);
    const void* rough = d.rough;
    // byte offsets of row y from the cavity's (uniform) array bases
    const unsigned row = (unsigned)y * (unsigned)S::N * (unsigned)sizeof(T);
    // aperture coordinates in units where u = X'^2 + Y'^2 and A = 2^(-u^h);
    // a point's X' is the lane's base plus a compile-time multiple of the step
    const T st = (T)d.ap_step;
    const T Yp = ((T)y - half) * st;
    const T Y2 = Yp * Yp;
    const T Xl = ((T)lane - half) * st;

    // modulated pump N0 (1 + m c(x) c(y)) = N0 + (N0 m c(y)) c(x)
    const T pmy = pc ? (T)(d.N0 * d.mod_amp) * pc[y] : (T)0;
    const cx<T> fy = foc ? foc[y] : cx<T>{(T)1, (T)0};
    const int h = kind == AP_SUPERGAUSS ? d.ap_half_order : 1;
    // the lane's points in chunks of CH: the aperture of a chunk is computed
    // right before its points are used, so only CH aperture values and
    // radii are live at a time.  The 4096-point row kernels run at the
    // register limit of 16 waves per CU, and chunks of 4 free 12 registers
    // there (spill 48 -> 28 bytes per lane); the other shapes compute all
    // their points in one chunk (smaller chunks measured 4% slower at 1024).
    constexpr int CH = S::N >= 4096 ? 4 : P;
    static_assert(P % CH == 0, "points per lane must be a multiple of the chunk");
    sfor<0, P / CH>([&](auto cc) {
        constexpr int c0 = decltype(cc)::value * CH;
        // aperture amplitude A(x, y) of the chunk
        T A[CH];
        if (kind == AP_MASK) {
            sfor<0, CH>([&](auto jc) {
                constexpr int i = c0 + decltype(jc)::value;
                A[decltype(jc)::value] =
                    gld<T>(d.mask, row + (unsigned)sizeof(T) * (unsigned)reg_pos<S, R>(lane, i / R, i % R));
            });
        } else if (kind == AP_NONE) {
            sfor<0, CH>([&](auto jc) { A[decltype(jc)::value] = (T)1; });
        } else {
            // u = c r^2 (see aperture_step), then u^h by binary powering in
            // loops uniform across lanes (u^5: three multiplies), A = 2^(-u^h)
            T u[CH];
            sfor<0, CH>([&](auto jc) {
                constexpr int j = decltype(jc)::value, i = c0 + j;
                constexpr int off = (i / R) * S::L + (i % R) * (S::N / R);   // reg_pos less the lane
                const T X = fma_((T)off, st, Xl);
                u[j] = fma_(X, X, Y2);
            });
            int e = h;
            for (; !(e & 1); e >>= 1) sfor<0, CH>([&](auto jc) { u[decltype(jc)::value] *= u[decltype(jc)::value]; });
            sfor<0, CH>([&](auto jc) { A[decltype(jc)::value] = u[decltype(jc)::value]; });
            for (e >>= 1; e; e >>= 1) {
                sfor<0, CH>([&](auto jc) { u[decltype(jc)::value] *= u[decltype(jc)::value]; });
                if (e & 1) sfor<0, CH>([&](auto jc) { A[decltype(jc)::value] *= u[decltype(jc)::value]; });
            }
            sfor<0, CH>([&](auto jc) { A[decltype(jc)::value] = ex2(-A[decltype(jc)::value]); });
        }
        sfor<0, CH>([&](auto jc) {
            constexpr int j = decltype(jc)::value, i = c0 + j;
            constexpr int b = i / R, r = i % R;
            const unsigned x = (unsigned)reg_pos<S, R>(lane, b, r);
            const cx<T> e = v[i];
            const T n = nv[i];
            const T I = fma_(e.re, e.re, e.im * e.im);
            // amplitude gain of the sheet: frozen inversion exp(N/2) (B class),
            // or the class-A saturable gain exp(N / (2 (1 + T1 I)))
            T eh;
            if constexpr (LS == 2) eh = ex2(HALF_LOG2E<T> * n * iT1 / (iT1 + I));
            else eh = ex2(HALF_LOG2E<T> * n);
            const T A2 = A[j] * A[j];
            const T aeh = A[j] * eh;
            // bookkeeping in FP64 from the first term: a product of two
            // FP32 values is exact in FP64
            const double Id = (double)I;
            const double ad = (double)aeh;
            acc[0] += Id;
            acc[1] = fma_((double)A2, Id, acc[1]);
            acc[2] = fma_(ad * ad, Id, acc[2]);
            acc[3] += (double)n;
            cx<T> g = scale(e, sqR * aeh);
            // phase of the complex aperture: mirror curvature exp(i k r^2/(2F))
            // as the product of its x and y factors, then the roughness
            // exp(i psi(x, y)) (compiled in for the roughness kernels only)
            if (foc) g = cmul(g, cmul(gld<cx<T>>(foc, (unsigned)sizeof(cx<T>) * x), fy));
            if constexpr (ROUGH) g = cmul(g, gld<cx<T>>(rough, 2u * row + (unsigned)sizeof(cx<T>) * x));
            v[i] = g;
            if constexpr (MODE != ROW_DIAG) {
                const T pump = pc ? fma_(gld<T>(pc, (unsigned)sizeof(T) * x), pmy, N0) : N0;
                T nn;
                if constexpr (LS == 0) {
                    // forward Euler over one trip
                    nn = fma_(-n, I, fma_(pump - n, iT1, n));
                } else if constexpr (LS == 1) {
                    // exact over one trip with I frozen: relax to N_eq at rate 1/T1 + I
                    const T neq = pump * iT1 / (iT1 + I);
                    nn = fma_(n - neq, ex(-(iT1 + I)), neq);
                } else {
                    nn = pump;   // class A: the inversion follows the pump
                }
                gst_nt<T, (int)sizeof(T) * (b * S::L + r * (S::N / R))>(
                    d.Ninv, row + (unsigned)sizeof(T) * (unsigned)lane, nn);
            }
        });
    });
}

// ---------------------------------------------------------------------------
// A task is split into its global loads (into registers) and its body, so a
// software-pipelined kernel can issue the next task's loads while the body of
// the current one runs.  The body calls prefetch() once the loaded tile is in
// LDS and the registers are free again.
template <class S, typename T>
struct RowRegs {
    typename V16<T>::type q[ROW_IT<S, T>];
    T nv[S::P];
};

template <class S, typename T, int MODE>
__device__ __forceinline__ void row_load(const CavDesc& d, int rb, RowRegs<S, T>& in) {
    const int tid = opaque_tid<true>();
    const int line = tid / S::L, lane = tid % S::L;
    const int y = rb * S::LPW + line;
    constexpr int RF = R_FIRST<S>;
    if constexpr (MODE != ROW_LAST && MODE != ROW_FWD) {
        const unsigned row = (unsigned)y * (unsigned)S::N * (unsigned)sizeof(T);
        sfor<0, S::P / RF>([&](auto bc) {
            sfor<0, RF>([&](auto rc) {
                constexpr int b = decltype(bc)::value, r = decltype(rc)::value;
                in.nv[b * RF + r] = gld_nt<T, (int)sizeof(T) * (b * S::L + r * (S::N / RF))>(
                    d.Ninv, row + (unsigned)sizeof(T) * (unsigned)lane);
            });
        });
    }
    load_rows<S, T>(static_cast<const cx<T>*>(d.E) + (size_t)rb * S::LPW * S::N, in.q, tid);
}

// TWS / ltw: twiddle source (TW_LDS: ltw is the workgroup's LDS copy).
template <class S, typename T, int MODE, int TWS = TW_GLOBAL, int MODEL = 0, class Prefetch>
__device__ __forceinline__ void row_body(const CavDesc& d, int rb, cx<T>* lds, double* red, RowRegs<S, T>& in,
                                         Prefetch&& prefetch, const cx<T>* ltw = nullptr) {
    const int tid = opaque_tid<true>();
    const int line = tid / S::L, lane = tid % S::L;
    const int y = rb * S::LPW + line;
    cx<T>* blk = static_cast<cx<T>*>(d.E) + (size_t)rb * S::LPW * S::N;
    const cx<T>* tw = TWS == TW_LDS ? ltw : static_cast<const cx<T>*>(d.tw);
    cx<T>* myl = lds + line * S::LINE;
    constexpr int RF = R_FIRST<S>;
    constexpr int RL = R_LAST<S>;

    T nv[S::P];
    if constexpr (MODE != ROW_LAST && MODE != ROW_FWD)
        sfor<0, S::P>([&](auto ic) { nv[decltype(ic)::value] = in.nv[decltype(ic)::value]; });
    if constexpr (MODE == ROW_FIRST || MODE == ROW_DIAG || MODE == ROW_FWD) commit_rows<S, T, 0>(in.q, lds, tid);
    else commit_rows<S, T, 1>(in.q, lds, tid);
    __syncthreads();
    prefetch();

    cx<T> v[S::P];
    if constexpr (MODE == ROW_MID || MODE == ROW_LAST) {
        gather_in<S, RL>(v, myl, lane);
        line_sync<S>();
        fft_line<S, INV, TWS>(v, myl, lane, tw);
    } else {
        gather_in<S, RF>(v, myl, lane);
        line_sync<S>();
    }
    if constexpr (MODE == ROW_LAST) {
        scatter_out<S, RF>(v, myl, lane);
        __syncthreads();
        stage_out_rows<S, T, 0>(blk, lds, tid);
        return;
    } else {
        // diagnostics sums in FP64 throughout: per lane, across the wave,
        // across the workgroup
        if constexpr (MODE != ROW_FWD) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            local_step<S, T, MODE, MODEL>(v, nv, d, y, lane, acc);
            block_sums_store<S>(acc, red, d.partials + 4 * rb, tid);
        }
        fft_line<S, FWD, TWS>(v, myl, lane, tw);
        scatter_out<S, RL>(v, myl, lane);
        __syncthreads();
        cx<T>* dst = blk;
        if constexpr (MODE == ROW_DIAG || MODE == ROW_FWD)
            dst = static_cast<cx<T>*>(d.scratch) + (size_t)rb * S::LPW * S::N;
        stage_out_rows<S, T, 1>(dst, lds, tid);
    }
}

template <class S, typename T, int MODE, int MODEL = 0>
__device__ __forceinline__ void row_task(const CavDesc& d, int rb, cx<T>* lds, double* red) {
    RowRegs<S, T> in;
    row_load<S, T, MODE>(d, rb, in);
    row_body<S, T, MODE, TW_GLOBAL, MODEL>(d, rb, lds, red, in, [] {});
}

// PROP: propagator form of the column pass -- PROP_TABLE multiplies by the
// FP64-built separable table hx(p) hx(q); PROP_PHASE evaluates the phase
// pi lambda L (fx^2 + fy^2) in the field's precision (the plain form);
// PROP_TRANS multiplies by a general N x N transfer function (the map with
// kernel K of Eq. (10)), read by column: 8 more bytes per point.
enum : int { PROP_TABLE = 0, PROP_PHASE = 1, PROP_TRANS = 2 };

// Column-task registers; with HXREG the task's propagator table hx travels
// with the tile (HX_IT 16-byte chunks per thread) and is committed to LDS.
// hx(p) depends on p~^2 only, so the LDS copy keeps entries 0..N/2 (HXN,
// rounded up to whole 16-byte chunks) and is indexed by |p~|.
template <class S, typename T> constexpr int HXN = ((S::N / 2 + 1) * (int)sizeof(cx<T>) + 15) / 16 * 16 / (int)sizeof(cx<T>);
template <class S, typename T> constexpr int HX_CH = HXN<S, T> * (int)sizeof(cx<T>) / 16;
template <class S, typename T> constexpr int HX_IT = (HX_CH<S, T> + S::THREADS - 1) / S::THREADS;

template <class S, typename T, bool HXREG = false>
struct ColRegs {
    typename V16<T>::type q[COL_IT<S, T>];
    typename V16<T>::type hq[HXREG ? HX_IT<S, T> : 1];
};

template <class S, typename T, int MODE, bool HXREG = false>
__device__ __forceinline__ void col_load(const CavDesc& d, int cb, ColRegs<S, T, HXREG>& in) {
    const int tid = opaque_tid();
    const cx<T>* E = static_cast<const cx<T>*>(MODE == COL_DIAG ? d.scratch : d.E);
    load_cols<S, T>(E, cb, in.q, tid);
    if constexpr (HXREG) {
        using V = typename V16<T>::type;
        constexpr int NCH = HX_CH<S, T>;
        sfor<0, HX_IT<S, T>>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const int c = tid + i * S::THREADS;
            if (NCH % S::THREADS == 0 || c < NCH) in.hq[i] = gld<V>(d.hx, 16u * (unsigned)c);
        });
    }
}

// TWS / ltw: twiddle source; HXREG / lhx: the propagator table comes from the
// task registers through the LDS buffer lhx (HXN entries, index |p~|).
template <class S, typename T, int MODE, int PROP, int TWS = TW_GLOBAL, bool HXREG = false, class Prefetch>
__device__ __forceinline__ void col_body(const CavDesc& d, int cb, cx<T>* lds, ColRegs<S, T, HXREG>& in,
                                         Prefetch&& prefetch, const cx<T>* ltw = nullptr, cx<T>* lhx = nullptr) {
    const int tid = opaque_tid();
    const int line = tid / S::L, lane = tid % S::L;
    cx<T>* E = static_cast<cx<T>*>(MODE == COL_DIAG ? d.scratch : d.E);
    const cx<T>* tw = TWS == TW_LDS ? ltw : static_cast<const cx<T>*>(d.tw);
    cx<T>* myl = lds + line * S::LINE;
    constexpr int RF = R_FIRST<S>;
    constexpr int RL = R_LAST<S>;
    constexpr int B = S::P / RL;

    commit_cols<S, T>(in.q, lds, tid);
    if constexpr (HXREG) {
        constexpr int NCH = HX_CH<S, T>;
        sfor<0, HX_IT<S, T>>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const int c = tid + i * S::THREADS;
            if (NCH % S::THREADS == 0 || c < NCH) {
                cx<T> e[EPC<T>];
                unpack16<T>(in.hq[i], e);
                sfor<0, EPC<T>>([&](auto kc) { lhx[c * EPC<T> + decltype(kc)::value] = e[decltype(kc)::value]; });
            }
        });
    }
    __syncthreads();
    prefetch();
    cx<T> v[S::P];
    gather_in<S, RF>(v, myl, lane);
    line_sync<S>();
    fft_line<S, FWD, TWS>(v, myl, lane, tw);
    const int kx = cb * S::LPW + line;
    const int px = signed_idx(kx, S::N);

    if constexpr (MODE == COL_DIAG) {
        // far-field radial spectrum |FFT2(G)|^2 binned by round(|(p~, q~)|)
        __syncthreads();
        double* hist = reinterpret_cast<double*>(lds);
        for (int i = tid; i < d.nbins; i += S::THREADS) hist[i] = 0.0;
        __syncthreads();
        sfor<0, B>([&](auto bc) {
            sfor<0, RL>([&](auto rc) {
                constexpr int b = decltype(bc)::value, r = decltype(rc)::value;
                const int q = signed_idx(reg_pos<S, RL>(lane, b, r), S::N);
                atomicAdd(&hist[round_sqrt(px * px + q * q)], (double)norm2(v[b * RL + r]));
            });
        });
        __syncthreads();
        for (int i = tid; i < d.nbins; i += S::THREADS) d.radial_part[(size_t)cb * d.nbins + i] = hist[i];
        return;
    } else {
        // propagator H(kx, ky) = exp(-i pi lambda L (fx^2 + fy^2)) / N^2
        if constexpr (PROP == PROP_PHASE) {
            const T c = (T)d.phase_c, inn = (T)d.inv_nn;
            const int px2 = px * px;
            sfor<0, B>([&](auto bc) {
                sfor<0, RL>([&](auto rc) {
                    constexpr int b = decltype(bc)::value, r = decltype(rc)::value;
                    const int q = signed_idx(reg_pos<S, RL>(lane, b, r), S::N);
                    T s, co;
                    sc((T)(px2 + q * q) * c, &s, &co);
                    v[b * RL + r] = cmul(v[b * RL + r], cx<T>{co * inn, -s * inn});
                });
            });
        } else if constexpr (PROP == PROP_TRANS) {
            // column kx of the transfer table: N contiguous entries
            const cx<T>* tt = static_cast<const cx<T>*>(d.trans);
            const unsigned col = (unsigned)kx * (unsigned)S::N * (unsigned)sizeof(cx<T>);
            sfor<0, B>([&](auto bc) {
                sfor<0, RL>([&](auto rc) {
                    constexpr int b = decltype(bc)::value, r = decltype(rc)::value;
                    const unsigned q = (unsigned)reg_pos<S, RL>(lane, b, r);
                    v[b * RL + r] = cmul(v[b * RL + r], gld<cx<T>>(tt, col + (unsigned)sizeof(cx<T>) * q));
                });
            });
        } else if constexpr (HXREG) {
            const cx<T> hk = lhx[px < 0 ? -px : px];
            sfor<0, B>([&](auto bc) {
                sfor<0, RL>([&](auto rc) {
                    constexpr int b = decltype(bc)::value, r = decltype(rc)::value;
                    const int p = reg_pos<S, RL>(lane, b, r);
                    const int ap = p <= S::N / 2 ? p : S::N - p;
                    v[b * RL + r] = cmul(v[b * RL + r], cmul(hk, lhx[ap]));
                });
            });
        } else {
            const cx<T>* hx = static_cast<const cx<T>*>(d.hx);
            const cx<T> hk = gld<cx<T>>(hx, (unsigned)sizeof(cx<T>) * (unsigned)kx);
            sfor<0, B>([&](auto bc) {
                sfor<0, RL>([&](auto rc) {
                    constexpr int b = decltype(bc)::value, r = decltype(rc)::value;
                    const cx<T> h = cmul(hk, gld<cx<T>>(hx, (unsigned)sizeof(cx<T>) * (unsigned)reg_pos<S, RL>(lane, b, r)));
                    v[b * RL + r] = cmul(v[b * RL + r], h);
                });
            });
        }
        fft_line<S, INV, TWS>(v, myl, lane, tw);
        scatter_out<S, RF>(v, myl, lane);
        __syncthreads();
        stage_out_cols<S, T>(E, cb, lds, tid);
    }
}

template <class S, typename T, int MODE, int PROP = PROP_TABLE>
__device__ __forceinline__ void col_task(const CavDesc& d, int cb, cx<T>* lds) {
    ColRegs<S, T> in;
    col_load<S, T, MODE>(d, cb, in);
    col_body<S, T, MODE, PROP>(d, cb, lds, in, [] {});
}

}  // namespace lsr
