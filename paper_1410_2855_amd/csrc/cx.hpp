// cx.hpp -- complex arithmetic in registers and compile-time trigonometry.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <utility>

namespace lsr {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// The library is compiled with -ffp-contract=off, so every rounding is the one
// written here: fused multiply-adds are explicit.  This keeps a split run
// (trip kernels launched separately) bitwise equal to a continuous one.
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {fma_(a.re, b.re, -(a.im * b.im)), fma_(a.re, b.im, a.im * b.re)};
}
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// a * (DIR * i): DIR = -1 gives -i (forward quarter turn), +1 gives +i.
template <int DIR, typename T>
__device__ __forceinline__ cx<T> rot_q(cx<T> a) {
    if constexpr (DIR > 0) return {-a.im, a.re};
    else return {a.im, -a.re};
}

// Global memory access at a 32-bit byte offset from a uniform base.  The
// pointers of a cavity reach the kernels inside a descriptor, so the compiler
// cannot tell they address global memory and would emit flat accesses with a
// 64-bit address each; the cast to the global address space and the 32-bit
// offset let it use global_load/store with a scalar base and a 32-bit vector
// offset.  A cavity's arrays are far below 4 GiB.
// (The host pass of this single-source file parses device functions too;
// there the qualifier is dropped.)
#if defined(__HIP_DEVICE_COMPILE__)
#define LSR_GLOBAL __attribute__((address_space(1)))
#else
#define LSR_GLOBAL
#endif
// CST is a compile-time byte offset applied on the pointer side, so it folds
// into the instruction's immediate offset.
template <typename V, int CST = 0>
__device__ __forceinline__ V gld(const void* base, unsigned byte_off) {
    const LSR_GLOBAL char* b = (const LSR_GLOBAL char*)base + CST;
    return *(const LSR_GLOBAL V*)(b + byte_off);
}
template <typename V, int CST = 0>
__device__ __forceinline__ void gst(void* base, unsigned byte_off, const V& v) {
    LSR_GLOBAL char* b = (LSR_GLOBAL char*)base + CST;
    *(LSR_GLOBAL V*)(b + byte_off) = v;
}

// Streaming forms for data touched once per pass (the field and the
// inversion): non-temporal loads and stores, so the stream neither allocates
// nor keeps lines in the caches that hold the reused tables.  The value goes
// through the clang vector type of the same size.
template <typename V> struct NtVec;
template <> struct NtVec<float> { using type = float; };
template <> struct NtVec<double> { using type = double; };
template <> struct NtVec<float4> { using type = float __attribute__((ext_vector_type(4))); };
template <> struct NtVec<double2> { using type = double __attribute__((ext_vector_type(2))); };

template <typename V, int CST = 0>
__device__ __forceinline__ V gld_nt(const void* base, unsigned byte_off) {
    using W = typename NtVec<V>::type;
    static_assert(sizeof(W) == sizeof(V), "streaming type size");
    const LSR_GLOBAL char* b = (const LSR_GLOBAL char*)base + CST;
    const W w = __builtin_nontemporal_load((const LSR_GLOBAL W*)(b + byte_off));
    V v;
    __builtin_memcpy(&v, &w, sizeof(V));
    return v;
}
template <typename V, int CST = 0>
__device__ __forceinline__ void gst_nt(void* base, unsigned byte_off, const V& v) {
    using W = typename NtVec<V>::type;
    W w;
    __builtin_memcpy(&w, &v, sizeof(V));
    LSR_GLOBAL char* b = (LSR_GLOBAL char*)base + CST;
    __builtin_nontemporal_store(w, (LSR_GLOBAL W*)(b + byte_off));
}

// Compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// Compile-time sin/cos (Taylor series after reduction to [-pi, pi]); used
// only for the constant twiddles inside the small register DFTs.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ce_reduce(double x) {
    while (x > kPi) x -= 2.0 * kPi;
    while (x < -kPi) x += 2.0 * kPi;
    return x;
}
constexpr double ce_sin(double x) {
    x = ce_reduce(x);
    double term = x, sum = x;
    for (int n = 1; n < 40; ++n) {
        term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ce_cos(double x) {
    x = ce_reduce(x);
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 40; ++n) {
        term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}

}  // namespace lsr
