// shapes.hpp -- compile-time description of the per-line FFT of each grid
// size: lanes per line, lines per workgroup, and the Stockham radix sequence.
// Shared by host (table builders, packer) and device (kernels).
//
// A "line" is one row (row pass) or one column (column pass) of the N x N
// grid.  A line is transformed by L lanes, each holding P = N/L points in
// registers; a workgroup handles LPW lines.  The same LPW is the edge of the
// square tile of the internal field layout (layout notes in map.hpp):
// row-pass workgroups own LPW consecutive rows, column-pass workgroups LPW
// consecutive columns, and every global access is a whole LPW x LPW tile.
//
// Forward passes use RAD[0..NP-1] in order; inverse passes the reverse order,
// so the inverse's last radix equals the forward's first (and vice versa) and
// the register layout at the end of one transform is the start layout of the
// next: the row pass goes inverse -> local step -> forward and the column
// pass forward -> propagator -> inverse with no LDS exchange at the seam.
#pragma once

#include <cstdint>

namespace lsr {

enum : int { FWD = -1, INV = +1 };   // sign of the DFT exponent

template <int N_, int L_, int LPW_, int... R>
struct Shape {
    static constexpr int N = N_;
    static constexpr int L = L_;
    static constexpr int LPW = LPW_;
    static constexpr int P = N_ / L_;
    static constexpr int THREADS = L_ * LPW_;
    static constexpr int NP = sizeof...(R);

    static constexpr int rad_fwd(int s) {
        constexpr int a[] = {R...};
        return a[s];
    }
    // radix of pass s in direction dir
    static constexpr int rad(int dir, int s) {
        return dir == FWD ? rad_fwd(s) : rad_fwd(NP - 1 - s);
    }
    // product of the radices of the passes before s (Stockham sub-length)
    static constexpr int ns(int dir, int s) {
        int p = 1;
        for (int i = 0; i < s; ++i) p *= rad(dir, i);
        return p;
    }
    static constexpr int prod() {
        int p = 1;
        for (int i = 0; i < NP; ++i) p *= rad_fwd(i);
        return p;
    }
    // twiddle-table segment of pass s: Ns*R entries (see tw_index) when Ns > 1
    static constexpr int tw_len(int dir, int s) { return ns(dir, s) > 1 ? ns(dir, s) * rad(dir, s) : 0; }
    static constexpr int tw_off(int dir, int s) {
        int o = 0;
        if (dir == INV)
            for (int i = 0; i < NP; ++i) o += tw_len(FWD, i);
        for (int i = 0; i < s; ++i) o += tw_len(dir, i);
        return o;
    }
    static constexpr int TW_TOTAL = tw_off(INV, NP);

    // LDS: one padded line per handled line; one spare element per 16 keeps
    // the Stockham scatter of small sub-lengths free of bank conflicts, and a
    // line stride of 4 (mod 16) elements puts the LPW lines a staging chunk
    // row touches on different banks.
    static constexpr int pad(int i) { return i + (i >> 4); }
    static constexpr int LINE = ((N_ + (N_ >> 4) + 15) / 16) * 16 + 4;
    static constexpr int LDS_ELEMS = LPW_ * LINE;

    static constexpr bool valid() {
        if (prod() != N_ || N_ % L_ != 0 || N_ % LPW_ != 0) return false;
        for (int i = 0; i < NP; ++i)
            if (P % rad_fwd(i) != 0) return false;
        if (THREADS > 1024 || THREADS % 64 != 0) return false;
        if (L_ > 64 && L_ % 64 != 0) return false;
        if (64 % L_ != 0 && L_ < 64) return false;
        return true;
    }
};

// Position of twiddle w^(r k) (sub-transform k < Ns, r < R) inside its pass's
// segment.  Lanes of a wave hold consecutive k, so the table is laid out for
// contiguous loads across lanes: with pairs (complex FP32 entries, R even) the
// two twiddles r, r+1 of one k are adjacent and consecutive k follow, so one
// 16-byte load per lane reads a pair and a wave reads 1 KB contiguous;
// otherwise (complex FP64) the table is r-major, entry r*Ns + k.
constexpr int tw_index(int Ns, int R, int k, int r, bool pairs) {
    return (pairs && R % 2 == 0) ? (r / 2) * 2 * Ns + 2 * k + (r % 2) : r * Ns + k;
}

// ---------------------------------------------------------------------------
// The compiled shapes.  FP32 complex field (8 B/point):
using S256  = Shape<256, 16, 16, 16, 16>;
using S384  = Shape<384, 32, 8, 12, 4, 4, 2>;
using S512  = Shape<512, 32, 8, 8, 8, 8>;
using S768  = Shape<768, 64, 4, 12, 4, 4, 4>;
using S1024 = Shape<1024, 64, 4, 4, 16, 16>;
using S2048 = Shape<2048, 128, 4, 8, 16, 16>;
using S4096 = Shape<4096, 256, 4, 16, 16, 16>;
// Alternative plans for batches, chosen per grid size by the autotuner: the
// same transform with another radix order (r) or with 8 x 8 tiles of eight
// lines per workgroup (t).  Each pass is a whole 1D DFT in natural order, so
// only the twiddle table and the tile edge go with the choice.
using S512r  = Shape<512, 32, 8, 16, 8, 4>;
using S1024r = Shape<1024, 64, 4, 16, 16, 4>;
using S1024t = Shape<1024, 64, 8, 4, 16, 16>;
using S2048r = Shape<2048, 128, 4, 16, 16, 8>;
// 4096 with half the lanes per line (32 points per lane, 512 threads): the
// same 4 x 4 tiles and LDS, two waves per SIMD with the registers to hold
// every value without spilling.
using S4096w = Shape<4096, 128, 4, 16, 16, 16>;
// A one-cavity plan of 256 can take a shape with 8 points per lane instead
// of 16 (lsr_plan_set_fft_plan): a lone small cavity keeps few workgroups
// busy, so its passes are bound by the chain of dependent instructions of a
// lane, which fewer points per lane shorten (15.7 -> 11.8 us per trip).
// Shapes of 8 points per lane for 1024 (128 lanes, radices 8 8 4 4) and
// 2048 (256 lanes, 8 8 8 4) measured slower than the defaults (22.3 ->
// 24.3 and 44.5 -> 57.2 us): their lines span several waves, so every
// exchange becomes a workgroup barrier.
using L256  = Shape<256, 32, 8, 8, 8, 4>;
// Four points per lane (a wave per line, radix 4 throughout) on four or two
// lines per workgroup: the shortest per-lane chain for a lone 256^2 cavity.
using L256q = Shape<256, 64, 4, 4, 4, 4, 4>;
using L256p = Shape<256, 64, 2, 4, 4, 4, 4>;
// A wave per 2048-point line (32 points per lane): its exchanges need no
// workgroup barrier, at two waves per SIMD.
using L2048w = Shape<2048, 64, 4, 8, 16, 16>;
// FP64 complex field (16 B/point): half the lines per workgroup.
using D256  = Shape<256, 16, 8, 16, 16>;
using D384  = Shape<384, 16, 8, 8, 12, 4>;
using D512  = Shape<512, 32, 4, 8, 8, 8>;
using D768  = Shape<768, 32, 4, 8, 12, 8>;
using D1024 = Shape<1024, 64, 2, 4, 16, 16>;
using D2048 = Shape<2048, 64, 2, 8, 16, 16>;
using D4096 = Shape<4096, 256, 2, 16, 16, 16>;

static_assert(S256::valid() && S384::valid() && S512::valid() && S768::valid() &&
              S1024::valid() && S2048::valid() && S4096::valid(), "bad fp32 shape");
static_assert(S512r::valid() && S1024r::valid() && S1024t::valid() && S2048r::valid() && S4096w::valid(),
              "bad alternative shape");
static_assert(L256::valid() && L256q::valid() && L256p::valid() && L2048w::valid(), "bad one-cavity shape");
static_assert(D256::valid() && D384::valid() && D512::valid() && D768::valid() &&
              D1024::valid() && D2048::valid() && D4096::valid(), "bad fp64 shape");

// Runtime description of a shape (host side).
struct ShapeInfo {
    int N, L, LPW, NP;
    int rad[8];
    int tw_total;
    int threads;
};

template <class S>
inline ShapeInfo shape_info() {
    ShapeInfo s{};
    s.N = S::N; s.L = S::L; s.LPW = S::LPW; s.NP = S::NP;
    for (int i = 0; i < S::NP; ++i) s.rad[i] = S::rad_fwd(i);
    s.tw_total = S::TW_TOTAL;
    s.threads = S::THREADS;
    return s;
}

}  // namespace lsr
