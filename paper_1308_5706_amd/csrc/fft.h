// Power-of-two FFTs held in LDS for gfx950 (FP64 complex), used as the engine of the
// odd-length (2L-1) transforms through Bluestein's chirp convolution.
//
// LDS layout: element i of a column lives at pad(i) = i + i/16, so that the stride-16
// stores of the first radix-16 pass spread over all banks.  A column needs padded(P)
// double2 slots.
//
// Stockham autosort formulation: a length-P transform runs as passes of radix R in
// {16, 8, 4, 2}; pass s reads the P values with stride P/R, multiplies by the twiddles
// of the current span Ns, does an R-point DFT in registers and writes the outputs at
// their sorted positions.  The pass is in place: every thread reads its inputs, the
// workgroup synchronises, then every thread writes.  A column uses P/RM threads for a
// main radix RM.
#pragma once

#include <hip/hip_runtime.h>

namespace s2dw {
namespace fft {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

__host__ __device__ constexpr int padded(int P) { return P + P / 16; }
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// a * (SIGN i)
template <int SIGN>
__device__ __forceinline__ double2 mul_si(double2 a) {
    return SIGN > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// In-register DFTs: v'[k] = sum_r v[r] e^{SIGN 2 pi i r k / R}, natural order in and out.
template <int SIGN>
__device__ __forceinline__ void dft2(double2 *v) {
    const double2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <int SIGN>
__device__ __forceinline__ void dft4s(double2 &v0, double2 &v1, double2 &v2, double2 &v3) {
    const double2 a = cadd(v0, v2), b = csub(v0, v2), c = cadd(v1, v3), d = mul_si<SIGN>(csub(v1, v3));
    v0 = cadd(a, c);
    v2 = csub(a, c);
    v1 = cadd(b, d);
    v3 = csub(b, d);
}

template <int SIGN>
__device__ __forceinline__ void dft4(double2 *v) {
    dft4s<SIGN>(v[0], v[1], v[2], v[3]);
}

template <int SIGN>
__device__ __forceinline__ void dft8(double2 *v) {
    // n = 2 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle w8^{n2 k1}, DFT2 over n2
    constexpr double c = 0.70710678118654752440;
    dft4s<SIGN>(v[0], v[2], v[4], v[6]);
    dft4s<SIGN>(v[1], v[3], v[5], v[7]);
    v[3] = cmul(v[3], make_double2(c, SIGN * c));
    v[5] = mul_si<SIGN>(v[5]);
    v[7] = cmul(v[7], make_double2(-c, SIGN * c));
    double2 o[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        o[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
        o[k1 + 4] = csub(v[2 * k1], v[2 * k1 + 1]);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = o[i];
}

template <int SIGN>
__device__ __forceinline__ void dft16(double2 *v) {
    // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle w16^{n2 k1}, DFT4 over n2
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4s<SIGN>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // Y[n2][k1] sits at v[n2 + 4 k1]
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, c2 = 0.70710678118654752440;
    v[1 + 4 * 1] = cmul(v[1 + 4 * 1], make_double2(c1, SIGN * s1));   // w^1
    v[1 + 4 * 2] = cmul(v[1 + 4 * 2], make_double2(c2, SIGN * c2));   // w^2
    v[1 + 4 * 3] = cmul(v[1 + 4 * 3], make_double2(s1, SIGN * c1));   // w^3
    v[2 + 4 * 1] = cmul(v[2 + 4 * 1], make_double2(c2, SIGN * c2));   // w^2
    v[2 + 4 * 2] = mul_si<SIGN>(v[2 + 4 * 2]);                         // w^4
    v[2 + 4 * 3] = cmul(v[2 + 4 * 3], make_double2(-c2, SIGN * c2));  // w^6
    v[3 + 4 * 1] = cmul(v[3 + 4 * 1], make_double2(s1, SIGN * c1));   // w^3
    v[3 + 4 * 2] = cmul(v[3 + 4 * 2], make_double2(-c2, SIGN * c2));  // w^6
    v[3 + 4 * 3] = cmul(v[3 + 4 * 3], make_double2(-c1, -SIGN * s1)); // w^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4s<SIGN>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // X[k1 + 4 k2] now sits at v[k2 + 4 k1] (out_pos gives the position of X[k])
}

// Register holding output k of dft_reg<R>: natural order except for R = 16.
template <int R>
__device__ __forceinline__ constexpr int out_pos(int k) {
    return R == 16 ? ((k >> 2) + 4 * (k & 3)) : k;
}

template <int R, int SIGN>
__device__ __forceinline__ void dft_reg(double2 *v) {
    if constexpr (R == 2) dft2<SIGN>(v);
    else if constexpr (R == 4) dft4<SIGN>(v);
    else if constexpr (R == 8) dft8<SIGN>(v);
    else dft16<SIGN>(v);
}

// Reads and writes of a column held in LDS.
struct LdsIn {
    const double2 *buf;
    __device__ __forceinline__ double2 operator()(int i) const { return buf[pad(i)]; }
};
struct LdsOut {
    double2 *buf;
    __device__ __forceinline__ void operator()(int i, double2 v) const { buf[pad(i)] = v; }
};

// log2 of a power of two, at compile time
__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// Pass structure of a length-P transform with main radix RM on NT = P/RM threads: one
// leading pass of radix REM (what is left of P after the radix-RM passes), then NMAIN
// passes of radix RM.  Every thread handles RM values in every pass.
template <int P, int RM>
struct Plan {
    static constexpr int NT = P / RM;
    static constexpr int NMAIN = ilog2(P) / ilog2(RM);
    static constexpr int REM = 1 << (ilog2(P) % ilog2(RM));
    static constexpr int NPASS = NMAIN + (REM > 1 ? 1 : 0);
};

// One Stockham pass of radix R over a column of P values held by NT threads: inputs come
// from `in` (LDS or a loader), outputs go to `out` (LDS or a storer).  tw[t] = e^{-2 pi i
// t/P} (the inverse transform, SIGN = +1, uses its conjugate).  If pm is not null each
// output X[i] is multiplied by pm[i] before it is stored.  The pass is in place: all
// reads, a barrier, all writes, a barrier.  The twiddles are requested before the reads
// so that their latency overlaps the reads and the barrier.
template <int P, int NT, int R, int SIGN, class In, class Out>
__device__ __forceinline__ void pass(int Ns, int tid0, const double2 *__restrict__ tw, const double2 *__restrict__ pm,
                                     In in, Out out) {
    constexpr int NB = P / R;       // butterflies
    constexpr int PER = NB / NT;    // butterflies per thread
    // The thread index is made opaque per pass so that the index arithmetic and bounds
    // masks of one pass are not hoisted and kept live across the others.
    int tid = tid0;
    __asm__ volatile("" : "+v"(tid));
    double2 v[PER][R], w[PER][R];
    if (Ns > 1) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int j = tid + q * NT;
            const int st = (j & (Ns - 1)) * (P / (Ns * R));
            // w^r for r < R from one table entry: w^2 = w w, w^4 = w^2 w^2, ... and the
            // other powers as products of those (at most six products deep: a few ulp)
            w[q][1] = tw[st];
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = in(j + r * NB);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
        const int k = j & (Ns - 1);
        if (Ns > 1) {
#pragma unroll
            for (int r = 2; r < R; ++r) {
                if ((r & (r - 1)) == 0) w[q][r] = cmul(w[q][r / 2], w[q][r / 2]);
                else w[q][r] = cmul(w[q][r & (r - 1)], w[q][r & -r]);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) v[q][r] = SIGN < 0 ? cmul(v[q][r], w[q][r]) : cmulc(v[q][r], w[q][r]);
        }
        dft_reg<R, SIGN>(v[q]);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double2 x = v[q][out_pos<R>(r)];
            if (pm) x = cmul(x, pm[base + r * Ns]);
            out(base + r * Ns, x);
        }
    }
    __syncthreads();
}

// Unnormalised DFT of a column, X_k = sum_n x_n e^{SIGN 2 pi i n k / P}, on P/RM threads:
// the first pass reads x through `in`, the last pass writes X (times pm, if given)
// through `out`; the passes in between work in LDS (buf).
template <int P, int RM, int SIGN, class In, class Out>
__device__ __forceinline__ void transform_io(double2 *buf, int tid, const double2 *__restrict__ tw,
                                             const double2 *__restrict__ pm, In in, Out out) {
    static_assert(P >= 32 && (P & (P - 1)) == 0, "power of two >= 32");
    using PL = Plan<P, RM>;
    constexpr int NT = PL::NT;
    LdsIn li{buf};
    LdsOut lo{buf};
    int Ns = 1;
    int p = 0;
    if constexpr (PL::REM > 1) {
        if constexpr (PL::NPASS == 1) pass<P, NT, PL::REM, SIGN>(Ns, tid, tw, pm, in, out);
        else pass<P, NT, PL::REM, SIGN>(Ns, tid, tw, nullptr, in, lo);
        Ns *= PL::REM;
        ++p;
    }
#pragma unroll
    for (int s = 0; s < PL::NMAIN; ++s) {
        const bool first = (p == 0), last = (p == PL::NPASS - 1);
        if (first && last) pass<P, NT, RM, SIGN>(Ns, tid, tw, pm, in, out);
        else if (first) pass<P, NT, RM, SIGN>(Ns, tid, tw, nullptr, in, lo);
        else if (last) pass<P, NT, RM, SIGN>(Ns, tid, tw, pm, li, out);
        else pass<P, NT, RM, SIGN>(Ns, tid, tw, nullptr, li, lo);
        Ns *= RM;
        ++p;
    }
}

// The last forward pass, the product with the spectrum and the first inverse pass, fused
// in registers.  With the partial pass of radix R = P / (P/R) taken last in the forward
// transform and first in the inverse one, butterfly j of the forward pass produces
// X[j + r P/R] (r < R) and butterfly j of the inverse pass consumes exactly those values,
// so they never go through LDS.  Outputs of the inverse pass go to out(j R + r).
template <int P, int NT, int R, class In, class Out>
__device__ __forceinline__ void mid_pass(int tid0, const double2 *__restrict__ tw, const double2 *__restrict__ hh,
                                         In in, Out out) {
    constexpr int NB = P / R;
    constexpr int PER = NB / NT;
    int tid = tid0;
    __asm__ volatile("" : "+v"(tid));
    double2 v[PER][R], w[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
        w[q][1] = tw[j];
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = in(j + r * NB);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
#pragma unroll
        for (int r = 2; r < R; ++r) {
            if ((r & (r - 1)) == 0) w[q][r] = cmul(w[q][r / 2], w[q][r / 2]);
            else w[q][r] = cmul(w[q][r & (r - 1)], w[q][r & -r]);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], w[q][r]);
        dft_reg<R, -1>(v[q]);
        double2 x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = cmul(v[q][out_pos<R>(r)], hh[j + r * NB]);
        dft_reg<R, +1>(x);
#pragma unroll
        for (int r = 0; r < R; ++r) out(j * R + r, x[out_pos<R>(r)]);
    }
    __syncthreads();
}

// Linear convolution through the FFT: the column is read by `in`, transformed, multiplied
// by the spectrum hh, transformed back and written by `out` (unnormalised: hh carries 1/P).
// Forward passes: radix RM (span 1, RM, ...), then the partial radix last; inverse passes:
// the partial radix first, then radix RM.  The pass at the junction is fused (mid_pass).
template <int P, int RM, class In, class Out>
__device__ __forceinline__ void convolve_io(double2 *buf, int tid, const double2 *__restrict__ tw,
                                            const double2 *__restrict__ hh, In in, Out out) {
    static_assert(P >= 32 && (P & (P - 1)) == 0, "power of two >= 32");
    using PL = Plan<P, RM>;
    constexpr int NT = PL::NT;
    constexpr int RJ = PL::REM > 1 ? PL::REM : RM;  // radix at the junction
    constexpr int NSIDE = PL::NPASS - 1;             // passes on each side of the junction
    LdsIn li{buf};
    LdsOut lo{buf};
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < NSIDE; ++s) {
        if (s == 0) pass<P, NT, RM, -1>(Ns, tid, tw, nullptr, in, lo);
        else pass<P, NT, RM, -1>(Ns, tid, tw, nullptr, li, lo);
        Ns *= RM;
    }
    if constexpr (NSIDE == 0) mid_pass<P, NT, RJ>(tid, tw, hh, in, out);
    else mid_pass<P, NT, RJ>(tid, tw, hh, li, lo);
    Ns = RJ;
#pragma unroll
    for (int s = 0; s < NSIDE; ++s) {
        if (s == NSIDE - 1) pass<P, NT, RM, +1>(Ns, tid, tw, nullptr, li, out);
        else pass<P, NT, RM, +1>(Ns, tid, tw, nullptr, li, lo);
        Ns *= RM;
    }
}

}  // namespace fft
}  // namespace s2dw
