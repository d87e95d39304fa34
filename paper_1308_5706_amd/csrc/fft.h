// Power-of-two FFTs held in LDS for gfx950, used as the engine of the odd-length (2L-1)
// transforms through Bluestein's chirp convolution.  Complex values are double2 (FP64
// path) or float2 (mixed-precision path); every function is generic over that type.
//
// LDS layout: element i of a column lives at pad(i) = i + i/16, so that strided stores of
// the first passes spread over all banks.  A column needs padded(P) slots.
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

template <class C> struct real_of;
template <> struct real_of<double2> { using type = double; };
template <> struct real_of<float2> { using type = float; };
template <class C> using real_t = typename real_of<C>::type;

template <class C>
__device__ __forceinline__ C mk(real_t<C> x, real_t<C> y) {
    C r;
    r.x = x;
    r.y = y;
    return r;
}

template <class C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <class C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <class C> __device__ __forceinline__ C cmul(C a, C b) {
    return mk<C>(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
template <class C> __device__ __forceinline__ C cmulc(C a, C b) {  // a * conj(b)
    return mk<C>(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}
template <class C> __device__ __forceinline__ C cconj(C a) { return mk<C>(a.x, -a.y); }
template <class C> __device__ __forceinline__ C cscale(C a, real_t<C> s) { return mk<C>(a.x * s, a.y * s); }

#ifndef S2DW_LDS_PAD_SHIFT
#define S2DW_LDS_PAD_SHIFT 4
#endif
__host__ __device__ constexpr int padded(int P) { return P + (P >> S2DW_LDS_PAD_SHIFT); }
__device__ __forceinline__ int pad(int i) { return i + (i >> S2DW_LDS_PAD_SHIFT); }

// a * (SIGN i)
template <int SIGN, class C>
__device__ __forceinline__ C mul_si(C a) {
    return SIGN > 0 ? mk<C>(-a.y, a.x) : mk<C>(a.y, -a.x);
}

// In-register DFTs: v'[k] = sum_r v[r] e^{SIGN 2 pi i r k / R}, natural order in and out.
template <int SIGN, class C>
__device__ __forceinline__ void dft2(C *v) {
    const C a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <int SIGN, class C>
__device__ __forceinline__ void dft4s(C &v0, C &v1, C &v2, C &v3) {
    const C a = cadd(v0, v2), b = csub(v0, v2), c = cadd(v1, v3), d = mul_si<SIGN>(csub(v1, v3));
    v0 = cadd(a, c);
    v2 = csub(a, c);
    v1 = cadd(b, d);
    v3 = csub(b, d);
}

template <int SIGN, class C>
__device__ __forceinline__ void dft4(C *v) {
    dft4s<SIGN>(v[0], v[1], v[2], v[3]);
}

// Second half of dft8: the twiddles w8^{n2 k1} and the DFT2 over n2.
template <int SIGN, class C>
__device__ __forceinline__ void dft8_tail(C *v) {
    using R = real_t<C>;
    constexpr R c = (R)0.70710678118654752440;
    v[3] = cmul(v[3], mk<C>(c, SIGN * c));
    v[5] = mul_si<SIGN>(v[5]);
    v[7] = cmul(v[7], mk<C>(-c, SIGN * c));
    C o[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        o[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
        o[k1 + 4] = csub(v[2 * k1], v[2 * k1 + 1]);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = o[i];
}

template <int SIGN, class C>
__device__ __forceinline__ void dft8(C *v) {
    // n = 2 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle w8^{n2 k1}, DFT2 over n2
    dft4s<SIGN>(v[0], v[2], v[4], v[6]);
    dft4s<SIGN>(v[1], v[3], v[5], v[7]);
    dft8_tail<SIGN>(v);
}

// dft8 of inputs whose upper half v[4..7] is zero (v[4..7] are not read): the DFT4s over n1
// then see two zero inputs each.
template <int SIGN, class C>
__device__ __forceinline__ void dft8_low(C *v) {
#pragma unroll
    for (int n2 = 0; n2 < 2; ++n2) {
        const C x0 = v[n2], x1 = v[2 + n2], d = mul_si<SIGN>(x1);
        v[n2] = cadd(x0, x1);
        v[4 + n2] = csub(x0, x1);
        v[2 + n2] = cadd(x0, d);
        v[6 + n2] = csub(x0, d);
    }
    dft8_tail<SIGN>(v);
}

template <int SIGN, class C>
__device__ __forceinline__ void dft16(C *v) {
    // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle w16^{n2 k1}, DFT4 over n2
    using R = real_t<C>;
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4s<SIGN>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // Y[n2][k1] sits at v[n2 + 4 k1]
    constexpr R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173, c2 = (R)0.70710678118654752440;
    v[1 + 4 * 1] = cmul(v[1 + 4 * 1], mk<C>(c1, SIGN * s1));   // w^1
    v[1 + 4 * 2] = cmul(v[1 + 4 * 2], mk<C>(c2, SIGN * c2));   // w^2
    v[1 + 4 * 3] = cmul(v[1 + 4 * 3], mk<C>(s1, SIGN * c1));   // w^3
    v[2 + 4 * 1] = cmul(v[2 + 4 * 1], mk<C>(c2, SIGN * c2));   // w^2
    v[2 + 4 * 2] = mul_si<SIGN>(v[2 + 4 * 2]);                  // w^4
    v[2 + 4 * 3] = cmul(v[2 + 4 * 3], mk<C>(-c2, SIGN * c2));  // w^6
    v[3 + 4 * 1] = cmul(v[3 + 4 * 1], mk<C>(s1, SIGN * c1));   // w^3
    v[3 + 4 * 2] = cmul(v[3 + 4 * 2], mk<C>(-c2, SIGN * c2));  // w^6
    v[3 + 4 * 3] = cmul(v[3 + 4 * 3], mk<C>(-c1, -SIGN * s1)); // w^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4s<SIGN>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // X[k1 + 4 k2] now sits at v[k2 + 4 k1] (out_pos gives the position of X[k])
}

// Register holding output k of dft_reg<R>: natural order except for R = 16.
template <int R>
__device__ __forceinline__ constexpr int out_pos(int k) {
    return R == 16 ? ((k >> 2) + 4 * (k & 3)) : k;
}

template <int R, int SIGN, class C>
__device__ __forceinline__ void dft_reg(C *v) {
    if constexpr (R == 2) dft2<SIGN>(v);
    else if constexpr (R == 4) dft4<SIGN>(v);
    else if constexpr (R == 8) dft8<SIGN>(v);
    else dft16<SIGN>(v);
}

// Reads and writes of a column held in LDS.
template <class C>
struct LdsIn {
    const C *buf;
    __device__ __forceinline__ C operator()(int i, int = 0) const { return buf[pad(i)]; }
};
template <class C>
struct LdsOut {
    C *buf;
    __device__ __forceinline__ void operator()(int i, C v, int = 0) const { buf[pad(i)] = v; }
};

// log2 of a power of two, at compile time
__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// Pass structure of a length-P transform with main radix RM on NT = P/RM threads: NMAIN
// passes of radix RM and, if P is not a power of RM, one partial pass of radix REM.
// Every thread handles RM values in every pass.
template <int P, int RM>
struct Plan {
    static constexpr int NT = P / RM;
    static constexpr int NMAIN = ilog2(P) / ilog2(RM);
    static constexpr int REM = 1 << (ilog2(P) % ilog2(RM));
    static constexpr int NPASS = NMAIN + (REM > 1 ? 1 : 0);
};

// w^r, r < R, from w^1: w^2 = w w, w^4 = w^2 w^2, ... and the other powers as products
// of those (at most six products deep: a few ulp).
template <int R, class C>
__device__ __forceinline__ void twiddle_powers(C *w) {
#pragma unroll
    for (int r = 2; r < R; ++r) {
        if ((r & (r - 1)) == 0) w[r] = cmul(w[r / 2], w[r / 2]);
        else w[r] = cmul(w[r & (r - 1)], w[r & -r]);
    }
}

// One Stockham pass of radix R and span Ns over a column of P values held by NT threads:
// inputs come from `in` (LDS or a loader), outputs go to `out` (LDS or a storer).  Both are
// called with the element index and the thread's slot q R + r (q < P/(R NT), r < R), a
// compile-time constant once the loops are unrolled, so that a loader or storer can keep
// per-thread values in registers; every pass gives a thread P/NT slots.
// tw[t] = e^{-2 pi i t/P} (the inverse transform, SIGN = +1, uses its conjugate).  The
// pass is in place: all reads, a barrier, all writes, a barrier.  The twiddle entry is
// requested before the reads so that its latency overlaps them.
template <int P, int NT, int R, int SIGN, class C, class In, class Out>
__device__ __forceinline__ void pass(int Ns, int tid0, const C *__restrict__ tw, In in, Out out) {
    constexpr int NB = P / R;       // butterflies
    constexpr int PER = NB / NT;    // butterflies per thread
    // The thread index is made opaque per pass so that the index arithmetic and bounds
    // masks of one pass are not hoisted and kept live across the others.
    int tid = tid0;
    __asm__ volatile("" : "+v"(tid));
    C v[PER][R], w[PER][R];
    if (Ns > 1) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int j = tid + q * NT;
            w[q][1] = tw[(j & (Ns - 1)) * (P / (Ns * R))];
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = in(j + r * NB, q * R + r);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
        const int k = j & (Ns - 1);
        if (Ns > 1) {
            twiddle_powers<R>(w[q]);
#pragma unroll
            for (int r = 1; r < R; ++r) v[q][r] = SIGN < 0 ? cmul(v[q][r], w[q][r]) : cmulc(v[q][r], w[q][r]);
        }
        dft_reg<R, SIGN>(v[q]);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) out(base + r * Ns, v[q][out_pos<R>(r)], q * R + r);
    }
    __syncthreads();
}

// The first forward pass (span 1, no twiddles) of radix 8 when the column has at most P/2
// nonzero inputs: inputs j + r P/8 with r >= 4 lie at or beyond P/2, so they are zero and
// are neither read nor added (dft8_low).  Same outputs as pass() up to the sign of zeros.
template <int P, int NT, int SIGN, class C, class In, class Out>
__device__ __forceinline__ void pass_first_low(int tid0, In in, Out out) {
    constexpr int R = 8, NB = P / R, PER = NB / NT;
    int tid = tid0;
    __asm__ volatile("" : "+v"(tid));
    C v[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
#pragma unroll
        for (int r = 0; r < R / 2; ++r) v[q][r] = in(j + r * NB, q * R + r);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
        dft8_low<SIGN>(v[q]);
#pragma unroll
        for (int r = 0; r < R; ++r) out(j * R + r, v[q][r], q * R + r);
    }
    __syncthreads();
}

// The last forward pass, the product with the spectrum and the first inverse pass, fused
// in registers.  With the partial pass of radix R = P / (P/R) taken last in the forward
// transform and first in the inverse one, butterfly j of the forward pass produces
// X[j + r P/R] (r < R) and butterfly j of the inverse pass consumes exactly those values,
// so they never go through LDS.  Outputs of the inverse pass go to out(j R + r).
template <int P, int NT, int R, class C, class In, class Out>
__device__ __forceinline__ void mid_pass(int tid0, const C *__restrict__ tw, const C *__restrict__ hh, In in,
                                         Out out) {
    constexpr int NB = P / R;
    constexpr int PER = NB / NT;
    int tid = tid0;
    __asm__ volatile("" : "+v"(tid));
    C v[PER][R], w[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
        w[q][1] = tw[j];
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = in(j + r * NB, q * R + r);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
        twiddle_powers<R>(w[q]);
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], w[q][r]);
        dft_reg<R, -1>(v[q]);
        C x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = cmul(v[q][out_pos<R>(r)], hh[j + r * NB]);
        dft_reg<R, +1>(x);
#pragma unroll
        for (int r = 0; r < R; ++r) out(j * R + r, x[out_pos<R>(r)], q * R + r);
    }
    __syncthreads();
}

// Linear convolution through the FFT: the column is read by `in`, transformed, multiplied
// by the spectrum hh, transformed back and written by `out` (unnormalised: hh carries 1/P).
// Forward passes: radix RM (span 1, RM, ...), then the partial radix last; inverse passes:
// the partial radix first, then radix RM.  The pass at the junction is fused (mid_pass).
// n_in: `in` returns zero at every index >= n_in (with RM = 8 and n_in <= P/2 the first
// pass skips the zero half).
template <int P, int RM, class C, class In, class Out>
__device__ __forceinline__ void convolve_io(C *buf, int tid, const C *__restrict__ tw, const C *__restrict__ hh,
                                            In in, Out out, int n_in = P) {
    static_assert(P >= 32 && (P & (P - 1)) == 0, "power of two >= 32");
    using PL = Plan<P, RM>;
    constexpr int NT = PL::NT;
    constexpr int RJ = PL::REM > 1 ? PL::REM : RM;  // radix at the junction
    constexpr int NSIDE = PL::NPASS - 1;             // passes on each side of the junction
    LdsIn<C> li{buf};
    LdsOut<C> lo{buf};
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < NSIDE; ++s) {
        if (s == 0) {
            if constexpr (RM == 8) {
                if (n_in <= P / 2) pass_first_low<P, NT, -1, C>(tid, in, lo);
                else pass<P, NT, RM, -1>(Ns, tid, tw, in, lo);
            } else {
                pass<P, NT, RM, -1>(Ns, tid, tw, in, lo);
            }
        } else {
            pass<P, NT, RM, -1>(Ns, tid, tw, li, lo);
        }
        Ns *= RM;
    }
    if constexpr (NSIDE == 0) mid_pass<P, NT, RJ>(tid, tw, hh, in, out);
    else mid_pass<P, NT, RJ>(tid, tw, hh, li, lo);
    Ns = RJ;
#pragma unroll
    for (int s = 0; s < NSIDE; ++s) {
        if (s == NSIDE - 1) pass<P, NT, RM, +1>(Ns, tid, tw, li, out);
        else pass<P, NT, RM, +1>(Ns, tid, tw, li, lo);
        Ns *= RM;
    }
}

}  // namespace fft
}  // namespace s2dw
