// Separation-of-variables stages of the wavelet transform (Sec. 3.2-3.3) on gfx950,
// on the equiangular grid
//   alpha_a = 2 pi a/T (a < T), beta_b = pi (2b+1)/T (b < L), gamma_g = 2 pi g/(2N-1),
// with T = 2L - 1.  Every length-T sum is a Bluestein chirp convolution: with
// 2 x y = x^2 + y^2 - (y - x)^2,
//   sum_x a_x e^{2 pi i x y/T} = e^{i pi y^2/T} sum_x (a_x e^{i pi x^2/T}) e^{-i pi (y-x)^2/T},
// a linear convolution evaluated by a power-of-two FFT of size P held in LDS (fft.h);
// the spectrum of each chirp (divided by P) and the chirps themselves,
// csq[i] = e^{i pi i^2/T} (i < T) and cpp[p + L - 1] = e^{i pi p(p+1)/T} (|p| < L), are
// precomputed per plan with the phases reduced exactly modulo 2T.
//
// A convolution z(k) = sum_n a(n) h(k - n), n in [n0, n0+Na), k in [k0, k0+Nk), is
// computed as c = IFFT(FFT(a') * FFT(h')) with a'(i) = a(n0+i) and
// h'(i) = h(k0 - n0 - Na + 1 + i) (i < Na + Nk - 1, zero elsewhere), P >= Na + Nk - 1;
// then z(k0 + q) = c[q + Na - 1].  Column element i is held at LDS slot fft::pad(i).
//
// Every stage kernel is a template over the complex type C: double2 for the FP64 path,
// float2 for the mixed-precision path (FP32 transforms, tables and accumulation; the
// analysis input U is FP64 in both).
#pragma once

#include "fft.h"
#include "kernels.h"
#include "pfa.h"

#ifndef S2DW_FFT_RADIX
#define S2DW_FFT_RADIX 8
#endif

namespace s2dw {

using fft::cadd;
using fft::cconj;
using fft::cmul;
using fft::cmulc;
using fft::cscale;
using fft::csub;
using fft::pad;

namespace {

// Main FFT radix: a column of P values is handled by P / kRM threads.
constexpr int kRM = S2DW_FFT_RADIX;
// Waves per SIMD the FFT kernels must fit (two P = 4096 columns share a CU's LDS).
constexpr int kMinWaves = kRM >= 16 ? 2 : 4;

using fft::mk;
using fft::real_t;

template <class C>
__device__ __forceinline__ C rot_i(C z, int e) {
    e &= 3;
    if (e == 0) return z;
    if (e == 1) return mk<C>(-z.y, z.x);
    if (e == 2) return mk<C>(-z.x, -z.y);
    return mk<C>(z.y, -z.x);
}

template <class C>
__device__ __forceinline__ C zero2() { return mk<C>(0, 0); }

template <class C>
__device__ __forceinline__ C to_c(double2 v) { return mk<C>((real_t<C>)v.x, (real_t<C>)v.y); }

}  // namespace

// ------------------------------------------------------------------- analysis: beta (Eq. 29)
// Column (n, m) of scale j: Ub(b) = sum_{|m'|<Lj} U_{m m' n} e^{i m' beta_b}, b < nb, with
// U_{m,-m',n} = (-1)^{m+n} U_{m m' n} (only m' >= 0 is stored) and beta_b = pi (2b+1)/Tb:
// the equiangular grid has Tb = 2L - 1, nb = L, the Driscoll-Healy grid (Eq. 17) Tb = 4L,
// nb = 2L.  Since m' beta_b = 2 pi m' b/Tb + pi m'/Tb, the chirp input is
// U e^{i pi m'(m'+1)/Tb}; the chirp tables of the launch are those of Tb.
template <class C, int P>
__device__ __forceinline__ void beta_fwd_fft_body(const StageArgs &a, int bx, int by, int tid, C *buf) {
    const int Lj = a.Lj, L = a.L, nb = a.nb;
    const int col = bx;  // ni * Lj + m
    const int ni = col / Lj, m = col - ni * Lj;
    const int n = 2 * ni - (a.N - 1);
    const bool odd = ((m + n) & 1) != 0;
    const double2 *__restrict__ Uc = (const double2 *)a.in + by * a.s_in + (size_t)col * Lj;
    const C *__restrict__ cpp = (const C *)a.cpp + (L - 1);
    const C *__restrict__ csq = (const C *)a.csq;
    const int Na = 2 * Lj - 1;
    C *__restrict__ out = (C *)a.out + by * a.s_out + (size_t)col * nb;
    auto in = [&](int i, int = 0) {
        if (i >= Na) return zero2<C>();
        const int mp = i - (Lj - 1);
        C v = to_c<C>(Uc[mp < 0 ? -mp : mp]);
        if (mp < 0 && odd) v = mk<C>(-v.x, -v.y);
        return cmul(v, cpp[mp]);
    };
    auto st = [&](int i, C v, int = 0) {
        const int b = i - (Na - 1);
        if (b >= 0 && b < nb) out[b] = cmul(v, csq[b]);
    };
    fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, (const C *)a.hh, in, st, Na);
}

template <class C, int P>
__global__ void __launch_bounds__(P / kRM, kMinWaves) beta_fwd_fft_kernel(const StageArgs a) {
    __shared__ C buf[fft::padded(P)];
    beta_fwd_fft_body<C, P>(a, blockIdx.x, blockIdx.y, threadIdx.x, buf);
}

// Two columns (n, m0) and (n, m0 + 1) of the equiangular grid in one transform.  With
// s = (-1)^{m+n}, F(beta) = sum_{m'} U_{m m' n} e^{i m' beta} obeys F(2 pi - beta) = s F(beta), and
// the two columns have opposite s.  The transform of their sum, evaluated at all T ring
// positions beta_t = pi (2t+1)/T (t < T; beta_{T-1-b} = 2 pi - beta_b), is F_z = F_a + F_b, so
//   F_a(beta_b) = (F_z(beta_b) + s_a F_z(beta_{T-1-b}))/2,  F_b(beta_b) = (F_z(beta_b) - s_a F_z(beta_{T-1-b}))/2.
// Taken where the convolution of 2Lj - 1 inputs and T outputs needs no larger transform than
// the single column's (the scales with Lj = L).  Workgroup col = ni ceil(Lj/2) + c takes
// columns m0 = 2c and m0 + 1.
template <class C, int P>
__device__ __forceinline__ void beta_fwd_pair_body(const StageArgs &a, int bx, int by, int tid, C *buf) {
    const int Lj = a.Lj, L = a.L, T = 2 * L - 1;
    const int Mp = (Lj + 1) >> 1;
    const int ni = bx / Mp, m0 = 2 * (bx - ni * Mp);
    const bool two = m0 + 1 < Lj;
    const int n = 2 * ni - (a.N - 1);
    const bool odd0 = ((m0 + n) & 1) != 0;  // s of column m0 is -1
    const double2 *__restrict__ Ua = (const double2 *)a.in + by * a.s_in + ((size_t)ni * Lj + m0) * Lj;
    const double2 *__restrict__ Ub = Ua + Lj;
    const C *__restrict__ cpp = (const C *)a.cpp + (L - 1);
    const C *__restrict__ csq = (const C *)a.csq;
    const int Na = 2 * Lj - 1;
    auto in = [&](int i, int = 0) {
        if (i >= Na) return zero2<C>();
        const int mp = i - (Lj - 1), am = mp < 0 ? -mp : mp;
        C va = to_c<C>(Ua[am]);
        C vb = two ? to_c<C>(Ub[am]) : zero2<C>();
        if (mp < 0) {
            if (odd0) va = mk<C>(-va.x, -va.y);
            else vb = mk<C>(-vb.x, -vb.y);
        }
        return cmul(cadd(va, vb), cpp[mp]);
    };
    auto st = [&](int i, C v, int = 0) {
        const int t = i - (Na - 1);
        if (t >= 0 && t < T) buf[pad(t)] = cmul(v, csq[t]);
    };
    fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, (const C *)a.hh, in, st, Na);
    C *__restrict__ oa = (C *)a.out + by * a.s_out + ((size_t)ni * Lj + m0) * L;
    C *__restrict__ ob = oa + L;
    const real_t<C> h = (real_t<C>)0.5;
    for (int b = tid; b < L; b += P / kRM) {
        const C x = buf[pad(b)], y = buf[pad(T - 1 - b)];
        const C p = cscale(cadd(x, y), h), q = cscale(csub(x, y), h);
        oa[b] = odd0 ? q : p;
        if (two) ob[b] = odd0 ? p : q;
    }
}

template <class C, int P>
__global__ void __launch_bounds__(P / kRM, kMinWaves) beta_fwd_pair_kernel(const StageArgs a) {
    __shared__ C buf[fft::padded(P)];
    beta_fwd_pair_body<C, P>(a, blockIdx.x, blockIdx.y, threadIdx.x, buf);
}

// Waves per SIMD the prime-factor kernels are built for: two eight-wave workgroups per CU
// (their LDS allows two) for the eight-wave form, else as the registers fall.
template <class LN>
constexpr int pfa_min_waves() { return LN::NTH == 512 ? 4 : 1; }

// The same two-column transform as a direct prime-factor transform of length T (pfa.h):
//   F_z(beta_t) = sum_{m'} [z(m') e^{i pi m'/T}] e^{2 pi i m' t/T},  input index n = m' mod T,
// for every scale of the equiangular grid when T is one of its lengths; LN::NC column pairs per
// workgroup.  e^{i pi m'/T} = eph[m'/2 mod T] for even m', -eph[(m' + T)/2 mod T] for odd m'.
// Workgroup g of a scale of band-limit Lj; U and Ub: the scale's arrays of the map.
template <class C, class LN>
__device__ __forceinline__ void beta_fwd_pfa_body(const StageArgs &a, int Lj, const double2 *__restrict__ U,
                                                  C *__restrict__ Ub, int g, int tid, C *buf) {
    const int L = a.L, T = LN::T, N = a.N;
    const int Mp = (Lj + 1) >> 1, ncols = N * Mp;
    const int u0 = g * LN::NC, ncol = min(LN::NC, ncols - u0);
    const C *__restrict__ eph = (const C *)a.eph;
    auto in = [&](int c, int n) {
        const int u = u0 + c, ni = u / Mp, m0 = 2 * (u - (u / Mp) * Mp);
        const int mp = n < Lj ? n : (n > T - Lj ? n - T : T);
        if (mp == T) return mk<C>(0, 0);
        const bool two = m0 + 1 < Lj;
        const bool odd0 = ((m0 + 2 * ni - (N - 1)) & 1) != 0;
        const int am = mp < 0 ? -mp : mp;
        const double2 *Ua = U + ((size_t)ni * Lj + m0) * Lj;
        C va = to_c<C>(Ua[am]);
        C vb = two ? to_c<C>(Ua[Lj + am]) : mk<C>(0, 0);
        if (mp < 0) {
            if (odd0) va = mk<C>(-va.x, -va.y);
            else vb = mk<C>(-vb.x, -vb.y);
        }
        const bool oddm = (mp & 1) != 0;
        int r = oddm ? (mp + T) / 2 : mp / 2;
        r %= T;
        if (r < 0) r += T;
        C e = eph[r];
        if (oddm) e = mk<C>(-e.x, -e.y);
        return cmul(cadd(va, vb), e);
    };
    pfa::dft_lds<LN, +1>(buf, (const C *)a.pcs, tid, ncol, in);
    const real_t<C> h = (real_t<C>)0.5;
    for (int e = tid; e < ncol * L; e += LN::NTH) {
        const int c = e / L, b = e - (e / L) * L;
        const int u = u0 + c, ni = u / Mp, m0 = 2 * (u - (u / Mp) * Mp);
        const bool two = m0 + 1 < Lj;
        const bool odd0 = ((m0 + 2 * ni - (N - 1)) & 1) != 0;
        const C x = buf[c * LN::CS + LN::pos_out(b)], y = buf[c * LN::CS + LN::pos_out(T - 1 - b)];
        const C p = cscale(cadd(x, y), h), q = cscale(csub(x, y), h);
        C *__restrict__ oa = Ub + ((size_t)ni * Lj + m0) * L;
        oa[b] = odd0 ? q : p;
        if (two) oa[L + b] = odd0 ? p : q;
    }
}

template <class C, class LN>
__global__ void __launch_bounds__(LN::NTH, pfa_min_waves<LN>()) beta_fwd_pfa_kernel(const StageArgs a) {
    __shared__ C buf[LN::lds];
    const int nwg = (a.N * ((a.Lj + 1) >> 1) + LN::NC - 1) / LN::NC;
    if ((int)blockIdx.x >= nwg) return;
    beta_fwd_pfa_body<C, LN>(a, a.Lj, (const double2 *)a.in + blockIdx.y * a.s_in,
                             (C *)a.out + blockIdx.y * a.s_out, blockIdx.x, threadIdx.x, buf);
}

// The coarse scales of a map in one launch (each alone fills only a few workgroups and takes a
// launch's latency): workgroups [tab[s].first, tab[s + 1].first) take scale s, whose U starts
// tab[s].in_off elements after a.in and whose Ub goes tab[s].out_off elements after a.out.
template <class C, class LN>
__global__ void __launch_bounds__(LN::NTH, pfa_min_waves<LN>()) beta_fwd_pfa_multi_kernel(const StageArgs a,
                                                                                          const BetaAdjScale *tab,
                                                                                          int ns) {
    __shared__ C buf[LN::lds];
    const int bx = blockIdx.x;
    int s = 0;
    for (int i = 1; i < ns; ++i)
        if (bx >= tab[i].first) s = i;
    const BetaAdjScale e = tab[s];
    beta_fwd_pfa_body<C, LN>(a, e.Lj, (const double2 *)a.in + blockIdx.y * a.s_in + e.in_off,
                             (C *)a.out + blockIdx.y * a.s_out + e.out_off, bx - e.first, threadIdx.x, buf);
}

// ------------------------------------------------------------------ alpha and gamma stages
// Only the orders n with N + n odd are present, and W is real, so the coefficients obey
// C_{-n}(-m) = conj(C_n(m)).  The alpha sums therefore run over the rows n >= 0 only
// (Nh = ceil(N/2) complex rows per beta ring instead of 2N - 1 real ones), and the gamma
// sums are separate streaming passes over the sample grid:
//   analysis:  Y_n(b, a) = sum_{|m|<Lj} C_n(b, m) e^{i m alpha_a}   (Eq. 30, n >= 0)
//              W(g, b, a) = Re Y_0 + 2 Re sum_{n>0} Y_n e^{i n gamma_g}   (Eq. 28)
//   synthesis: X_n(b, a) = sum_g W(g, b, a) e^{-i n gamma_g}   (Eq. 39, n >= 0)
//              Gs_n(b, m) = wa wg sum_a X_n(b, a) e^{-i m alpha_a},  Gs_{-n}(b, m) = conj Gs_n(b, -m)
// with C_n(b, m) = Ub[n][m][b] for m >= 0 and conj(Ub[-n][-m][b]) for m < 0.
//
// Column order: blockIdx.x -> t = (b, n') is remapped so that the workgroups that run on
// one XCD (dispatched round-robin over the 8 XCDs) take consecutive t; the [n][m][b]
// arrays, read and written with stride nb along m, then share L2 lines across neighbouring
// rings b.  nb = number of beta rings (L, or 2L on the Driscoll-Healy grid); alpha has
// T = 2L - 1 samples on both grids.
__device__ __forceinline__ int xcd_column(int x, int ncols) {
    const int per = (ncols + 7) >> 3;
    return (x & 7) * per + (x >> 3);
}

template <class C, int P>
__device__ __forceinline__ void alpha_fwd_fft_body(const StageArgs &a, int bx, int by, int tid, C *buf) {
    const int Lj = a.Lj, L = a.L, T = 2 * L - 1, N = a.N, Nh = a.Nh, nb = a.nb;
    const int t = bx;
    const int b = t / Nh, np = t - (t / Nh) * Nh;
    const int ni = (N / 2) + np, nj = N - 1 - ni;  // rows of n >= 0 and of -n
    const bool zero_n = ni == nj;
    const C *__restrict__ Up = (const C *)a.in + by * a.s_in + (size_t)ni * Lj * nb + b;
    const C *__restrict__ Um = (const C *)a.in + by * a.s_in + (size_t)nj * Lj * nb + b;
    const C *__restrict__ csq = (const C *)a.csq;
    const int Na = 2 * Lj - 1;
    // The alpha loaders are branch-free: an index past the end is clamped, so that the load
    // stays in bounds and is issued with the thread's others (all in flight together), and
    // its value is then replaced by zero.
    auto in = [&](int i, int = 0) {
        const bool ok = i < Na;
        const int m = (ok ? i : Na - 1) - (Lj - 1), am = m < 0 ? -m : m;
        C c = (m >= 0 ? Up : Um)[(size_t)am * nb];
        const C w = csq[am];
        if (m < 0) c = cconj(c);
        if (m == 0 && zero_n) c.y = 0.0;
        c = cmul(c, w);
        return ok ? c : zero2<C>();
    };
    C *__restrict__ Y = (C *)a.out + by * a.s_out + ((size_t)np * nb + b) * T;
    auto st = [&](int i, C v, int = 0) {
        const int x = i - (Na - 1);
        if (x >= 0 && x < T) Y[x] = cmul(v, csq[x]);
    };
    fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, (const C *)a.hh, in, st, Na);
}

template <class C, int P>
__global__ void __launch_bounds__(P / kRM, kMinWaves) alpha_fwd_fft_kernel(const StageArgs a) {
    __shared__ C buf[fft::padded(P)];
    const int t = xcd_column(blockIdx.x, a.Nh * a.nb);
    if (t >= a.Nh * a.nb) return;
    alpha_fwd_fft_body<C, P>(a, t, blockIdx.y, threadIdx.x, buf);
}

template <class C, int P>
__device__ __forceinline__ void alpha_adj_fft_body(const StageArgs &a, int bx, int by, int tid, C *buf) {
    const int Lj = a.Lj, L = a.L, T = 2 * L - 1, N = a.N, Nh = a.Nh, nb = a.nb;
    const int t = bx;
    const int b = t / Nh, np = t - (t / Nh) * Nh;
    const int ni = (N / 2) + np, nj = N - 1 - ni;
    const bool zero_n = ni == nj;
    const C *__restrict__ X = (const C *)a.in + by * a.s_in + ((size_t)np * nb + b) * T;
    const C *__restrict__ csq = (const C *)a.csq;
    auto in = [&](int i, int = 0) {  // branch-free (see alpha_fwd_fft_kernel)
        const bool ok = i < T;
        const int ic = ok ? i : T - 1;
        const C v = cmulc(X[ic], csq[ic]);
        return ok ? v : zero2<C>();
    };
    // Zh(m), q = m + Lj - 1 < 2Lj - 1, comes out at q + T - 1
    const int Nk = 2 * Lj - 1;
    const real_t<C> s = (real_t<C>)a.scale;
    C *__restrict__ Gp = (C *)a.out + by * a.s_out + (size_t)ni * Lj * nb + b;
    C *__restrict__ Gm = (C *)a.out + by * a.s_out + (size_t)nj * Lj * nb + b;
    auto st = [&](int i, C v, int = 0) {
        const int q = i - (T - 1);
        if (q >= 0 && q < Nk) {
            const int m = q - (Lj - 1);
            const C z = cscale(cmulc(v, csq[m < 0 ? -m : m]), s);
            if (m >= 0) Gp[(size_t)m * nb] = z;
            if (m <= 0 && !zero_n) Gm[(size_t)(-m) * nb] = cconj(z);
        }
    };
    fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, (const C *)a.hh, in, st, T);
}

template <class C, int P>
__global__ void __launch_bounds__(P / kRM, kMinWaves) alpha_adj_fft_kernel(const StageArgs a) {
    __shared__ C buf[fft::padded(P)];
    const int t = xcd_column(blockIdx.x, a.Nh * a.nb);
    if (t >= a.Nh * a.nb) return;
    alpha_adj_fft_body<C, P>(a, t, blockIdx.y, threadIdx.x, buf);
}

// The same alpha sums as direct prime-factor transforms of length T (pfa.h) where T is one of
// its lengths: LN::NC consecutive rings b of one order row per workgroup, no chirps.
//   analysis:  Y(a) = sum_{|m|<Lj} C(m) e^{2 pi i m a/T}: input index n = m mod T (sign +1)
//   synthesis: Gs(m) = wa wg sum_a X(a) e^{-2 pi i m a/T}: output index k = m mod T (sign -1)
template <class C, class LN>
__global__ void __launch_bounds__(LN::NTH, pfa_min_waves<LN>()) alpha_fwd_pfa_kernel(const StageArgs a) {
    __shared__ C buf[LN::lds];
    const int tid = threadIdx.x;
    const int Lj = a.Lj, T = LN::T, N = a.N, Nh = a.Nh, nb = a.nb;
    const int ncols = Nh * nb, nwg = (ncols + LN::NC - 1) / LN::NC;
    const int g = xcd_column(blockIdx.x, nwg);
    if (g >= nwg) return;
    const int t0 = g * LN::NC, ncol = min(LN::NC, ncols - t0);
    const C *__restrict__ U = (const C *)a.in + blockIdx.y * a.s_in;
    C *__restrict__ Y = (C *)a.out + blockIdx.y * a.s_out;
    auto in = [&](int c, int n) {
        const int t = t0 + c, np = t / nb, b = t - (t / nb) * nb;
        const int ni = (N / 2) + np, nj = N - 1 - ni;
        const int m = n < Lj ? n : (n > T - Lj ? n - T : T);
        if (m == T) return mk<C>(0, 0);
        const int am = m < 0 ? -m : m;
        C v = U[((size_t)(m >= 0 ? ni : nj) * Lj + am) * nb + b];
        if (m < 0) v = cconj(v);
        if (m == 0 && ni == nj) v.y = 0;
        return v;
    };
    auto out = [&](int c, int k, C v) {
        const int t = t0 + c, np = t / nb, b = t - (t / nb) * nb;
        Y[((size_t)np * nb + b) * T + k] = v;
    };
    pfa::dft<LN, +1>(buf, (const C *)a.pcs, tid, ncol, in, out);
}

template <class C, class LN>
__global__ void __launch_bounds__(LN::NTH, pfa_min_waves<LN>()) alpha_adj_pfa_kernel(const StageArgs a) {
    __shared__ C buf[LN::lds];
    const int tid = threadIdx.x;
    const int Lj = a.Lj, T = LN::T, N = a.N, Nh = a.Nh, nb = a.nb;
    const int ncols = Nh * nb, nwg = (ncols + LN::NC - 1) / LN::NC;
    const int g = xcd_column(blockIdx.x, nwg);
    if (g >= nwg) return;
    const int t0 = g * LN::NC, ncol = min(LN::NC, ncols - t0);
    const C *__restrict__ X = (const C *)a.in + blockIdx.y * a.s_in;
    C *__restrict__ G = (C *)a.out + blockIdx.y * a.s_out;
    const real_t<C> sc = (real_t<C>)a.scale;
    auto in = [&](int c, int n) {
        const int t = t0 + c, np = t / nb, b = t - (t / nb) * nb;
        return X[((size_t)np * nb + b) * T + n];
    };
    auto out = [&](int c, int k, C v) {
        const int m = k < Lj ? k : (k > T - Lj ? k - T : T);
        if (m == T) return;
        const int t = t0 + c, np = t / nb, b = t - (t / nb) * nb;
        const int ni = (N / 2) + np, nj = N - 1 - ni;
        const C z = cscale(v, sc);
        if (m >= 0) G[((size_t)ni * Lj + m) * nb + b] = z;
        if (m <= 0 && ni != nj) G[((size_t)nj * Lj - m) * nb + b] = cconj(z);
    };
    pfa::dft<LN, -1>(buf, (const C *)a.pcs, tid, ncol, in, out);
}

// The alpha and gamma passes of one scale fused, one beta ring per workgroup, with the
// prime-factor transforms (real signals).  Each thread owns the samples a = tid + k NTH
// (k < KS).  Analysis: the NH orders n >= 0 of the ring pass through the transform LN::NC at
// a time; the owned outputs of the earlier passes wait in registers, and the gamma sum
//   W(g, b, a) = sum_{n'} Re(Y_{n'}(a) tg[g][n'])
// of the last pass writes W.  Synthesis: one sweep over the ring's W forms the gamma sums
//   X_{n'}(a) = sum_g W(g, b, a) tg[g][n'],
// of every order at the owned samples, and the orders pass through the transform NC at a
// time (the later ones waiting in registers).  The Y and X arrays of the two-pass form never
// go to HBM.  Register budget: the orders waiting in registers hold at most 16 complex values
// per thread (pfa_fused).
template <class LN>
constexpr int pfa_ks() { return (LN::T + LN::NTH - 1) / LN::NTH; }

template <class C, class LN, int NH>
__global__ void __launch_bounds__(LN::NTH, pfa_min_waves<LN>()) alpha_gamma_fwd_pfa_kernel(const StageArgs a) {
    using R = real_t<C>;
    constexpr int T = LN::T, NC = LN::NC, NTH = LN::NTH, KS = pfa_ks<LN>();
    constexpr int NP = (NH + NC - 1) / NC, NHOLD = (NP - 1) * NC, NLAST = NH - NHOLD;
    __shared__ C buf[LN::lds];
    const int tid = threadIdx.x;
    const int Lj = a.Lj, N = a.N, nb = a.nb, G = a.G;
    const int b = xcd_column(blockIdx.x, nb);
    if (b >= nb) return;
    const C *__restrict__ U = (const C *)a.in + blockIdx.y * a.s_in;
    const C *__restrict__ tab = (const C *)a.pcs;
    C held[NHOLD > 0 ? NHOLD : 1][KS];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int nrow = p < NP - 1 ? NC : NLAST;
        auto in = [&](int c, int n) {
            const int np = p * NC + c;
            const int ni = (N / 2) + np, nj = N - 1 - ni;
            const int m = n < Lj ? n : (n > T - Lj ? n - T : T);
            if (m == T) return mk<C>(0, 0);
            const int am = m < 0 ? -m : m;
            C v = U[((size_t)(m >= 0 ? ni : nj) * Lj + am) * nb + b];
            if (m < 0) v = cconj(v);
            if (m == 0 && ni == nj) v.y = 0;
            return v;
        };
        pfa::dft_lds<LN, +1>(buf, tab, tid, nrow, in);
        if (p < NP - 1) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const int x = tid + k * NTH;
                    if (x < T) held[p * NC + c][k] = buf[c * LN::CS + LN::pos_out(x)];
                }
            __syncthreads();
        }
    }
    R *__restrict__ W = (R *)a.wout + blockIdx.y * a.s_w + (size_t)b * T;
    const C *__restrict__ tg = (const C *)a.tg;
    const size_t plane = (size_t)nb * T;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int x = tid + k * NTH;
        if (x >= T) continue;
        C y[NH];
#pragma unroll
        for (int r = 0; r < NHOLD; ++r) y[r] = held[r][k];
#pragma unroll
        for (int c = 0; c < NLAST; ++c) y[NHOLD + c] = buf[c * LN::CS + LN::pos_out(x)];
        for (int g = 0; g < G; ++g) {
            R acc = 0;
#pragma unroll
            for (int r = 0; r < NH; ++r) {
                const C w = tg[g * NH + r];
                acc = fma(y[r].x, w.x, fma(-y[r].y, w.y, acc));
            }
            __builtin_nontemporal_store(acc, W + g * plane + x);  // written once, read by the synthesis
        }
    }
}

template <class C, class LN, int NH>
__global__ void __launch_bounds__(LN::NTH, pfa_min_waves<LN>()) gamma_alpha_adj_pfa_kernel(const StageArgs a) {
    using R = real_t<C>;
    constexpr int T = LN::T, NC = LN::NC, NTH = LN::NTH, KS = pfa_ks<LN>();
    constexpr int NP = (NH + NC - 1) / NC;
    __shared__ C buf[LN::lds];
    const int tid = threadIdx.x;
    const int Lj = a.Lj, N = a.N, nb = a.nb, G = a.G;
    const int b = xcd_column(blockIdx.x, nb);
    if (b >= nb) return;
    const R *__restrict__ W = (const R *)a.win + blockIdx.y * a.s_w + (size_t)b * T;
    const C *__restrict__ tg = (const C *)a.tg;
    const size_t plane = (size_t)nb * T;
    // the gamma sums of rows r0 .. r0 + NR - 1 into x[0 .. NR - 1]: plane by plane, the
    // thread's KS samples of a plane loaded together
    const int klast = (T - 1 - tid) / NTH;  // the thread's last sample: tid + klast NTH < T
    auto gamma_sums = [&](auto nr_c, int r0, C (*x)[KS]) {
        constexpr int NR = decltype(nr_c)::value;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int k = 0; k < KS; ++k) x[r][k] = mk<C>(0, 0);
        for (int g = 0; g < G; ++g) {
            R w[KS];
#pragma unroll
            for (int k = 0; k < KS; ++k)
                w[k] = __builtin_nontemporal_load(W + g * plane + tid + min(k, klast) * NTH);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const C t = r0 + r < NH ? tg[g * NH + r0 + r] : mk<C>(0, 0);
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    x[r][k].x = fma(w[k], t.x, x[r][k].x);
                    x[r][k].y = fma(w[k], t.y, x[r][k].y);
                }
            }
        }
    };
    // HOLD: every order's sums from one sweep over W, the later passes' waiting in registers;
    // else (FP64 at T = 2047 with more than two orders, which would take more than 128
    // registers for them next to the length-89 stage's) each pass sweeps W for its own rows
    constexpr bool HOLD = !(T == 2047 && sizeof(C) == 16 && NH > NC);
    C x[HOLD ? NH : NC][KS];
    C *__restrict__ Gout = (C *)a.out + blockIdx.y * a.s_out;
    const C *__restrict__ tab = (const C *)a.pcs;
    const real_t<C> sc = (real_t<C>)a.scale;
    // pass p: rows p NC .. of the transform, their sums at x[x0 ..]
    auto pass = [&](int p, int x0) {
        const int nrow = min(NC, NH - p * NC);
        if (p > 0) __syncthreads();  // the previous pass's outputs are read
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < nrow) {
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const int s = tid + k * NTH;
                    if (s < T) buf[c * LN::CS + LN::pos_in(s)] = x[x0 + c][k];
                }
            }
        __syncthreads();
        pfa::dft_stages<LN, -1>(buf, tab, tid, nrow);
        for (int e = tid; e < nrow * T; e += NTH) {
            const int c = e / T, k = e - (e / T) * T;
            const int m = k < Lj ? k : (k > T - Lj ? k - T : T);
            if (m == T) continue;
            const int np = p * NC + c, ni = (N / 2) + np, nj = N - 1 - ni;
            const C z = cscale(buf[c * LN::CS + LN::pos_out(k)], sc);
            if (m >= 0) Gout[((size_t)ni * Lj + m) * nb + b] = z;
            if (m <= 0 && ni != nj) Gout[((size_t)nj * Lj - m) * nb + b] = cconj(z);
        }
    };
    if constexpr (HOLD) {
        gamma_sums(std::integral_constant<int, NH>(), 0, x);
#pragma unroll
        for (int p = 0; p < NP; ++p) pass(p, p * NC);
    } else {
#pragma unroll 1
        for (int p = 0; p < NP; ++p) {
            gamma_sums(std::integral_constant<int, NC>(), p * NC, x);
            pass(p, 0);
        }
    }
}

// Blocked alpha sums for scales with few coefficients (2Lj - 1 well below T): the T samples
// are taken in nblk blocks of B consecutive ones, each through a short chirp convolution of
// size P >= B + 2Lj - 2 instead of one of size >= T + 2Lj - 2.  With a = a0 + a' (a0 = k B),
//   sum_m C(m) e^{2 pi i m a/T} = sum_m [C(m) e^{2 pi i m a0/T}] e^{2 pi i m a'/T},
// so every block uses the same chirp spectrum and only the modulation e^{2 pi i m a0/T} =
// eph[(m a0) mod T] changes.  The workgroup loops over the blocks; in the synthesis the
// block results are summed in registers (the storer's slots are the same in every block).
template <class C, int P>
__device__ __forceinline__ void alpha_fwd_blk_body(const StageArgs &a, int bx, int by, int tid, C *buf) {
    static_assert(fft::Plan<P, kRM>::NPASS >= 2, "the first pass reads element tid + r NT into slot r");
    constexpr int NT = P / kRM;
    const int Lj = a.Lj, L = a.L, T = 2 * L - 1, N = a.N, Nh = a.Nh, nb = a.nb, B = a.B;
    const int t = bx;
    const int b = t / Nh, np = t - (t / Nh) * Nh;
    const int ni = (N / 2) + np, nj = N - 1 - ni;
    const bool zero_n = ni == nj;
    const C *__restrict__ Up = (const C *)a.in + by * a.s_in + (size_t)ni * Lj * nb + b;
    const C *__restrict__ Um = (const C *)a.in + by * a.s_in + (size_t)nj * Lj * nb + b;
    const C *__restrict__ csq = (const C *)a.csq;
    const C *__restrict__ eph = (const C *)a.eph;
    const int Na = 2 * Lj - 1;
    // this thread's chirped inputs, element tid + s NT in slot s, kept across the blocks
    C base[kRM];
#pragma unroll
    for (int s = 0; s < kRM; ++s) {  // branch-free (see alpha_fwd_fft_kernel)
        const int i = tid + s * NT;
        const bool ok = i < Na;
        const int m = (ok ? i : Na - 1) - (Lj - 1), am = m < 0 ? -m : m;
        C c = (m >= 0 ? Up : Um)[(size_t)am * nb];
        const C w = csq[am];
        if (m < 0) c = cconj(c);
        if (m == 0 && zero_n) c.y = 0.0;
        c = cmul(c, w);
        base[s] = ok ? c : zero2<C>();
    }
    C *__restrict__ Y = (C *)a.out + by * a.s_out + ((size_t)np * nb + b) * T;
    for (int k = 0; k < a.nblk; ++k) {
        const int a0 = k * B;
        auto in = [&](int i, int s) {
            int r = ((i - (Lj - 1)) * a0) % T;
            if (r < 0) r += T;
            return cmul(base[s], eph[r]);
        };
        auto st = [&](int i, C v, int = 0) {
            const int x = i - (Na - 1);
            if (x >= 0 && x < B && a0 + x < T) Y[a0 + x] = cmul(v, csq[x]);
        };
        fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, (const C *)a.hh, in, st, Na);
    }
}

template <class C, int P>
__global__ void __launch_bounds__(P / kRM) alpha_fwd_blk_kernel(const StageArgs a) {
    __shared__ C buf[fft::padded(P)];
    const int t = xcd_column(blockIdx.x, a.Nh * a.nb);
    if (t >= a.Nh * a.nb) return;
    alpha_fwd_blk_body<C, P>(a, t, blockIdx.y, threadIdx.x, buf);
}

// Synthesis: Gs(m) = sum_k e^{-2 pi i m a0/T} sum_{a' < B} X(a0 + a') e^{-2 pi i m a'/T}.
template <class C, int P>
__device__ __forceinline__ void alpha_adj_blk_body(const StageArgs &a, int bx, int by, int tid, C *buf) {
    const int Lj = a.Lj, L = a.L, T = 2 * L - 1, N = a.N, Nh = a.Nh, nb = a.nb, B = a.B;
    const int t = bx;
    const int b = t / Nh, np = t - (t / Nh) * Nh;
    const int ni = (N / 2) + np, nj = N - 1 - ni;
    const bool zero_n = ni == nj;
    const C *__restrict__ X = (const C *)a.in + by * a.s_in + ((size_t)np * nb + b) * T;
    const C *__restrict__ csq = (const C *)a.csq;
    const C *__restrict__ eph = (const C *)a.eph;
    const int Nk = 2 * Lj - 1;
    C acc[kRM];
    int qs[kRM];
#pragma unroll
    for (int s = 0; s < kRM; ++s) {
        acc[s] = zero2<C>();
        qs[s] = -1;
    }
    for (int k = 0; k < a.nblk; ++k) {
        const int a0 = k * B;
        auto in = [&](int i, int = 0) {  // branch-free (see alpha_fwd_fft_kernel)
            const bool ok = i < B && a0 + i < T;
            const int ic = ok ? i : 0;
            const C v = cmulc(X[a0 + ic], csq[ic]);
            return ok ? v : zero2<C>();
        };
        // the block's part of Zh(m), q = m + Lj - 1 < 2Lj - 1, comes out at q + B - 1
        auto st = [&](int i, C v, int s) {
            const int q = i - (B - 1);
            qs[s] = q;
            if (q >= 0 && q < Nk) {
                const int m = q - (Lj - 1);
                int r = (-m * a0) % T;
                if (r < 0) r += T;
                acc[s] = cadd(acc[s], cmul(cmulc(v, csq[m < 0 ? -m : m]), eph[r]));
            }
        };
        fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, (const C *)a.hh, in, st, B);
    }
    const real_t<C> sc = (real_t<C>)a.scale;
    C *__restrict__ Gp = (C *)a.out + by * a.s_out + (size_t)ni * Lj * nb + b;
    C *__restrict__ Gm = (C *)a.out + by * a.s_out + (size_t)nj * Lj * nb + b;
#pragma unroll
    for (int s = 0; s < kRM; ++s) {
        const int q = qs[s];
        if (q >= 0 && q < Nk) {
            const int m = q - (Lj - 1);
            const C z = cscale(acc[s], sc);
            if (m >= 0) Gp[(size_t)m * nb] = z;
            if (m <= 0 && !zero_n) Gm[(size_t)(-m) * nb] = cconj(z);
        }
    }
}

template <class C, int P>
__global__ void __launch_bounds__(P / kRM) alpha_adj_blk_kernel(const StageArgs a) {
    __shared__ C buf[fft::padded(P)];
    const int t = xcd_column(blockIdx.x, a.Nh * a.nb);
    if (t >= a.Nh * a.nb) return;
    alpha_adj_blk_body<C, P>(a, t, blockIdx.y, threadIdx.x, buf);
}

typedef double nt_double2 __attribute__((ext_vector_type(2)));
typedef float nt_float2 __attribute__((ext_vector_type(2)));

// non-temporal 16-byte (double2) or 8-byte (float2) accesses
__device__ __forceinline__ double2 nt_load(const double2 *p) {
    const nt_double2 v = __builtin_nontemporal_load((const nt_double2 *)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 nt_load(const float2 *p) {
    const nt_float2 v = __builtin_nontemporal_load((const nt_float2 *)p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void nt_store(double2 x, double2 *p) {
    nt_double2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_nontemporal_store(v, (nt_double2 *)p);
}
__device__ __forceinline__ void nt_store(float2 x, float2 *p) {
    nt_float2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_nontemporal_store(v, (nt_float2 *)p);
}

// Gamma passes: streaming kernels, each thread takes V consecutive grid points (b, a) of one
// plane (V = 2 when the plane size L T is even, so that W moves in pairs).  W, Y and X are
// touched once per pass, so the accesses are marked non-temporal.  C = double2 with W in
// FP64, or float2 with W in FP32 (mixed precision: FP32 arithmetic and accumulation).
//
// Analysis: W[g][b][a] = sum_{n'} Re(Y[n'][b][a] tg[g][n']), tg = (1 or 2) e^{i n gamma_g}.
template <class C, int V>
__device__ __forceinline__ void gamma_fwd_body(const GammaArgs &a, int bx, int by, int tid) {
    using R = real_t<C>;
    const size_t plane = (size_t)a.L * a.T;
    const size_t e0 = ((size_t)bx * 256 + tid) * V;
    if (e0 >= plane) return;
    const C *__restrict__ Y = (const C *)a.in + by * a.s_y;
    const C *__restrict__ tg = (const C *)a.tg;
    C y[kMaxK][V];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
        if (k < a.Nh) {
#pragma unroll
            for (int v = 0; v < V; ++v) y[k][v] = nt_load(Y + k * plane + e0 + v);
        }
    R *__restrict__ W = (R *)a.wout + by * a.s_w;
    for (int g = 0; g < a.G; ++g) {
        R acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k) {
            if (k < a.Nh) {
                const C w = tg[g * a.Nh + k];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] = fma(y[k][v].x, w.x, fma(-y[k][v].y, w.y, acc[v]));
            }
        }
        R *dst = W + g * plane + e0;
        if constexpr (V == 2) {
            nt_store(mk<C>(acc[0], acc[1]), (C *)dst);
        } else {
            __builtin_nontemporal_store(acc[0], dst);
        }
    }
}

template <class C, int V>
__global__ void __launch_bounds__(256) gamma_fwd_kernel(const GammaArgs a) {
    gamma_fwd_body<C, V>(a, blockIdx.x, blockIdx.y, threadIdx.x);
}

// Synthesis: X[n'][b][a] = sum_g W[g][b][a] tg[g][n'], tg = e^{-i n gamma_g}.
template <class C, int V>
__device__ __forceinline__ void gamma_adj_body(const GammaArgs &a, int bx, int by, int tid) {
    using R = real_t<C>;
    const size_t plane = (size_t)a.L * a.T;
    const size_t e0 = ((size_t)bx * 256 + tid) * V;
    if (e0 >= plane) return;
    const R *__restrict__ W = (const R *)a.win + by * a.s_w;
    const C *__restrict__ tg = (const C *)a.tg;
    C *__restrict__ X = (C *)a.out + by * a.s_y;
    C x[kMaxK][V];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
#pragma unroll
        for (int v = 0; v < V; ++v) x[k][v] = zero2<C>();
    for (int g = 0; g < a.G; ++g) {
        R w[V];
        const R *src = W + g * plane + e0;
        if constexpr (V == 2) {
            const C t = nt_load((const C *)src);
            w[0] = t.x;
            w[1] = t.y;
        } else {
            w[0] = __builtin_nontemporal_load(src);
        }
#pragma unroll
        for (int k = 0; k < kMaxK; ++k) {
            if (k < a.Nh) {
                const C t = tg[g * a.Nh + k];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    x[k][v].x = fma(w[v], t.x, x[k][v].x);
                    x[k][v].y = fma(w[v], t.y, x[k][v].y);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
        if (k < a.Nh) {
#pragma unroll
            for (int v = 0; v < V; ++v) nt_store(x[k][v], X + k * plane + e0 + v);
        }
}

template <class C, int V>
__global__ void __launch_bounds__(256) gamma_adj_kernel(const GammaArgs a) {
    gamma_adj_body<C, V>(a, blockIdx.x, blockIdx.y, threadIdx.x);
}

// Coarse scales of the analysis: both sums at once, sample by sample, without Y (FP64
// arithmetic; C = double2 with FP64 arrays, float2 with the FP32 Ub and W of the mixed path):
//   W(g, b, a) = sum_{n'} Re(tg[g][n'] Y_n'(b, a)),  Y_n(b, a) = sum_{|m|<Lj} C_n(b, m) z^m,
// z = e^{i alpha_a}.  With C_n(b, -m) = conj(Ub[-n][m][b]) and |z| = 1, Y_n = p(z) + conj(q(z)),
// p(z) = sum_{m>=0} Ub[n][m][b] z^m and q(z) = sum_{m>=1} Ub[-n][m][b] z^m, both by Horner's
// rule.  That is Nh (2Lj - 1) complex multiply-adds per sample instead of a blocked chirp
// transform and a pass over Y, worth it while Nh (2Lj - 1) is small next to the G values
// written per sample.  A row of workgroups per ring b; the ring's coefficients (stride nb
// apart in Ub) are staged in LDS once per workgroup and then read by every lane at the same
// address.  PAIR (plane and map stride even, W 16-byte aligned): a thread takes two
// consecutive samples and writes them with one 16-byte store; T being odd, element (b, 0)
// sits at an even offset exactly when b is even, so the pairs of ring b start at
// a = -(b & 1) and the ring's one unpaired sample (first or last) is written alone.
// Otherwise one sample per thread.  NH = Nh (a template parameter, so that the Y values
// of a thread take only the registers they need).
template <bool PAIR, int NH, class C>
__device__ __forceinline__ void alpha_gamma_fwd_body(const AlphaGammaArgs &a, int bx, int bb, int bz, int tid,
                                                     double2 *cs) {
    using R = real_t<C>;
    constexpr int V = PAIR ? 2 : 1;
    constexpr int Nh = NH;
    const int b = bb, Lj = a.Lj, nb = a.nb, N = a.N, T = a.T;
    const C *__restrict__ U = (const C *)a.in + bz * a.s_in + b;
    for (int i = tid; i < 2 * Nh * Lj; i += 256) {
        const int k = i / (2 * Lj), r = i - k * 2 * Lj, side = r >= Lj ? 1 : 0, m = r - side * Lj;
        const int ni = N / 2 + k, row = side ? N - 1 - ni : ni;
        const C u = U[((size_t)row * Lj + m) * nb];
        cs[i] = make_double2((double)u.x, (double)u.y);
    }
    __syncthreads();
    const int t = bx * 256 + tid;
    const int x0 = PAIR ? 2 * t - (b & 1) : t;
    bool ok[V];
    ok[0] = x0 >= 0 && x0 < T;
    if constexpr (PAIR) ok[1] = x0 + 1 < T;
    if (!ok[0] && !ok[V - 1]) return;
    const double2 *__restrict__ eph = (const double2 *)a.eph;
    double2 z[V];
#pragma unroll
    for (int v = 0; v < V; ++v) z[v] = eph[ok[v] ? x0 + v : 0];
    double2 y[NH][V];
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        const double2 *cp = cs + k * 2 * Lj, *cm = cp + Lj;
        {
            double2 p[V], q[V];
#pragma unroll
            for (int v = 0; v < V; ++v) p[v] = q[v] = zero2<double2>();
#pragma unroll 2
            for (int m = Lj - 1; m >= 1; --m) {
                const double2 up = cp[m], um = cm[m];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    p[v] = cadd(cmul(p[v], z[v]), up);
                    q[v] = cadd(cmul(q[v], z[v]), um);
                }
            }
            double2 c0 = cp[0];
            if (k == 0 && (N & 1)) c0.y = 0.0;  // the row n = 0 (N odd): C_0(b, 0) is real
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double2 pv = cadd(cmul(p[v], z[v]), c0), qv = cmul(q[v], z[v]);
                y[k][v] = mk<double2>(pv.x + qv.x, pv.y - qv.y);
            }
        }
    }
    const size_t plane = (size_t)nb * T;
    R *__restrict__ W = (R *)a.wout + bz * a.s_w + (size_t)b * T + x0;
    const double2 *__restrict__ tg = (const double2 *)a.tg;
    for (int g = 0; g < a.G; ++g) {
        double acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0.0;
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            const double2 w = tg[g * Nh + k];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = fma(y[k][v].x, w.x, fma(-y[k][v].y, w.y, acc[v]));
        }
        R *dst = W + g * plane;
        if (PAIR && ok[0] && ok[V - 1]) {
            nt_store(mk<C>((R)acc[0], (R)acc[V - 1]), (C *)dst);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (ok[v]) __builtin_nontemporal_store((R)acc[v], dst + v);
        }
    }
}

template <bool PAIR, int NH, class C>
__global__ void __launch_bounds__(256) alpha_gamma_fwd_kernel(const AlphaGammaArgs a) {
    __shared__ double2 cs[kAlphaGammaCoeffs];  // [k][side][m]: side 0 row n, side 1 row -n
    alpha_gamma_fwd_body<PAIR, NH, C>(a, blockIdx.x, blockIdx.y, blockIdx.z, threadIdx.x, cs);
}

// Coarse scales of the synthesis: both quadratures at once, ring by ring, without X (FP64
// arithmetic; C = double2 with FP64 arrays, float2 with the FP32 W and G of the mixed path):
//   Gs_n(b, m) = scale sum_a X_n(b, a) e^{-i m alpha_a},  X_n(b, a) = sum_g W(g, b, a) tg[g][n],
// for n >= 0 and |m| < Lj.  One workgroup per ring b; the T samples go in chunks of 256:
// the workgroup forms X of the chunk in LDS (one sample per thread, the gamma sum), then
// each output (n, m) is summed over the chunk by H = 256 / ceil(Nh (2Lj - 1) / 2) threads
// (a thread carries two outputs), each over a contiguous run of the chunk as a polynomial
// in rho = e^{-i m alpha_1} (Horner's rule, at most 256 terms) times rho^s0 from the exact
// table at the run's start s0; the H partial sums are added in a fixed order at the end.
// The outputs
// are stored as the alpha stage stores them: Gs_n(b, m) in row n for m >= 0 and conj Gs_n
// (b, m) in row -n at -m for m <= 0 (not for the row n = 0 of odd N).
template <int NH, class C>
__device__ __forceinline__ void gamma_alpha_adj_body(const GammaAlphaArgs &a, int bx, int by, int tid,
                                                     double2 (*xs)[256], double2 (*red)[256]) {
    using R = real_t<C>;
    constexpr int NT = 256;
    const int b = bx, T = a.T, Lj = a.Lj, N = a.N, G = a.G;
    // a thread takes the outputs o and o + np (np = ceil(nouts / 2)) over the same run of
    // samples: two independent Horner chains (the second a copy of the first when o + np
    // is past the end, its result unused)
    const int nm = 2 * Lj - 1, nouts = NH * nm, np = (nouts + 1) >> 1, H = NT / np;
    const int p = tid % np, h = tid / np;
    const bool act = h < H;
    const int o2 = p + np < nouts ? p + np : p;
    const int k1 = p / nm, m1 = p - k1 * nm - (Lj - 1);
    const int k2 = o2 / nm, m2 = o2 - k2 * nm - (Lj - 1);
    const int mm1 = m1 < 0 ? m1 + T : m1, mm2 = m2 < 0 ? m2 + T : m2;  // m mod T
    const double2 *__restrict__ eph = (const double2 *)a.eph;
    const double2 rho1 = cconj(eph[mm1]), rho2 = cconj(eph[mm2]);  // e^{-i m alpha_1}
    const int len = (NT + H - 1) / H;
    const size_t plane = (size_t)a.nb * T;
    const R *__restrict__ Wr = (const R *)a.win + by * a.s_w + (size_t)b * T;
    const double2 *__restrict__ tg = (const double2 *)a.tg;
    // W of the next chunk waits in registers (G <= GMAX = 4 NH - 1, since N <= 2 NH): its
    // loads are issued before the alpha sums of the current chunk
    constexpr int GMAX = 4 * NH - 1;
    double wn[GMAX];
    auto load_chunk = [&](int a0) {
        const int x = a0 + tid;
#pragma unroll
        for (int g = 0; g < GMAX; ++g)
            wn[g] = (g < G && x < T) ? (double)__builtin_nontemporal_load(Wr + g * plane + x) : 0.0;
    };
    load_chunk(0);
    double2 acc1 = zero2<double2>(), acc2 = zero2<double2>();
    for (int a0 = 0; a0 < T; a0 += NT) {
        {
            double2 xv[NH];
#pragma unroll
            for (int kk = 0; kk < NH; ++kk) xv[kk] = zero2<double2>();
#pragma unroll
            for (int g = 0; g < GMAX; ++g) {
                if (g < G) {
#pragma unroll
                    for (int kk = 0; kk < NH; ++kk) {
                        const double2 t = tg[g * NH + kk];
                        xv[kk].x = fma(wn[g], t.x, xv[kk].x);
                        xv[kk].y = fma(wn[g], t.y, xv[kk].y);
                    }
                }
            }
#pragma unroll
            for (int kk = 0; kk < NH; ++kk) xs[kk][tid] = xv[kk];
        }
        if (a0 + NT < T) load_chunk(a0 + NT);
        __syncthreads();
        if (act) {
            // sum_{x in [s0, s1)} X(x) rho^x = rho^s0 sum_j X(s0 + j) rho^j, by Horner's rule in rho
            const int s0 = a0 + h * len, s1 = min(min(s0 + len, a0 + NT), T);
            if (s0 < s1) {
                double2 h1 = zero2<double2>(), h2 = zero2<double2>();
                for (int x = s1 - 1; x >= s0; --x) {
                    const double2 y1 = xs[k1][x - a0], y2 = xs[k2][x - a0];
                    h1 = mk<double2>(fma(h1.x, rho1.x, fma(-h1.y, rho1.y, y1.x)), fma(h1.x, rho1.y, fma(h1.y, rho1.x, y1.y)));
                    h2 = mk<double2>(fma(h2.x, rho2.x, fma(-h2.y, rho2.y, y2.x)), fma(h2.x, rho2.y, fma(h2.y, rho2.x, y2.y)));
                }
                acc1 = cadd(acc1, cmul(h1, cconj(eph[(int)(((long long)mm1 * s0) % T)])));
                acc2 = cadd(acc2, cmul(h2, cconj(eph[(int)(((long long)mm2 * s0) % T)])));
            }
        }
        __syncthreads();
    }
    red[0][tid] = act ? acc1 : zero2<double2>();
    red[1][tid] = act ? acc2 : zero2<double2>();
    __syncthreads();
    if (tid < nouts) {
        const int side = tid < np ? 0 : 1, pp = tid - side * np;
        double2 tot = red[side][pp];
        for (int hh = 1; hh < H; ++hh) tot = cadd(tot, red[side][hh * np + pp]);
        const int k = tid / nm, m = tid - k * nm - (Lj - 1);
        const C z = mk<C>((R)(tot.x * a.scale), (R)(tot.y * a.scale));
        const int ni = N / 2 + k, nj = N - 1 - ni;
        C *__restrict__ Gout = (C *)a.out + by * a.s_out + b;
        if (m >= 0) Gout[((size_t)ni * Lj + m) * a.nb] = z;
        if (m <= 0 && ni != nj) Gout[((size_t)nj * Lj + (size_t)(-m)) * a.nb] = cconj(z);
    }
}

template <int NH, class C>
__global__ void __launch_bounds__(256) gamma_alpha_adj_kernel(const GammaAlphaArgs a) {
    __shared__ double2 xs[NH][256];
    __shared__ double2 red[2][256];
    gamma_alpha_adj_body<NH, C>(a, blockIdx.x, blockIdx.y, threadIdx.x, xs, red);
}

// Complex signals: complex map z = real maps 2z (real part of f) and 2z + 1 (imaginary part);
// W = W_2z + i W_2z+1 (Eq. 1 is linear in f) is written as (re, im) pairs, one point per
// thread, and read back the same way in the synthesis.
template <class C>
__global__ void __launch_bounds__(256) gamma_fwd_cx_kernel(const GammaArgs a) {
    using R = real_t<C>;
    const size_t plane = (size_t)a.L * a.T;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= plane) return;
    const C *__restrict__ Ya = (const C *)a.in + (size_t)(2 * blockIdx.y) * a.s_y + e;
    const C *__restrict__ Yb = Ya + a.s_y;
    const C *__restrict__ tg = (const C *)a.tg;
    C ya[kMaxK], yb[kMaxK];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
        if (k < a.Nh) {
            ya[k] = nt_load(Ya + k * plane);
            yb[k] = nt_load(Yb + k * plane);
        }
    C *__restrict__ W = (C *)a.wout + blockIdx.y * a.s_w + e;
    for (int g = 0; g < a.G; ++g) {
        R ra = 0, rb = 0;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k) {
            if (k < a.Nh) {
                const C w = tg[g * a.Nh + k];
                ra = fma(ya[k].x, w.x, fma(-ya[k].y, w.y, ra));
                rb = fma(yb[k].x, w.x, fma(-yb[k].y, w.y, rb));
            }
        }
        nt_store(mk<C>(ra, rb), W + g * plane);
    }
}

template <class C>
__global__ void __launch_bounds__(256) gamma_adj_cx_kernel(const GammaArgs a) {
    const size_t plane = (size_t)a.L * a.T;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= plane) return;
    const C *__restrict__ W = (const C *)a.win + blockIdx.y * a.s_w + e;
    const C *__restrict__ tg = (const C *)a.tg;
    C xa[kMaxK], xb[kMaxK];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) xa[k] = xb[k] = zero2<C>();
    for (int g = 0; g < a.G; ++g) {
        const C w = nt_load(W + g * plane);
#pragma unroll
        for (int k = 0; k < kMaxK; ++k) {
            if (k < a.Nh) {
                const C t = tg[g * a.Nh + k];
                xa[k].x = fma(w.x, t.x, xa[k].x);
                xa[k].y = fma(w.x, t.y, xa[k].y);
                xb[k].x = fma(w.y, t.x, xb[k].x);
                xb[k].y = fma(w.y, t.y, xb[k].y);
            }
        }
    }
    C *__restrict__ Xa = (C *)a.out + (size_t)(2 * blockIdx.y) * a.s_y + e;
    C *__restrict__ Xb = Xa + a.s_y;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
        if (k < a.Nh) {
            nt_store(xa[k], Xa + k * plane);
            nt_store(xb[k], Xb + k * plane);
        }
}

// ------------------------------------------ synthesis: beta integral and m' folding (Eq. 35, 40)
// Step (3) of both beta quadratures below, once V(m') of the column pair is known: the fold
// over +-m' and the even/odd-l combinations P, Q of the two n columns (see the synthesis
// Wigner kernel).  On entry V of column +n sits in buf[q] (q = m' + Lj - 1) and, with two
// columns, V of column -n in buf[Nk + q].
template <class C, int NT>
__device__ __forceinline__ void fold_pq(C *buf, int tid, int Lj, int m, int n, int ncol, bool odd, int eta, C *Po,
                                        C *Qo) {
    const int Nk = 2 * Lj - 1;
    for (int mp = tid; mp < Lj; mp += NT) {
        C tp = buf[pad(mp + Lj - 1)], tm = ncol > 1 ? buf[pad(Nk + mp + Lj - 1)] : zero2<C>();
        if (mp > 0) {
            C up = buf[pad(-mp + Lj - 1)], um = ncol > 1 ? buf[pad(Nk - mp + Lj - 1)] : zero2<C>();
            if (odd) {
                up = mk<C>(-up.x, -up.y);
                um = mk<C>(-um.x, -um.y);
            }
            tp = cadd(tp, up);
            tm = cadd(tm, um);
        }
        C Pv, Qv;
        if (n == 0) {
            Pv = Qv = rot_i(tp, m + eta);
        } else {
            const C A = rot_i(tp, -n);
            C B = rot_i(tm, n);
            if (mp & 1) B = mk<C>(-B.x, -B.y);
            Pv = rot_i(cadd(A, B), m + eta);
            Qv = rot_i(csub(A, B), m + eta);
        }
        Po[mp] = Pv;
        Qo[mp] = Qv;
    }
}

// Equiangular grid.
// For one column (n, m): (1) Fourier coefficients of the samples extended to the full circle
// (G(2 pi - beta) = s G(beta), s = (-1)^{m+n}):
//   Gh(p) = (1/T) sum_{t<T} ext_t e^{-i p beta_t},  |p| < L,  beta_t = pi(2t+1)/T;
// (2) V(m') = sum_p Gh(p) w(p - m'), |m'| < Lj, with w(q) = int_0^pi sin(b) e^{i q b} db
// (2/(1-q^2) for even q, +-i pi/2 for q = +-1, else 0): the exact beta integral of the
// interpolant against e^{-i m' beta}; (3) the fold U(m') = V(m') + s V(-m') over +-m' (m' > 0;
// U(0) = V(0)) and the even/odd-l combinations P, Q of the two n columns (see the synthesis
// Wigner kernel).
//
// Columns m and m + 1 have opposite s, and one convolution serves both.  Every sample but the
// one at beta = pi (t = L - 1, its own mirror image) pairs with its mirror, so Gh is even in p
// for s = +1 and odd for s = -1 once the beta = pi sample of the s = -1 column is set aside.
// With w = we + wo split into its even part (the even q) and its odd part (q = +-1), the fold
// of an even (odd) Gh only keeps 2 sum_p Gh(p) we(p - m'), and the we-convolution of an odd
// (even) Gh is odd (even) in m'.  So the packed column Gh_m + Gh_{m+1}, convolved with we into
// y(m'), |m'| < Lj, gives U_X(m') = y(m') + s_X y(-m') for both members X (m' > 0; at m' = 0 the
// even member's U is y(0), and the odd member's term is multiplied by Delta^l_{0m} Delta^l_{0n}
// = 0 in the contraction).  The set-aside beta = pi sample G_X(L-1) of the odd member adds
// (1/T) G_X(L-1) (-1)^p to its Gh; through the fold that contributes 2 sum_p (1/T) G_X(L-1) (-1)^p
// wo(p - m'), which vanishes except at m' = L - 1, where it is -(i pi/T) (-1)^L G_X(L-1).
// hh2 is the spectrum of we.
// Work item col = k Mp + c of a scale of band-limit Lj: order k, columns m0 = 2c and m0 + 1
// (Mp = ceil(Lj/2)); in / out: the scale's G and V of the map.
// DIRECT (P = 8192, T = 4095): step (1) as the prime-factor transform of length T (pfa.h).
// UNIFORM: the same barriers for every column (the persistent executor runs several columns in
// one workgroup): the column of order n = 0 also runs the second order's two transforms, on
// its own samples, into LDS slots that the fold does not read.
template <class C, int P, bool DIRECT = false, bool UNIFORM = false>
__device__ __forceinline__ void beta_adj_body(const StageArgs &a, C *buf, int col, int Lj, const C *in, C *out,
                                              const C *hh2, int tid) {
    constexpr int NT = P / kRM;
    const int L = a.L, T = 2 * L - 1, N = a.N;
    const int Mp = (Lj + 1) >> 1;
    const int k = col / Mp, m0 = 2 * (col - (col / Mp) * Mp);
    const bool two = m0 + 1 < Lj;  // column m0 + 1 present
    int n = 0;  // a.nk[k] without a dynamically indexed copy of the argument block
#pragma unroll
    for (int kk = 0; kk < kMaxK; ++kk)
        if (kk == k) n = a.nk[kk];
    const int ncol = n == 0 ? 1 : 2;
    const bool odd0 = ((m0 + n) & 1) != 0;  // column m0 is the odd member (s = -1), else m0 + 1
    const int Nk = 2 * Lj - 1;
    const C *__restrict__ csq = (const C *)a.csq;
    const C *__restrict__ cpp = (const C *)a.cpp;
    // y of order +n by storer slot (two orders).  The storer of the last inverse pass gets
    // element tid + s NT in slot s (span P/kRM = NT), so the slot gives the index back.
    C keep[kRM];
    const int nloop = UNIFORM ? 2 : ncol;
    for (int c = 0; c < nloop; ++c) {
        const int ni = ((c == 0 ? n : -n) + N - 1) >> 1;
        const C *__restrict__ Ga = in + ((size_t)ni * Lj + m0) * L;
        const C *__restrict__ Gb = Ga + L;  // column m0 + 1
        // the packed extended column at t < T
        auto ext = [&](int i) {
            const int b = i < L ? i : 2 * L - 2 - i;
            C va = Ga[b];
            C vb = two ? Gb[b] : zero2<C>();
            C &vo = odd0 ? va : vb;  // the odd member
            if (i == L - 1) vo = zero2<C>();
            else if (i >= L) vo = mk<C>(-vo.x, -vo.y);
            return cadd(va, vb);
        };
        if constexpr (DIRECT) {
            // Gh(p) = (1/T) e^{-i pi p/T} X[p mod T], X = sum_t ext_t e^{-2 pi i p t/T}; X[k] sits at
            // buf[pos_out(k)]; the first pass of the next convolution reads every input before it
            // writes its outputs, so the transform's layout may share the buffer
            static_assert(P == 8192, "the direct transform serves T = 4095");
            pfa::dft_lds<pfa::Len4095T<NT>, -1>(buf, (const C *)a.pcs, tid, 1, [&](int, int t) { return ext(t); });
        } else {
            auto in1 = [&](int i, int = 0) { return i < T ? cmulc(ext(i), csq[i]) : zero2<C>(); };
            // Gh(p), q = p + L - 1 < T, comes out at q + T - 1 (1/T is folded into the spectrum)
            auto st1 = [&](int i, C v, int = 0) {
                const int q = i - (T - 1);
                if (q >= 0 && q < T) buf[pad(q)] = cmulc(v, cpp[q]);
            };
            fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, (const C *)a.hh, in1, st1, T);
        }
        const C *__restrict__ eph = (const C *)a.eph;
        const real_t<C> invT = (real_t<C>)(1.0 / T);
        auto in2 = [&](int i, int = 0) {
            if (i >= T) return zero2<C>();
            if constexpr (!DIRECT) return buf[pad(i)];
            // p = i - (L - 1); e^{i pi p/T} = eph[p/2 mod T] (p even), -eph[(p + T)/2 mod T] (p odd)
            const int p = i - (L - 1);
            const bool oddp = (p & 1) != 0;
            int r = oddp ? (p + T) / 2 : p / 2;
            r %= T;
            if (r < 0) r += T;
            C e = eph[r];
            if (oddp) e = mk<C>(-e.x, -e.y);
            return cscale(cmulc(buf[pfa::Len4095::pos_out(p < 0 ? p + T : p)], e), invT);
        };
        // y(m'), q = m' + Lj - 1 < 2Lj - 1, comes out at q + T - 1.  With two orders the
        // first one waits in registers (each thread keeps the outputs of its storer slots)
        // while the second one uses the whole buffer; the second one goes to slots Nk + q.
        if (c == 0 && nloop > 1) {
            auto st2 = [&](int, C v, int slot) { keep[slot] = v; };
            fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, hh2, in2, st2, T);
        } else {
            const int sh = c * Nk;
            auto st2 = [&](int i, C v, int = 0) {
                const int q = i - (T - 1);
                if (q >= 0 && q < Nk) buf[pad(sh + q)] = v;
            };
            fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, hh2, in2, st2, T);
        }
    }
    if (nloop > 1) {
#pragma unroll
        for (int r = 0; r < kRM; ++r) {
            const int q = tid + r * NT - (T - 1);
            if (q >= 0 && q < Nk) buf[pad(q)] = keep[r];
        }
    }
    __syncthreads();
    // the fold and the P, Q combinations of both members
    using R = real_t<C>;
    const int eta = a.eta_imag ? 1 : 0;
    const R dsc = (R)((L & 1) ? M_PI / T : -M_PI / T);  // -(pi/T) (-1)^L: times i G(L-1)
    for (int x = 0; x < (two ? 2 : 1); ++x) {
        const int m = m0 + x;
        const bool oddx = (x == 0) == odd0;  // this member has s = -1
        C *__restrict__ Po = out + (((size_t)k * 2 + 0) * Lj + m) * Lj;
        C *__restrict__ Qo = out + (((size_t)k * 2 + 1) * Lj + m) * Lj;
        const C *Gx = in + m * (size_t)L;
        for (int mp = tid; mp < Lj; mp += NT) {
            C tp, tm;
            if (mp == 0) {
                tp = oddx ? zero2<C>() : buf[pad(Lj - 1)];
                tm = (oddx || ncol == 1) ? zero2<C>() : buf[pad(Nk + Lj - 1)];
            } else {
                const C yp = buf[pad(mp + Lj - 1)], yn = buf[pad(-mp + Lj - 1)];
                tp = oddx ? csub(yp, yn) : cadd(yp, yn);
                if (ncol > 1) {
                    const C zp = buf[pad(Nk + mp + Lj - 1)], zn = buf[pad(Nk - mp + Lj - 1)];
                    tm = oddx ? csub(zp, zn) : cadd(zp, zn);
                } else {
                    tm = zero2<C>();
                }
                if (oddx && mp == L - 1) {
                    // the set-aside beta = pi samples of orders +n and -n
                    const C gp = Gx[((size_t)((n + N - 1) >> 1) * Lj) * L + (L - 1)];
                    tp = cadd(tp, mk<C>(-dsc * gp.y, dsc * gp.x));
                    if (ncol > 1) {
                        const C gm = Gx[((size_t)((-n + N - 1) >> 1) * Lj) * L + (L - 1)];
                        tm = cadd(tm, mk<C>(-dsc * gm.y, dsc * gm.x));
                    }
                }
            }
            C Pv, Qv;
            if (n == 0) {
                Pv = Qv = rot_i(tp, m + eta);
            } else {
                const C A = rot_i(tp, -n);
                C B = rot_i(tm, n);
                if (mp & 1) B = mk<C>(-B.x, -B.y);
                Pv = rot_i(cadd(A, B), m + eta);
                Qv = rot_i(csub(A, B), m + eta);
            }
            Po[mp] = Pv;
            Qo[mp] = Qv;
        }
    }
}

template <class C, int P, bool DIRECT = false>
__global__ void __launch_bounds__(P / kRM, kMinWaves) beta_adj_fft_kernel(const StageArgs a) {
    __shared__ C buf[fft::padded(P)];
    beta_adj_body<C, P, DIRECT>(a, buf, blockIdx.x, a.Lj, (const C *)a.in + blockIdx.y * a.s_in,
                                (C *)a.out + blockIdx.y * a.s_out, (const C *)a.hh2, threadIdx.x);
}

// The coarse scales of a map in one launch (each alone would fill only a few workgroups):
// workgroups [tab[s].first, tab[s + 1].first) take scale s.
template <class C, int P, bool DIRECT = false, bool UNIFORM = false>
__device__ __forceinline__ void beta_adj_multi_body(const StageArgs &a, const BetaAdjScale *tab, int ns, int bx, int by,
                                                    int tid, C *buf) {
    int s = 0;
    for (int i = 1; i < ns; ++i)
        if (bx >= tab[i].first) s = i;
    const BetaAdjScale e = tab[s];
    beta_adj_body<C, P, DIRECT, UNIFORM>(a, buf, bx - e.first, e.Lj, (const C *)a.in + by * a.s_in + e.in_off,
                                         (C *)a.out + by * a.s_out + e.out_off, (const C *)e.hh2, tid);
}

template <class C, int P, bool DIRECT = false>
__global__ void __launch_bounds__(P / kRM, kMinWaves) beta_adj_multi_kernel(const StageArgs a,
                                                                              const BetaAdjScale *tab, int ns) {
    __shared__ C buf[fft::padded(P)];
    beta_adj_multi_body<C, P, DIRECT>(a, tab, ns, blockIdx.x, blockIdx.y, threadIdx.x, buf);
}

// Driscoll-Healy grid (Eq. 17-18 and 40): theta_t = pi (2t+1)/Tb, t < nb, Tb = 4L, nb = 2L,
// with the quadrature weights q_t of Eq. 18 (sin(theta) included), which integrate the
// product of the samples and e^{-i m' theta} exactly:
//   V(m') = sum_{t<nb} q_t G(theta_t) e^{-i m' theta_t},  |m'| < Lj,
// then the fold (3).  Since m' theta_t = (m'^2 + m' + t^2 - (m' - t)^2) pi/Tb, the sum is one
// chirp convolution per column: V(m') = conj(cpp(m')) sum_t [q_t G_t conj(csq_t)] e^{i pi (m'-t)^2/Tb}.
template <class C, int P>
__global__ void __launch_bounds__(P / kRM, kMinWaves) beta_adj_dh_kernel(const StageArgs a) {
    __shared__ C buf[fft::padded(P)];
    constexpr int NT = P / kRM;
    const int tid = threadIdx.x;
    const int Lj = a.Lj, L = a.L, N = a.N, nb = a.nb;
    const int k = blockIdx.x / Lj, m = blockIdx.x - (blockIdx.x / Lj) * Lj;
    int n = 0;
#pragma unroll
    for (int kk = 0; kk < kMaxK; ++kk)
        if (kk == k) n = a.nk[kk];
    const int ncol = n == 0 ? 1 : 2;
    const bool odd = ((m + n) & 1) != 0;
    const int Nk = 2 * Lj - 1;
    const C *__restrict__ csq = (const C *)a.csq;
    const C *__restrict__ cpp = (const C *)a.cpp + (L - 1);
    const real_t<C> *__restrict__ qw = (const real_t<C> *)a.qw;
    C *__restrict__ Po = (C *)a.out + blockIdx.y * a.s_out + (((size_t)k * 2 + 0) * Lj + m) * Lj;
    C *__restrict__ Qo = (C *)a.out + blockIdx.y * a.s_out + (((size_t)k * 2 + 1) * Lj + m) * Lj;
    // V of column +n by storer slot (two columns); slot s holds element tid + s NT
    C keep[kRM];
    for (int c = 0; c < ncol; ++c) {
        const int ni = ((c == 0 ? n : -n) + N - 1) >> 1;
        const C *__restrict__ Gc = (const C *)a.in + blockIdx.y * a.s_in + ((size_t)ni * Lj + m) * nb;
        auto in = [&](int i, int = 0) { return i < nb ? cscale(cmulc(Gc[i], csq[i]), qw[i]) : zero2<C>(); };
        // V(m'), q = m' + Lj - 1 < 2Lj - 1, comes out at q + nb - 1
        if (c == 0 && ncol > 1) {
            auto st = [&](int i, C v, int slot) {
                const int q = i - (nb - 1);
                keep[slot] = (q >= 0 && q < Nk) ? cmulc(v, cpp[q - (Lj - 1)]) : v;
            };
            fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, (const C *)a.hh, in, st, nb);
        } else {
            const int sh = c * Nk;
            auto st = [&](int i, C v, int = 0) {
                const int q = i - (nb - 1);
                if (q >= 0 && q < Nk) buf[pad(sh + q)] = cmulc(v, cpp[q - (Lj - 1)]);
            };
            fft::convolve_io<P, kRM>(buf, tid, (const C *)a.tw, (const C *)a.hh, in, st, nb);
        }
    }
    if (ncol > 1) {
#pragma unroll
        for (int r = 0; r < kRM; ++r) {
            const int q = tid + r * NT - (nb - 1);
            if (q >= 0 && q < Nk) buf[pad(q)] = keep[r];
        }
    }
    __syncthreads();
    fold_pq<C, NT>(buf, tid, Lj, m, n, ncol, odd, a.eta_imag ? 1 : 0, Po, Qo);
}

}  // namespace s2dw
