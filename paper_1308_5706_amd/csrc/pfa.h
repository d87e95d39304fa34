// Direct odd-length DFTs held in LDS for gfx950 by the prime-factor (Good-Thomas) mapping,
// for the transform lengths T = 2L - 1 of two band-limits: T = 2047 = 23 x 89 (L = 1024) and
// T = 4095 = 5 x 7 x 9 x 13 (L = 2048).  They replace the chirp convolution (two FFTs of
// about 2T points) where they apply.
//
// With T = q_1 ... q_D, pairwise coprime factors, an input index n is held at the
// coordinates n_i = (n mod q_i) inv(T/q_i mod q_i) mod q_i, so that n = sum_i (T/q_i) n_i
// (mod T); then n k / T = sum_i n_i k / q_i (mod 1), and
//     X[k] = sum_{n_1 .. n_D} x[n] prod_i e^{S 2 pi i n_i k_i / q_i},   k_i = k mod q_i:
// a D-dimensional DFT with no twiddle factors, one length-q_i DFT along each dimension.
// A column lives in LDS as the array [q_1]...[q_D] (last index fastest).
//
// Length-q DFTs (q odd) by the symmetric form: with a_r = x_r + x_{q-r}, b_r = x_r - x_{q-r},
//     X_0 = x_0 + sum_r a_r,
//     X_k = x_0 + sum_r a_r cos(2 pi r k/q) + S i sum_r b_r sin(2 pi r k/q),
//     X_{q-k} = x_0 + sum_r a_r cos(...) - S i sum_r b_r sin(...),      r, k = 1 .. (q-1)/2,
// (q - 1)^2 real multiply-adds per line.  Small q: one thread per line, the line in
// registers.  Large q (89): the lanes of a wave take the lines of the workgroup's columns
// and each wave a group of output pairs k, so that the cosines and sines a wave needs are
// the same in all its lanes (scalar loads).
//
// cs: per factor q, cos and sin of 2 pi j/q for j < q; for q = 89 also, per wave w of the
// large stage, the values at r (1 + w KG + kk) for r = 1..44, kk < KG, in that order.
#pragma once

#include <hip/hip_runtime.h>

#include "fft.h"

namespace s2dw {
namespace pfa {

using fft::cadd;
using fft::csub;
using fft::mk;
using fft::real_t;

// Offsets (in entries) of the constant tables of each length.
struct Tab2047 {
    static constexpr int c23 = 0, c89 = 23, g89 = 23 + 89;
    static constexpr int NW = 4, KG = 11;  // waves of the large stage, output pairs per wave
    // the same constants grouped for eight waves of six output pairs (the last wave's four
    // pairs beyond k = 44 are computed and not used)
    static constexpr int g89w = g89 + NW * 44 * KG, NWW = 8, KGW = 6;
    static constexpr int size = g89w + NWW * 44 * KGW;
};
struct Tab4095 {
    static constexpr int c5 = 0, c7 = 5, c9 = 12, c13 = 21;
    static constexpr int size = 5 + 7 + 9 + 13;
};

// a + S i b, a - S i b
template <int S, class C>
__device__ __forceinline__ void plus_minus_ib(C a, C b, C &p, C &m) {
    // i b = (-b.y, b.x)
    const C ib = S > 0 ? mk<C>(-b.y, b.x) : mk<C>(b.y, -b.x);
    p = cadd(a, ib);
    m = csub(a, ib);
}

// Length-Q DFTs (Q odd, small) along the dimension of element stride ST of NC columns of T
// elements (column c at buf + c * CS), one thread per line, in place; tab: cos and sin of
// 2 pi j/Q.  Every line is read and written by one thread only.
template <int Q, int ST, int T, int NTH, int S, class C>
__device__ __forceinline__ void stage_small(C *buf, int CS, int NC, const C *__restrict__ tab, int tid) {
    constexpr int H = (Q - 1) / 2, LINES = T / Q;
    for (int li = tid; li < NC * LINES; li += NTH) {
        const int c = li / LINES, l = li - c * LINES;
        C *p = buf + c * CS + (l / ST) * (Q * ST) + (l % ST);
        const C x0 = p[0];
        C a[H], b[H];
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            const C u = p[r * ST], v = p[(Q - r) * ST];
            a[r - 1] = cadd(u, v);
            b[r - 1] = csub(u, v);
        }
        C s0 = x0;
#pragma unroll
        for (int r = 0; r < H; ++r) s0 = cadd(s0, a[r]);
        p[0] = s0;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            C A = x0, B = mk<C>(0, 0);
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                const C t = tab[(r * k) % Q];
                A.x = fma(a[r - 1].x, t.x, A.x);
                A.y = fma(a[r - 1].y, t.x, A.y);
                B.x = fma(b[r - 1].x, t.y, B.x);
                B.y = fma(b[r - 1].y, t.y, B.y);
            }
            C xp, xm;
            plus_minus_ib<S>(A, B, xp, xm);
            p[k * ST] = xp;
            p[(Q - k) * ST] = xm;
        }
    }
}

// Length-89 DFTs along the contiguous dimension of NC columns of T elements (NC * T/89 <= 64
// lines): lane = line, wave w = output pairs k = 1 + w KG .. (wave 0 also X_0).  tabg: the
// constants of the groups (see above).  Ends with a barrier; the lines are rewritten in place
// after every wave has read them.
template <int T, int NW, int KG, int S, class C>
__device__ __forceinline__ void stage89(C *buf, int CS, int NC, const C *__restrict__ tabg, int tid) {
    constexpr int Q = 89, H = 44, LINES = T / Q;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool act = lane < NC * LINES;
    const int c = lane / LINES, l = lane - (lane / LINES) * LINES;
    C *p = buf + (act ? c * CS + l * Q : 0);
    const C x0 = p[0];
    C A[KG], B[KG];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
        A[kk] = x0;
        B[kk] = mk<C>(0, 0);
    }
    C s0 = x0;
    const C *__restrict__ tw = tabg + w * (H * KG);
#pragma unroll 4
    for (int r = 1; r <= H; ++r) {
        const C u = p[r], v = p[Q - r];
        const C ar = cadd(u, v), br = csub(u, v);
        s0 = cadd(s0, ar);
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            const C t = tw[(r - 1) * KG + kk];
            A[kk].x = fma(ar.x, t.x, A[kk].x);
            A[kk].y = fma(ar.y, t.x, A[kk].y);
            B[kk].x = fma(br.x, t.y, B[kk].x);
            B[kk].y = fma(br.y, t.y, B[kk].y);
        }
    }
    __syncthreads();
    if (act) {
        if (w == 0) p[0] = s0;
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            const int k = 1 + w * KG + kk;
            if (k <= H) {
                C xp, xm;
                plus_minus_ib<S>(A[kk], B[kk], xp, xm);
                p[k] = xp;
                p[Q - k] = xm;
            }
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------------ T = 2047 = 23 x 89
// Two columns per workgroup of 256 threads (4 waves), 2 x 2047 elements of LDS.
struct Len2047 {
    static constexpr int T = 2047, NC = 2, NTH = 256, CS = 2047;
    static constexpr int lds = NC * CS;
    // the length-89 stage: waves, output pairs per wave, offset of its constants
    static constexpr int NW = Tab2047::NW, KG = Tab2047::KG, G89 = Tab2047::g89;
    // coordinates of index n: (n mod 23) * 15 mod 23 (15 = 89^-1 mod 23) and
    // (n mod 89) * 31 mod 89 (31 = 23^-1 mod 89); the array is [23][89]
    __device__ static __forceinline__ int pos_in(int n) { return ((n % 23) * 15 % 23) * 89 + (n % 89) * 31 % 89; }
    __device__ static __forceinline__ int pos_out(int k) { return (k % 23) * 89 + (k % 89); }
};

// The same length on workgroups of 512 threads (8 waves): two columns as before, the
// length-89 stage spread over eight waves of six output pairs each, so that a wave holds
// fewer accumulators and twice as many waves share the CU.
struct Len2047W : Len2047 {
    static constexpr int NTH = 512, NW = Tab2047::NWW, KG = Tab2047::KGW, G89 = Tab2047::g89w;
};

// The stages alone, on inputs already placed at buf[c * CS + pos_in(n)] (after a barrier);
// output k of column c ends at buf[c * CS + pos_out(k)] (after a barrier).
template <int S, class LN, class C>
__device__ __forceinline__ void dft2047_stages(C *buf, const C *__restrict__ tab, int tid, int ncol) {
    stage_small<23, 89, LN::T, LN::NTH, S>(buf, LN::CS, ncol, tab + Tab2047::c23, tid);
    __syncthreads();
    stage89<LN::T, LN::NW, LN::KG, S>(buf, LN::CS, ncol, tab + LN::G89, tid);
}

// in(c, n) gives element n < T of column c; on return output k of column c sits at
// buf[c * CS + pos_out(k)] (after a barrier).
template <int S, class LN, class C, class In>
__device__ __forceinline__ void dft2047_lds(C *buf, const C *__restrict__ tab, int tid, int ncol, In in) {
    for (int e = tid; e < ncol * LN::T; e += LN::NTH) {
        const int c = e / LN::T, n = e - (e / LN::T) * LN::T;
        buf[c * LN::CS + LN::pos_in(n)] = in(c, n);
    }
    __syncthreads();
    dft2047_stages<S, LN>(buf, tab, tid, ncol);
}

// ------------------------------------------------------------------ T = 4095 = 5 x 7 x 9 x 13
// One column per workgroup of 256 threads, 4095 elements of LDS, the array [5][7][9][13].
struct Len4095 {
    static constexpr int T = 4095, NC = 1, NTH = 256, CS = 4095;
    static constexpr int lds = CS;
    // inverses: (819 mod 5)^-1 = 4, (585 mod 7)^-1 = 2, (455 mod 9)^-1 = 2, (315 mod 13)^-1 = 9
    __device__ static __forceinline__ int pos_in(int n) {
        return ((n % 5) * 4 % 5) * 819 + ((n % 7) * 2 % 7) * 117 + ((n % 9) * 2 % 9) * 13 + (n % 13) * 9 % 13;
    }
    __device__ static __forceinline__ int pos_out(int k) { return (k % 5) * 819 + (k % 7) * 117 + (k % 9) * 13 + k % 13; }
};

// The same length with NTH threads per workgroup (the chirp kernels' thread counts).
template <int NTH_>
struct Len4095T : Len4095 {
    static constexpr int NTH = NTH_;
};

template <int S, int NTH, class C>
__device__ __forceinline__ void dft4095_stages(C *buf, const C *__restrict__ tab, int tid, int ncol) {
    using L = Len4095;
    stage_small<13, 1, L::T, NTH, S>(buf, L::CS, ncol, tab + Tab4095::c13, tid);
    __syncthreads();
    stage_small<9, 13, L::T, NTH, S>(buf, L::CS, ncol, tab + Tab4095::c9, tid);
    __syncthreads();
    stage_small<7, 117, L::T, NTH, S>(buf, L::CS, ncol, tab + Tab4095::c7, tid);
    __syncthreads();
    stage_small<5, 819, L::T, NTH, S>(buf, L::CS, ncol, tab + Tab4095::c5, tid);
    __syncthreads();
}

template <int S, int NTH, class C, class In>
__device__ __forceinline__ void dft4095_lds(C *buf, const C *__restrict__ tab, int tid, int ncol, In in) {
    using L = Len4095;
    for (int e = tid; e < ncol * L::T; e += NTH) {
        const int c = e / L::T, n = e - (e / L::T) * L::T;
        buf[c * L::CS + L::pos_in(n)] = in(c, n);
    }
    __syncthreads();
    dft4095_stages<S, NTH>(buf, tab, tid, ncol);
}

// The transform of length LN::T of ncol columns: in(c, n) gives element n of column c,
// out(c, k, X) takes output k.
template <class LN, int S, class C, class In, class Out>
__device__ __forceinline__ void dft(C *buf, const C *__restrict__ tab, int tid, int ncol, In in, Out out) {
    if constexpr (LN::T == 2047) dft2047_lds<S, LN>(buf, tab, tid, ncol, in);
    else dft4095_lds<S, LN::NTH>(buf, tab, tid, ncol, in);
    for (int e = tid; e < ncol * LN::T; e += LN::NTH) {
        const int c = e / LN::T, k = e - (e / LN::T) * LN::T;
        out(c, k, buf[c * LN::CS + LN::pos_out(k)]);
    }
}

// The stages of LN on inputs already placed at buf[c * CS + pos_in(n)] (after a barrier);
// output k of column c ends at buf[c * CS + pos_out(k)] (after a barrier).
template <class LN, int S, class C>
__device__ __forceinline__ void dft_stages(C *buf, const C *__restrict__ tab, int tid, int ncol) {
    if constexpr (LN::T == 2047) dft2047_stages<S, LN>(buf, tab, tid, ncol);
    else dft4095_stages<S, LN::NTH>(buf, tab, tid, ncol);
}

// As dft, leaving output k of column c at buf[c * CS + pos_out(k)].
template <class LN, int S, class C, class In>
__device__ __forceinline__ void dft_lds(C *buf, const C *__restrict__ tab, int tid, int ncol, In in) {
    if constexpr (LN::T == 2047) dft2047_lds<S, LN>(buf, tab, tid, ncol, in);
    else dft4095_lds<S, LN::NTH>(buf, tab, tid, ncol, in);
}

}  // namespace pfa
}  // namespace s2dw
