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
#include "fft.h"
#include "kernels.h"

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

__device__ __forceinline__ double2 rot_i(double2 z, int e) {
    e &= 3;
    if (e == 0) return z;
    if (e == 1) return make_double2(-z.y, z.x);
    if (e == 2) return make_double2(-z.x, -z.y);
    return make_double2(z.y, -z.x);
}

__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }

}  // namespace

// ------------------------------------------------------------------- analysis: beta (Eq. 29)
// Column (n, m) of scale j: Ub(b) = sum_{|m'|<Lj} U_{m m' n} e^{i m' beta_b}, b < L, with
// U_{m,-m',n} = (-1)^{m+n} U_{m m' n} (only m' >= 0 is stored).  Since m' beta_b =
// 2 pi m' b/T + pi m'/T, the chirp input is U e^{i pi m'(m'+1)/T}.
template <int P>
__global__ void __launch_bounds__(P / kRM, kMinWaves) beta_fwd_fft_kernel(const StageArgs a) {
    __shared__ double2 buf[fft::padded(P)];
    const int tid = threadIdx.x;
    const int Lj = a.Lj, L = a.L;
    const int col = blockIdx.x;  // ni * Lj + m
    const int ni = col / Lj, m = col - ni * Lj;
    const int n = 2 * ni - (a.N - 1);
    const bool odd = ((m + n) & 1) != 0;
    const double2 *__restrict__ Uc = a.in + (size_t)col * Lj;
    const double2 *__restrict__ cpp = a.cpp + (L - 1);
    const double2 *__restrict__ csq = a.csq;
    const int Na = 2 * Lj - 1;
    double2 *__restrict__ out = a.out + (size_t)col * L;
    auto in = [&](int i) {
        if (i >= Na) return zero2();
        const int mp = i - (Lj - 1);
        double2 v = Uc[mp < 0 ? -mp : mp];
        if (mp < 0 && odd) v = make_double2(-v.x, -v.y);
        return cmul(v, cpp[mp]);
    };
    auto st = [&](int i, double2 v) {
        const int b = i - (Na - 1);
        if (b >= 0 && b < L) out[b] = cmul(v, csq[b]);
    };
    fft::convolve_io<P, kRM>(buf, tid, a.tw, a.hh, in, st);
}

// ------------------------------------------------------ analysis: alpha (Eq. 30), two gamma rows
// W(a) = sum_{|m|<Lj} H_m e^{2 pi i m a/T} with H_{-m} = conj(H_m) (real W); the rows g1 and g2
// are packed as H1 + i H2, whose transform is W1 + i W2.
template <int P>
__global__ void __launch_bounds__(P / kRM, kMinWaves) alpha_fwd_fft_kernel(const StageArgs a) {
    __shared__ double2 buf[fft::padded(P)];
    const int tid = threadIdx.x;
    const int Lj = a.Lj, L = a.L, T = 2 * L - 1, G = a.G;
    const int ngp = (G + 1) / 2;
    const int b = blockIdx.x / ngp, gp = blockIdx.x - (blockIdx.x / ngp) * ngp;
    const int g1 = 2 * gp, g2 = 2 * gp + 1;
    const bool two = g2 < G;
    const double2 *__restrict__ H1 = a.in + ((size_t)g1 * L + b) * Lj;
    const double2 *__restrict__ H2 = a.in + ((size_t)(two ? g2 : g1) * L + b) * Lj;
    const double2 *__restrict__ csq = a.csq;
    const int Na = 2 * Lj - 1;
    auto in = [&](int i) {
        if (i >= Na) return zero2();
        const int m = i - (Lj - 1);
        const int am = m < 0 ? -m : m;
        double2 h1 = H1[am], h2 = two ? H2[am] : zero2();
        if (m == 0) {
            h1.y = 0.0;
            h2.y = 0.0;
        } else if (m < 0) {
            h1.y = -h1.y;
            h2.y = -h2.y;
        }
        return cmul(make_double2(h1.x - h2.y, h1.y + h2.x), csq[am]);
    };
    const size_t o1 = ((size_t)g1 * L + b) * T, o2 = ((size_t)g2 * L + b) * T;
    if (a.f32) {
        float *Wf = (float *)a.wout;
        auto st = [&](int i, double2 v) {
            const int x = i - (Na - 1);
            if (x >= 0 && x < T) {
                const double2 c = cmul(v, csq[x]);
                Wf[o1 + x] = (float)c.x;
                if (two) Wf[o2 + x] = (float)c.y;
            }
        };
        fft::convolve_io<P, kRM>(buf, tid, a.tw, a.hh, in, st);
    } else {
        double *W = (double *)a.wout;
        auto st = [&](int i, double2 v) {
            const int x = i - (Na - 1);
            if (x >= 0 && x < T) {
                const double2 c = cmul(v, csq[x]);
                W[o1 + x] = c.x;
                if (two) W[o2 + x] = c.y;
            }
        };
        fft::convolve_io<P, kRM>(buf, tid, a.tw, a.hh, in, st);
    }
}

// ----------------------------------------------------- synthesis: alpha (Eq. 37), two gamma rows
// Zh(m) = sum_a (W1 + i W2)(a) e^{-2 pi i m a/T} for |m| < Lj; then
// W1h(m) = (Zh(m) + conj Zh(-m))/2, W2h(m) = (Zh(m) - conj Zh(-m))/(2i), times 2 pi/T.
template <int P, bool F32>
__device__ __forceinline__ void alpha_adj_body(const StageArgs &a, double2 *buf) {
    const int tid = threadIdx.x;
    constexpr int NT = P / kRM;
    const int Lj = a.Lj, L = a.L, T = 2 * L - 1, G = a.G;
    const int ngp = (G + 1) / 2;
    const int b = blockIdx.x / ngp, gp = blockIdx.x - (blockIdx.x / ngp) * ngp;
    const int g1 = 2 * gp, g2 = 2 * gp + 1;
    const bool two = g2 < G;
    using WT = typename std::conditional<F32, float, double>::type;
    const WT *__restrict__ W1 = (const WT *)a.win + ((size_t)g1 * L + b) * T;
    const WT *__restrict__ W2 = (const WT *)a.win + ((size_t)(two ? g2 : g1) * L + b) * T;
    const double2 *__restrict__ csq = a.csq;
    auto in = [&](int i) {
        if (i >= T) return zero2();
        const double w1 = (double)W1[i];
        const double w2 = two ? (double)W2[i] : 0.0;
        return cmulc(make_double2(w1, w2), csq[i]);
    };
    // Zh(m) for m = q - (Lj-1), q < 2Lj-1, comes out at q + T - 1; it is stored at slot q
    const int Nk = 2 * Lj - 1;
    auto st = [&](int i, double2 v) {
        const int q = i - (T - 1);
        if (q >= 0 && q < Nk) {
            const int m = q - (Lj - 1);
            buf[pad(q)] = cmulc(v, csq[m < 0 ? -m : m]);
        }
    };
    fft::convolve_io<P, kRM>(buf, tid, a.tw, a.hh, in, st);
    const double wa = 0.5 * a.scale;
    double2 *__restrict__ out1 = a.out + ((size_t)g1 * L + b) * Lj;
    double2 *__restrict__ out2 = a.out + ((size_t)g2 * L + b) * Lj;
    for (int m = tid; m < Lj; m += NT) {
        const double2 zp = buf[pad(m + Lj - 1)], zm = buf[pad(-m + Lj - 1)];
        out1[m] = make_double2(wa * (zp.x + zm.x), wa * (zp.y - zm.y));
        if (two) out2[m] = make_double2(wa * (zp.y + zm.y), -wa * (zp.x - zm.x));
    }
}

template <int P>
__global__ void __launch_bounds__(P / kRM, kMinWaves) alpha_adj_fft_kernel(const StageArgs a) {
    __shared__ double2 buf[fft::padded(P)];
    if (a.f32) alpha_adj_body<P, true>(a, buf);
    else alpha_adj_body<P, false>(a, buf);
}

// -------------------------------------------- gamma sums fused with the (m, b) <-> (b, m) transposes
// Analysis (Eq. 28): Hg[g][b][m] = sum_n Ub[n][m][b] e^{i n gamma_g}, g in [gbase, gbase + 16).
__global__ void __launch_bounds__(1024) gamma_fwd_kernel(const GammaArgs a) {
    __shared__ double2 tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int b0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
    const int L = a.L, Lj = a.Lj, N = a.N, G = 2 * N - 1;
    double2 acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int ni = 0; ni < N; ++ni) {
        const int mm = m0 + ty, bb = b0 + tx;
        tile[ty][tx] = (mm < Lj && bb < L) ? a.in[((size_t)ni * Lj + mm) * L + bb] : make_double2(0.0, 0.0);
        __syncthreads();
        const double2 w = tile[tx][ty];  // element (m0 + tx, b0 + ty)
        const int n = 2 * ni - (N - 1);
#pragma unroll
        for (int gg = 0; gg < 16; ++gg) {
            const int g = a.gbase + gg;
            if (g < G) {
                int k = (n * g) % G;
                if (k < 0) k += G;
                acc[gg] = cadd(acc[gg], cmul(w, a.twg[k]));
            }
        }
        __syncthreads();
    }
    const int bb = b0 + ty, mm = m0 + tx;
    if (bb < L && mm < Lj) {
#pragma unroll
        for (int gg = 0; gg < 16; ++gg) {
            const int g = a.gbase + gg;
            if (g < G) a.out[((size_t)g * L + bb) * Lj + mm] = acc[gg];
        }
    }
}

// Synthesis (Eq. 39 with the uniform rule): Gout[n][m][b] = wg sum_g Wh[g][b][m] e^{-i n gamma_g}.
__global__ void __launch_bounds__(1024) gamma_adj_kernel(const GammaArgs a) {
    __shared__ double2 tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int b0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
    const int L = a.L, Lj = a.Lj, N = a.N, G = 2 * N - 1;
    double2 acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int g = 0; g < G; ++g) {
        const int bb = b0 + ty, mm = m0 + tx;
        tile[ty][tx] = (bb < L && mm < Lj) ? a.in[((size_t)g * L + bb) * Lj + mm] : make_double2(0.0, 0.0);
        __syncthreads();
        const double2 w = tile[tx][ty];  // element (b0 + tx, m0 + ty)
#pragma unroll
        for (int ni = 0; ni < 16; ++ni) {
            if (ni < N) {
                const int n = 2 * ni - (N - 1);
                int k = (n * g) % G;
                if (k < 0) k += G;
                acc[ni] = cadd(acc[ni], cmulc(w, a.twg[k]));
            }
        }
        __syncthreads();
    }
    const int mm = m0 + ty, bb = b0 + tx;
    if (bb < L && mm < Lj) {
#pragma unroll
        for (int ni = 0; ni < 16; ++ni)
            if (ni < N) a.out[((size_t)ni * Lj + mm) * L + bb] = cscale(acc[ni], a.scale);
    }
}

// ------------------------------------------ synthesis: beta integral and m' folding (Eq. 35, 40)
// Column pair (+n, -n), fixed m.  (1) Fourier coefficients of the samples extended to the
// full circle (G(2 pi - beta) = (-1)^{m+n} G(beta)):
//   Gh(p) = (1/T) sum_{t<T} ext_t e^{-i p beta_t},  |p| < L,  beta_t = pi(2t+1)/T;
// (2) V(m') = sum_p Gh(p) w(p - m'), |m'| < Lj, with w(q) = int_0^pi sin(b) e^{i q b} db
// (2/(1-q^2) for even q, +-i pi/2 for q = +-1, else 0): the exact beta integral of the
// interpolant against e^{-i m' beta}; (3) the fold over +-m' and the even/odd-l
// combinations P, Q of the two n columns (see the synthesis Wigner kernel).
template <int P>
__global__ void __launch_bounds__(P / kRM, kMinWaves) beta_adj_fft_kernel(const StageArgs a) {
    __shared__ double2 buf[fft::padded(P)];
    constexpr int NT = P / kRM;
    const int tid = threadIdx.x;
    const int Lj = a.Lj, L = a.L, T = 2 * L - 1, N = a.N;
    const int k = blockIdx.x / Lj, m = blockIdx.x - (blockIdx.x / Lj) * Lj;
    int n = 0;  // a.nk[k] without a dynamically indexed copy of the argument block
#pragma unroll
    for (int kk = 0; kk < kMaxK; ++kk)
        if (kk == k) n = a.nk[kk];
    const int ncol = n == 0 ? 1 : 2;
    const bool odd = ((m + n) & 1) != 0;
    const int Nk = 2 * Lj - 1;
    const double2 *__restrict__ csq = a.csq;
    const double2 *__restrict__ cpp = a.cpp;
    double2 *__restrict__ Po = a.out + (((size_t)k * 2 + 0) * Lj + m) * Lj;
    double2 *__restrict__ Qo = a.out + (((size_t)k * 2 + 1) * Lj + m) * Lj;
    for (int c = 0; c < ncol; ++c) {
        const int ni = ((c == 0 ? n : -n) + N - 1) >> 1;
        const double2 *__restrict__ Gc = a.in + ((size_t)ni * Lj + m) * L;
        auto in1 = [&](int i) {
            if (i >= T) return zero2();
            double2 v = i < L ? Gc[i] : Gc[2 * L - 2 - i];
            if (i >= L && odd) v = make_double2(-v.x, -v.y);
            return cmulc(v, csq[i]);
        };
        // Gh(p), q = p + L - 1 < T, comes out at q + T - 1 (1/T is folded into the spectrum)
        auto st1 = [&](int i, double2 v) {
            const int q = i - (T - 1);
            if (q >= 0 && q < T) buf[pad(q)] = cmulc(v, cpp[q]);
        };
        fft::convolve_io<P, kRM>(buf, tid, a.tw, a.hh, in1, st1);
        auto in2 = [&](int i) { return i < T ? buf[pad(i)] : zero2(); };
        // V(m'), q = m' + Lj - 1 < 2Lj - 1, comes out at q + T - 1.  With two columns the
        // first one waits in this block's own output rows (2 Lj slots) while the second one
        // uses the whole buffer; the second one goes to slots Nk + q.
        if (c == 0 && ncol > 1) {
            auto st2 = [&](int i, double2 v) {
                const int q = i - (T - 1);
                if (q >= 0 && q < Nk) {
                    if (q < Lj) Po[q] = v;
                    else Qo[q - Lj] = v;
                }
            };
            fft::convolve_io<P, kRM>(buf, tid, a.tw, a.hh2, in2, st2);
        } else {
            const int sh = c * Nk;
            auto st2 = [&](int i, double2 v) {
                const int q = i - (T - 1);
                if (q >= 0 && q < Nk) buf[pad(sh + q)] = v;
            };
            fft::convolve_io<P, kRM>(buf, tid, a.tw, a.hh2, in2, st2);
        }
    }
    if (ncol > 1) {
        for (int q = tid; q < Nk; q += NT) buf[pad(q)] = q < Lj ? Po[q] : Qo[q - Lj];
        __syncthreads();
    }
    const int eta = a.eta_imag ? 1 : 0;
    for (int mp = tid; mp < Lj; mp += NT) {
        double2 tp = buf[pad(mp + Lj - 1)], tm = ncol > 1 ? buf[pad(Nk + mp + Lj - 1)] : zero2();
        if (mp > 0) {
            double2 up = buf[pad(-mp + Lj - 1)], um = ncol > 1 ? buf[pad(Nk - mp + Lj - 1)] : zero2();
            if (odd) {
                up = make_double2(-up.x, -up.y);
                um = make_double2(-um.x, -um.y);
            }
            tp = cadd(tp, up);
            tm = cadd(tm, um);
        }
        double2 Pv, Qv;
        if (n == 0) {
            Pv = Qv = rot_i(tp, m + eta);
        } else {
            const double2 A = rot_i(tp, -n);
            double2 B = rot_i(tm, n);
            if (mp & 1) B = make_double2(-B.x, -B.y);
            Pv = rot_i(cadd(A, B), m + eta);
            Qv = rot_i(csub(A, B), m + eta);
        }
        Po[mp] = Pv;
        Qo[mp] = Qv;
    }
}

// ------------------------------------------------------------------------------ launchers

#define S2DW_P_SWITCH(P, KER, GRID, ARGS)                                                        \
    switch (P) {                                                                                 \
        case 32: hipLaunchKernelGGL(KER<32>, GRID, dim3(32 / kRM), 0, st, ARGS); break;          \
        case 64: hipLaunchKernelGGL(KER<64>, GRID, dim3(64 / kRM), 0, st, ARGS); break;          \
        case 128: hipLaunchKernelGGL(KER<128>, GRID, dim3(128 / kRM), 0, st, ARGS); break;       \
        case 256: hipLaunchKernelGGL(KER<256>, GRID, dim3(256 / kRM), 0, st, ARGS); break;       \
        case 512: hipLaunchKernelGGL(KER<512>, GRID, dim3(512 / kRM), 0, st, ARGS); break;       \
        case 1024: hipLaunchKernelGGL(KER<1024>, GRID, dim3(1024 / kRM), 0, st, ARGS); break;    \
        case 2048: hipLaunchKernelGGL(KER<2048>, GRID, dim3(2048 / kRM), 0, st, ARGS); break;    \
        case 4096: hipLaunchKernelGGL(KER<4096>, GRID, dim3(4096 / kRM), 0, st, ARGS); break;    \
        case 8192: hipLaunchKernelGGL(KER<8192>, GRID, dim3(8192 / kRM), 0, st, ARGS); break;    \
        default: return hipErrorInvalidValue;                                                    \
    }

hipError_t launch_beta_fwd_fft(const StageArgs &a, int P, hipStream_t st) {
    S2DW_P_SWITCH(P, beta_fwd_fft_kernel, dim3(a.N * a.Lj), a)
    return hipGetLastError();
}

hipError_t launch_alpha_fwd_fft(const StageArgs &a, int P, hipStream_t st) {
    S2DW_P_SWITCH(P, alpha_fwd_fft_kernel, dim3(a.L * ((a.G + 1) / 2)), a)
    return hipGetLastError();
}

hipError_t launch_alpha_adj_fft(const StageArgs &a, int P, hipStream_t st) {
    S2DW_P_SWITCH(P, alpha_adj_fft_kernel, dim3(a.L * ((a.G + 1) / 2)), a)
    return hipGetLastError();
}

hipError_t launch_beta_adj_fft(const StageArgs &a, int P, hipStream_t st) {
    S2DW_P_SWITCH(P, beta_adj_fft_kernel, dim3(a.K * a.Lj), a)
    return hipGetLastError();
}

hipError_t launch_gamma_fwd(const GammaArgs &a0, hipStream_t st) {
    dim3 grid((a0.L + 31) / 32, (a0.Lj + 31) / 32);
    const int G = 2 * a0.N - 1;
    for (int gb = 0; gb < G; gb += 16) {
        GammaArgs a = a0;
        a.gbase = gb;
        hipLaunchKernelGGL(gamma_fwd_kernel, grid, dim3(1024), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_gamma_adj(const GammaArgs &a, hipStream_t st) {
    dim3 grid((a.L + 31) / 32, (a.Lj + 31) / 32);
    hipLaunchKernelGGL(gamma_adj_kernel, grid, dim3(1024), 0, st, a);
    return hipGetLastError();
}

}  // namespace s2dw
