// Separation-of-variables stages of the wavelet transform (Sec. 3.2-3.3) on gfx950:
// the beta, gamma and alpha sums of analysis (Eq. 28-30) and the alpha, gamma and
// beta quadratures of synthesis (Eq. 36-40) on the equiangular grid
//   alpha_a = 2 pi a/(2L-1), beta_b = pi (2b+1)/(2L-1) (b < L), gamma_g = 2 pi g/(2N-1).
// These are direct sums (O(L) per output) with exact twiddle indexing.
#include "kernels.h"

namespace s2dw {

// ------------------------------------------------------------------ analysis: beta (Eq. 29)
// Ub_{mn}(beta_b) = sum_{|m'|<Lj} U_{m m' n} e^{i m' beta_b}.  With U_{m,-m',n} =
// (-1)^{m+n} U_{m m' n} this is U_{m0n} + 2 sum_{m'>0} U cos(m' beta) for even m+n and
// 2i sum_{m'>0} U sin(m' beta) for odd m+n.
__global__ void __launch_bounds__(256) beta_fwd_kernel(const BetaFwdArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = blockIdx.x * 64 + lane;
    const int b = blockIdx.y * 4 + wave;
    const int ni = blockIdx.z;
    const int L = a.L, Lj = a.Lj;
    if (m >= Lj || b >= L) return;
    const int n = 2 * ni - (a.N - 1);
    const bool cosine = ((m + n) & 1) == 0;
    const double2 *__restrict__ U = a.U + (size_t)ni * Lj * Lj + m;
    const int P = 4 * L - 2, st = 2 * b + 1;
    int idx = 0;
    double ar = 0.0, ai = 0.0;
    for (int mp = 1; mp < Lj; ++mp) {
        idx += st;
        if (idx >= P) idx -= P;
        const double2 e = a.twb[idx];
        const double w = cosine ? e.x : e.y;
        const double2 u = U[(size_t)mp * Lj];
        ar = fma(u.x, w, ar);
        ai = fma(u.y, w, ai);
    }
    const double2 u0 = U[0];
    a.Ub[((size_t)ni * L + b) * Lj + m] =
        cosine ? make_double2(u0.x + 2.0 * ar, u0.y + 2.0 * ai) : make_double2(-2.0 * ai, 2.0 * ar);
}

hipError_t launch_beta_fwd(const BetaFwdArgs &a, hipStream_t st) {
    dim3 grid((a.Lj + 63) / 64, (a.L + 3) / 4, a.N);
    hipLaunchKernelGGL(beta_fwd_kernel, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------------ analysis: gamma + alpha (Eq. 28, 30)
// H_m = sum_n Ub_{mn}(beta_b) e^{i n gamma_g};  W(alpha_a) = Re H_0 + 2 Re sum_{m>0} H_m e^{i m alpha_a}
// (the m < 0 half is the complex conjugate for a real signal).
__global__ void __launch_bounds__(256) alpha_fwd_kernel(const AlphaFwdArgs a) {
    extern __shared__ double2 lds[];
    const int L = a.L, Lj = a.Lj, M = 2 * L - 1, G = 2 * a.N - 1;
    double2 *H = lds;
    double2 *tw = lds + Lj;
    const int b = blockIdx.x, g = blockIdx.y;
    for (int i = threadIdx.x; i < M; i += blockDim.x) tw[i] = a.twa[i];
    for (int m = threadIdx.x; m < Lj; m += blockDim.x) {
        double hr = 0.0, hi = 0.0;
        for (int ni = 0; ni < a.N; ++ni) {
            const int n = 2 * ni - (a.N - 1);
            int k = (n * g) % G;
            if (k < 0) k += G;
            const double2 e = a.twg[k];
            const double2 u = a.Ub[((size_t)ni * L + b) * Lj + m];
            hr += u.x * e.x - u.y * e.y;
            hi += u.x * e.y + u.y * e.x;
        }
        H[m] = make_double2(hr, hi);
    }
    __syncthreads();
    for (int aa = threadIdx.x; aa < M; aa += blockDim.x) {
        double s = 0.0;
        int idx = 0;
        for (int mm = 1; mm < Lj; ++mm) {
            idx += aa;
            if (idx >= M) idx -= M;
            const double2 h = H[mm], e = tw[idx];
            s = fma(h.x, e.x, s);
            s = fma(-h.y, e.y, s);
        }
        s = H[0].x + 2.0 * s;
        const size_t o = ((size_t)g * L + b) * M + aa;
        if (a.f32) ((float *)a.W)[o] = (float)s;
        else ((double *)a.W)[o] = s;
    }
}

hipError_t launch_alpha_fwd(const AlphaFwdArgs &a, hipStream_t st) {
    size_t sh = sizeof(double2) * ((size_t)a.Lj + 2 * a.L - 1);
    if (sh > 65536) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(alpha_fwd_kernel, dim3(a.L, 2 * a.N - 1), dim3(256), sh, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------------ synthesis: alpha + gamma (Eq. 37, 39)
// G_mn(beta_b) = (2 pi/(2L-1)) (2 pi/(2N-1)) sum_g e^{-i n gamma_g} sum_a W(a,b,g) e^{-i m alpha_a}
// for 0 <= m < Lj: the uniform rules are exact for the band-limits in alpha and gamma.
__global__ void __launch_bounds__(256) alpha_adj_kernel(const AlphaAdjArgs a) {
    extern __shared__ double2 lds[];
    const int L = a.L, Lj = a.Lj, M = 2 * L - 1, G = 2 * a.N - 1;
    double2 *tw = lds;
    double *row = (double *)(lds + M);
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    for (int i = threadIdx.x; i < M; i += blockDim.x) tw[i] = a.twa[i];
    double accr[16], acci[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) accr[i] = acci[i] = 0.0;
    for (int g = 0; g < G; ++g) {
        __syncthreads();
        const size_t base = ((size_t)g * L + b) * M;
        for (int i = threadIdx.x; i < M; i += blockDim.x)
            row[i] = a.f32 ? (double)((const float *)a.W)[base + i] : ((const double *)a.W)[base + i];
        __syncthreads();
        if (m < Lj) {
            double hr = 0.0, hi = 0.0;
            int idx = 0;
            for (int aa = 0; aa < M; ++aa) {
                const double w = row[aa];
                const double2 e = tw[idx];
                hr = fma(w, e.x, hr);
                hi = fma(-w, e.y, hi);
                idx += m;
                if (idx >= M) idx -= M;
            }
#pragma unroll
            for (int ni = 0; ni < 16; ++ni) {
                if (ni < a.N) {
                    const int n = 2 * ni - (a.N - 1);
                    int k = (-n * g) % G;
                    if (k < 0) k += G;
                    const double2 e = a.twg[k];
                    accr[ni] += hr * e.x - hi * e.y;
                    acci[ni] += hr * e.y + hi * e.x;
                }
            }
        }
    }
    if (m < Lj) {
#pragma unroll
        for (int ni = 0; ni < 16; ++ni)
            if (ni < a.N) a.G[((size_t)ni * L + b) * Lj + m] = make_double2(a.scale * accr[ni], a.scale * acci[ni]);
    }
}

hipError_t launch_alpha_adj(const AlphaAdjArgs &a, hipStream_t st) {
    const int M = 2 * a.L - 1;
    size_t sh = sizeof(double2) * (size_t)M + sizeof(double) * (size_t)M;
    if (sh > 65536) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(alpha_adj_kernel, dim3((a.Lj + 255) / 256, a.L), dim3(256), sh, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------- synthesis: beta interpolation (Eq. 40)
// The samples G_mn(beta_b), b < L, extended to the full circle by G(2 pi - beta) =
// (-1)^{m+n} G(beta), have Fourier coefficients on |p| < L
//   Gh(p) = (1/(2L-1)) [ sum_{b<L-1} G_b (e^{-i p beta_b} + s e^{i p beta_b}) + G_{L-1} (-1)^p ]
// with s = (-1)^{m+n} (beta_{L-1} = pi is its own mirror image).
__global__ void __launch_bounds__(256) beta_hat_kernel(const BetaHatArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int L = a.L, Lj = a.Lj, M = 2 * L - 1;
    const int m = blockIdx.x * 64 + lane;
    const int pi = blockIdx.y * 4 + wave;
    const int ni = blockIdx.z;
    if (m >= Lj || pi >= M) return;
    const int p = pi - (L - 1);
    const int n = 2 * ni - (a.N - 1);
    const bool cosine = ((m + n) & 1) == 0;
    const double2 *__restrict__ G = a.G + (size_t)ni * L * Lj + m;
    const int P = 4 * L - 2;
    int pm = p % P;
    if (pm < 0) pm += P;
    const int st = (2 * pm) % P;
    int idx = pm;
    double ar = 0.0, ai = 0.0;
    for (int b = 0; b < L - 1; ++b) {
        const double2 e = a.twb[idx];
        const double w = cosine ? e.x : e.y;
        const double2 v = G[(size_t)b * Lj];
        ar = fma(v.x, w, ar);
        ai = fma(v.y, w, ai);
        idx += st;
        if (idx >= P) idx -= P;
    }
    double2 r = cosine ? make_double2(2.0 * ar, 2.0 * ai) : make_double2(2.0 * ai, -2.0 * ar);
    const double2 gl = G[(size_t)(L - 1) * Lj];
    const double sg = (p & 1) ? -1.0 : 1.0;
    r.x = (r.x + sg * gl.x) / (double)M;
    r.y = (r.y + sg * gl.y) / (double)M;
    a.Gh[((size_t)ni * M + pi) * Lj + m] = r;
}

hipError_t launch_beta_hat(const BetaHatArgs &a, hipStream_t st) {
    dim3 grid((a.Lj + 63) / 64, (2 * a.L - 1 + 3) / 4, a.N);
    hipLaunchKernelGGL(beta_hat_kernel, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

// ----------------------------------------------- synthesis: beta integral and m' folding (Eq. 35)
// V_{m m' n} = int_0^pi sin(beta) G_mn(beta) e^{-i m' beta} d beta = sum_p Gh(p) w(p - m') with
// w(q) = int_0^pi sin(b) e^{i q b} db = 2/(1-q^2) (q even), +-i pi/2 (q = +-1), 0 otherwise.
// Folded: Vt_{m'} = V_{m'} + (-1)^{m+n} V_{-m'} (m' > 0), Vt_0 = V_0.  Then with
// A = i^{-n} Vt(+n), B = (-1)^{m'} i^{n} Vt(-n):  P = eta i^m (A + B), Q = eta i^m (A - B),
// the values the synthesis Wigner kernel contracts at even and odd l.
__global__ void __launch_bounds__(256) beta_conv_kernel(const BetaConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int L = a.L, Lj = a.Lj, M = 2 * L - 1;
    const int m = blockIdx.x * 64 + lane;
    const int mp = blockIdx.y * 4 + wave;
    const int k = blockIdx.z;
    if (m >= Lj || mp >= Lj) return;
    const int n = a.nk[k];
    const int nip = (n + a.N - 1) >> 1, nim = (-n + a.N - 1) >> 1;
    const double2 *__restrict__ GP = a.Gh + (size_t)nip * M * Lj + m;
    const double2 *__restrict__ GM = a.Gh + (size_t)nim * M * Lj + m;
    const int W0 = 3 * L;
    double vpr = 0, vpi = 0, vmr = 0, vmi = 0;  // column +n: V(m'), V(-m')
    double upr = 0, upi = 0, umr = 0, umi = 0;  // column -n
    int pstart = -(L - 1);
    if (((pstart - mp) & 1) != 0) ++pstart;
    for (int p = pstart; p <= L - 1; p += 2) {
        const double w1 = a.wt[p - mp + W0], w2 = a.wt[p + mp + W0];
        const size_t o = (size_t)(p + L - 1) * Lj;
        const double2 gp = GP[o], gm = GM[o];
        vpr = fma(gp.x, w1, vpr); vpi = fma(gp.y, w1, vpi);
        vmr = fma(gp.x, w2, vmr); vmi = fma(gp.y, w2, vmi);
        upr = fma(gm.x, w1, upr); upi = fma(gm.y, w1, upi);
        umr = fma(gm.x, w2, umr); umi = fma(gm.y, w2, umi);
    }
    // q = +-1 terms: w(1) = i pi/2, w(-1) = -i pi/2
    const double h = 1.5707963267948966;
    auto add_i = [&](const double2 *Gc, int p, double c, double &re, double &im) {
        if (p < -(L - 1) || p > L - 1) return;
        const double2 g = Gc[(size_t)(p + L - 1) * Lj];
        re += -c * g.y;
        im += c * g.x;
    };
    add_i(GP, mp + 1, h, vpr, vpi);
    add_i(GP, mp - 1, -h, vpr, vpi);
    add_i(GP, 1 - mp, h, vmr, vmi);
    add_i(GP, -1 - mp, -h, vmr, vmi);
    add_i(GM, mp + 1, h, upr, upi);
    add_i(GM, mp - 1, -h, upr, upi);
    add_i(GM, 1 - mp, h, umr, umi);
    add_i(GM, -1 - mp, -h, umr, umi);
    const double s = ((m + n) & 1) ? -1.0 : 1.0;
    double2 tp, tm;  // folded values of the +n and -n columns
    if (mp == 0) {
        tp = make_double2(vpr, vpi);
        tm = make_double2(upr, upi);
    } else {
        tp = make_double2(vpr + s * vmr, vpi + s * vmi);
        tm = make_double2(upr + s * umr, upi + s * umi);
    }
    auto rot = [](double2 z, int e) {
        e &= 3;
        if (e == 0) return z;
        if (e == 1) return make_double2(-z.y, z.x);
        if (e == 2) return make_double2(-z.x, -z.y);
        return make_double2(z.y, -z.x);
    };
    const int eta = a.eta_imag ? 1 : 0;
    double2 P, Q;
    if (n == 0) {
        P = Q = rot(tp, m + eta);
    } else {
        double2 A = rot(tp, -n);
        double2 B = rot(tm, n);
        if (mp & 1) B = make_double2(-B.x, -B.y);
        P = rot(make_double2(A.x + B.x, A.y + B.y), m + eta);
        Q = rot(make_double2(A.x - B.x, A.y - B.y), m + eta);
    }
    a.V[(((size_t)k * 2 + 0) * Lj + mp) * Lj + m] = P;
    a.V[(((size_t)k * 2 + 1) * Lj + mp) * Lj + m] = Q;
}

hipError_t launch_beta_conv(const BetaConvArgs &a, hipStream_t st) {
    dim3 grid((a.Lj + 63) / 64, (a.Lj + 3) / 4, a.K);
    hipLaunchKernelGGL(beta_conv_kernel, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------- misc

__global__ void pad_flm_kernel(const double2 *flm, double2 *fpad, int L, int Lp) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (m >= Lp) return;
    fpad[(size_t)l * Lp + m] = (m <= l) ? flm[(size_t)l * l + l + m] : make_double2(0.0, 0.0);
}

hipError_t launch_pad_flm(const double2 *flm, double2 *fpad, int L, int Lp, hipStream_t st) {
    hipLaunchKernelGGL(pad_flm_kernel, dim3((Lp + 255) / 256, L), dim3(256), 0, st, flm, fpad, L, Lp);
    return hipGetLastError();
}

// W^Phi_lm = sqrt(4 pi/(2l+1)) f_lm Phi_l0 (Eq. 31); Phi is real.
__global__ void scaling_kernel(const double2 *flm, const double *phi, double2 *wphi, int L) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (m > 2 * l) return;
    const size_t i = (size_t)l * l + m;
    const double c = sqrt(4.0 * 3.14159265358979323846 / (2.0 * l + 1.0)) * phi[l];
    const double2 f = flm[i];
    wphi[i] = make_double2(c * f.x, c * f.y);
}

hipError_t launch_scaling(const double2 *flm, const double *phi, double2 *wphi, int L, hipStream_t st) {
    hipLaunchKernelGGL(scaling_kernel, dim3((2 * L - 1 + 255) / 256, L), dim3(256), 0, st, flm, phi, wphi, L);
    return hipGetLastError();
}

// f_lm = fac_l sum_g Fpart[g][l][m] + sqrt((2l+1)/(4 pi)) W^Phi_lm Phi_l0   (Eq. 32, 41), m >= 0;
// f_{l,-m} = (-1)^m conj(f_lm).
__global__ void syn_final_kernel(const double2 *Fpart, int nblk, int group, int Lmax, const double *fac,
                                 const double2 *wphi, const double *phi, double2 *flm, int L, int Lp) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (m > l) return;
    double fr = 0.0, fi = 0.0;
    // no wavelet coefficient reaches l >= Lmax; blocks starting above l hold no term of row l
    const int gmax = (l < Lmax && m < Lmax) ? min(nblk - 1, l / group) : -1;
    for (int g = 0; g <= gmax; ++g) {
        const double2 v = Fpart[((size_t)g * L + l) * Lp + m];
        fr += v.x;
        fi += v.y;
    }
    fr *= fac[l];
    fi *= fac[l];
    if (wphi) {
        const double c = sqrt((2.0 * l + 1.0) / (4.0 * 3.14159265358979323846)) * phi[l];
        const double2 w = wphi[(size_t)l * l + l + m];
        fr += c * w.x;
        fi += c * w.y;
    }
    flm[(size_t)l * l + l + m] = make_double2(fr, fi);
    if (m > 0) {
        const double sg = (m & 1) ? -1.0 : 1.0;
        flm[(size_t)l * l + l - m] = make_double2(sg * fr, -sg * fi);
    }
}

hipError_t launch_syn_final(const double2 *Fpart, int nblk, int group, int Lmax, const double *fac,
                            const double2 *wphi, const double *phi, double2 *flm, int L, int Lp, hipStream_t st) {
    hipLaunchKernelGGL(syn_final_kernel, dim3((L + 255) / 256, L), dim3(256), 0, st, Fpart, nblk, group, Lmax, fac,
                       wphi, phi, flm, L, Lp);
    return hipGetLastError();
}

__global__ void zero_kernel(double2 *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

hipError_t launch_zero(double2 *p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace s2dw
