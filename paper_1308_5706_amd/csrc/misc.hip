// Small kernels of the wavelet library: input padding, scaling coefficients, and the
// final reduction of the synthesis.
#include "misc_k.h"

namespace s2dw {

// ---------------------------------------------------------------------------------- misc

// Batched small kernels: map = blockIdx.z; f_lm and W^Phi_lm of map i start at i L^2.
// fpad = g_l(m) f_lm, m <= l: the Wigner stage's rescaled recurrence takes the factor g here.
__global__ void pad_flm_kernel(const double2 *flm, const double *g, double2 *fpad, int L, int Lp, size_t s_fpad) {
    pad_flm_elem(flm, g, fpad, L, Lp, s_fpad, blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, blockIdx.z);
}

hipError_t launch_pad_flm(const double2 *flm, const double *g, double2 *fpad, int L, int Lp, size_t s_fpad, int maps,
                          hipStream_t st) {
    if (t_rec) return rec_job(pkind(PS_PAD, 0), (long long)((Lp + 255) / 256) * L, maps, 256, PadArgs{flm, g, fpad, L, Lp, s_fpad});
    hipLaunchKernelGGL(pad_flm_kernel, dim3((Lp + 255) / 256, L, maps), dim3(256), 0, st, flm, g, fpad, L, Lp,
                       s_fpad);
    return hipGetLastError();
}

// Complex (non-real) signals run through the real path as two real signals: complex map z of
// a batch becomes real maps 2z (the real part of f on the sphere) and 2z + 1 (the imaginary
// part), since Eq. 1 is linear in f.  Their coefficients, for 0 <= m <= l, are
//   a_lm = (f_lm + (-1)^m conj f_{l,-m}) / 2,   b_lm = (f_lm - (-1)^m conj f_{l,-m}) / (2i).
__global__ void pad_flm_complex_kernel(const double2 *flm, const double *g, double2 *fpad, int L, int Lp,
                                       size_t s_fpad) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (m >= Lp) return;
    flm += (size_t)blockIdx.z * L * L;
    double2 *pa = fpad + (size_t)(2 * blockIdx.z) * s_fpad + (size_t)l * Lp + m;
    double2 *pb = pa + s_fpad;
    if (m > l) {
        *pa = make_double2(0.0, 0.0);
        *pb = make_double2(0.0, 0.0);
        return;
    }
    const double2 f = flm[(size_t)l * l + l + m], fm = flm[(size_t)l * l + l - m];
    const double sg = (m & 1) ? -1.0 : 1.0;
    const double cr = sg * fm.x, ci = -sg * fm.y;  // (-1)^m conj f_{l,-m}
    const double c = 0.5 * g[(size_t)l * Lp + m];  // with the factor g_l(m) (see pad_flm_kernel)
    *pa = make_double2(c * (f.x + cr), c * (f.y + ci));
    *pb = make_double2(c * (f.y - ci), -c * (f.x - cr));
}

hipError_t launch_pad_flm_complex(const double2 *flm, const double *g, double2 *fpad, int L, int Lp, size_t s_fpad,
                                  int cmaps, hipStream_t st) {
    if (t_rec) return hipErrorNotSupported;
    hipLaunchKernelGGL(pad_flm_complex_kernel, dim3((Lp + 255) / 256, L, cmaps), dim3(256), 0, st, flm, g, fpad, L,
                       Lp, s_fpad);
    return hipGetLastError();
}

// Synthesis of complex signals: f_lm = a_lm + i b_lm + sqrt((2l+1)/(4 pi)) W^Phi_lm Phi_l0
// (Eq. 41) for all m, from the real-signal syntheses a (map 2z) and b (map 2z + 1) at
// fab + k s_fab (k = 2z, 2z + 1), each L^2 complex.
__global__ void merge_complex_kernel(const double2 *fab, size_t s_fab, const double2 *wphi, const double *phi,
                                     double2 *flm, int L) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (i > 2 * l) return;
    const size_t k = (size_t)l * l + i;
    const double2 a = fab[(size_t)(2 * blockIdx.z) * s_fab + k], b = fab[(size_t)(2 * blockIdx.z + 1) * s_fab + k];
    double re = a.x - b.y, im = a.y + b.x;
    if (wphi) {
        const double c = sqrt((2.0 * l + 1.0) / (4.0 * 3.14159265358979323846)) * phi[l];
        const double2 w = wphi[(size_t)blockIdx.z * L * L + k];
        re += c * w.x;
        im += c * w.y;
    }
    flm[(size_t)blockIdx.z * L * L + k] = make_double2(re, im);
}

hipError_t launch_merge_complex(const double2 *fab, size_t s_fab, const double2 *wphi, const double *phi,
                                double2 *flm, int L, int cmaps, hipStream_t st) {
    if (t_rec) return hipErrorNotSupported;
    hipLaunchKernelGGL(merge_complex_kernel, dim3((2 * L - 1 + 255) / 256, L, cmaps), dim3(256), 0, st, fab, s_fab,
                       wphi, phi, flm, L);
    return hipGetLastError();
}

// W^Phi_lm = sqrt(4 pi/(2l+1)) f_lm Phi_l0 (Eq. 31); Phi is real.
__global__ void scaling_kernel(const double2 *flm, const double *phi, double2 *wphi, int L) {
    scaling_elem(flm, phi, wphi, L, blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, blockIdx.z);
}

hipError_t launch_scaling(const double2 *flm, const double *phi, double2 *wphi, int L, int maps, hipStream_t st) {
    if (t_rec) return rec_job(pkind(PS_SCALING, 0), (long long)((2 * L - 1 + 255) / 256) * L, maps, 256, ScalingArgs{flm, phi, wphi, L});
    hipLaunchKernelGGL(scaling_kernel, dim3((2 * L - 1 + 255) / 256, L, maps), dim3(256), 0, st, flm, phi, wphi, L);
    return hipGetLastError();
}

// f_lm = fac_l g_l(m) sum_grp Fpart[grp][l][m] + sqrt((2l+1)/(4 pi)) W^Phi_lm Phi_l0   (Eq. 32,
// 41), m >= 0 (g_l(m): the factor the rescaled Wigner recurrence leaves out of the sums);
// f_{l,-m} = (-1)^m conj(f_lm).
// Fpart holds double2 (FP64 path) or float2 (mixed precision) partial sums; the final sum
// over the m' groups and the harmonic synthesis factor are applied in FP64.
template <class VC>
// Rows in decreasing l: a row sums about l/group partial rows, so the heaviest rows start first
// and the light ones fill in at the end.
__global__ void syn_final_kernel(const VC *Fpart, size_t s_F, int nblk, int group, int Lmax, const double *fac,
                                 const double *gsc, const double2 *wphi, const double *phi, double2 *flm, int L,
                                 int Lp) {
    syn_final_elem(Fpart, s_F, nblk, group, Lmax, fac, gsc, wphi, phi, flm, L, Lp, blockIdx.x * blockDim.x + threadIdx.x,
                   (int)gridDim.y - 1 - (int)blockIdx.y, blockIdx.z);
}

hipError_t launch_syn_final(const void *Fpart, size_t s_F, int f32, int nblk, int group, int Lmax, const double *fac,
                            const double *g, const double2 *wphi, const double *phi, double2 *flm, int L, int Lp,
                            int maps, hipStream_t st) {
    if (t_rec)
        return rec_job(pkind(PS_SYNF, f32), (long long)((L + 255) / 256) * L, maps, 256,
                       SynFinalArgs{Fpart, s_F, nblk, group, Lmax, L, Lp, fac, g, phi, wphi, flm});
    const dim3 grid((L + 255) / 256, L, maps);
    if (f32)
        hipLaunchKernelGGL(syn_final_kernel<float2>, grid, dim3(256), 0, st, (const float2 *)Fpart, s_F, nblk, group,
                           Lmax, fac, g, wphi, phi, flm, L, Lp);
    else
        hipLaunchKernelGGL(syn_final_kernel<double2>, grid, dim3(256), 0, st, (const double2 *)Fpart, s_F, nblk,
                           group, Lmax, fac, g, wphi, phi, flm, L, Lp);
    return hipGetLastError();
}

// Clears n 32-bit words (a kernel rather than a memset node, so the call can be captured).
__global__ void zero_kernel(uint32_t *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero_words(void *p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (t_rec) return rec_job(pkind(PS_ZERO, 0), (long long)blocks, 1, 256, ZeroArgs{(uint32_t *)p, n});
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)p, n);
    return hipGetLastError();
}

// FP32 copies of plan tables for the mixed-precision path (round to nearest).
__global__ void to_f32_kernel(const double *src, float *dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

hipError_t launch_to_f32(const double *src, float *dst, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}


// ------------------------------------------------------------------------------- steering

// Wavelet coefficients at arbitrary third Euler angles (steerability, Eq. 9-10).  The wavelets
// carry only the orders n with |n| < N and n = N - 1 (mod 2) (Eq. 11), so W as a function of
// gamma is a trigonometric polynomial with those frequencies, fixed exactly by its G grid
// samples gamma_g = g step (G = 2N - 1, step = 2 pi/G on the equiangular grid; G = N base
// orientations, step = pi/N, on the Driscoll-Healy grid):
//   W(alpha, beta, gamma) = sum_g z(gamma - gamma_g) W(alpha, beta, gamma_g),
//   z(delta) = (1/G) sum_{n carried} cos(n delta).
// Block: kSteerQ target angles for 256 x V consecutive (beta, alpha) points of one plane set
// (map = blockIdx.z, scale = blockIdx.y); blockIdx.x = tile * nqc + q-chunk.  The weights of
// the block's angles sit in LDS; each point of the G input planes is read once per q-chunk.
constexpr int kSteerQ = 8;
constexpr int kSteerG = 31;  // 2N - 1 for N <= 16

template <class E, int V>
struct SteerVec {
    typedef E type __attribute__((ext_vector_type(V)));
};

template <class E, int V>
__global__ __launch_bounds__(256) void steer_kernel(const E *W, const double *gam, E *out, int N, int G,
                                                    double step, int Q, int nqc, size_t P, size_t s_in, size_t s_out) {
    typedef typename SteerVec<E, V>::type vec;
    __shared__ E zw[kSteerQ][kSteerG];
    const int qc = blockIdx.x % nqc;
    const size_t tile = blockIdx.x / nqc;
    const int q0 = qc * kSteerQ;
    const int qn = min(kSteerQ, Q - q0);
    for (int t = threadIdx.x; t < qn * G; t += blockDim.x) {
        const int q = t / G, g = t - q * G;
        const double d = gam[q0 + q] - step * (double)g;
        double z = 0.0;
        for (int n = -(N - 1); n <= N - 1; n += 2) z += cos((double)n * d);
        zw[q][g] = (E)(z / (double)G);
    }
    __syncthreads();
    const size_t i0 = (tile * blockDim.x + threadIdx.x) * V;
    if (i0 >= P) return;
    const E *src = W + blockIdx.z * s_in + (size_t)blockIdx.y * G * P + i0;
    E *dst = out + blockIdx.z * s_out + ((size_t)blockIdx.y * Q + q0) * P + i0;
    vec acc[kSteerQ];
#pragma unroll
    for (int q = 0; q < kSteerQ; ++q) acc[q] = (vec)(E)0;
    for (int g = 0; g < G; ++g) {
        const vec w = __builtin_nontemporal_load((const vec *)(src + (size_t)g * P));
#pragma unroll
        for (int q = 0; q < kSteerQ; ++q) acc[q] += zw[q][g] * w;
    }
#pragma unroll
    for (int q = 0; q < kSteerQ; ++q)
        if (q < qn) *(vec *)(dst + (size_t)q * P) = acc[q];
}

template <class E, int V>
void steer_launch(const void *W, const double *gam, void *out, int N, int G, double step, int Q, int S, size_t P,
                  size_t s_in, size_t s_out, int maps, hipStream_t st) {
    const int nqc = (Q + kSteerQ - 1) / kSteerQ;
    const size_t tiles = (P + 256 * V - 1) / (256 * V);
    hipLaunchKernelGGL((steer_kernel<E, V>), dim3((unsigned)(tiles * nqc), S, maps), dim3(256), 0, st, (const E *)W,
                       gam, (E *)out, N, G, step, Q, nqc, P, s_in, s_out);
}

hipError_t launch_steer(const void *W, const double *gam, void *out, int f32, int N, int G, double step, int Q,
                        int S, size_t P, size_t s_in, size_t s_out, int maps, hipStream_t st) {
    if (t_rec) return hipErrorNotSupported;
    // vector width: the plane size, the map strides and both base addresses are multiples of it
    const size_t es = f32 ? 4 : 8;
    auto fits = [&](int V) {
        return P % V == 0 && s_in % V == 0 && s_out % V == 0 && ((uintptr_t)W | (uintptr_t)out) % (V * es) == 0;
    };
    if (f32) {
        if (fits(4)) steer_launch<float, 4>(W, gam, out, N, G, step, Q, S, P, s_in, s_out, maps, st);
        else if (fits(2)) steer_launch<float, 2>(W, gam, out, N, G, step, Q, S, P, s_in, s_out, maps, st);
        else steer_launch<float, 1>(W, gam, out, N, G, step, Q, S, P, s_in, s_out, maps, st);
    } else {
        if (fits(2)) steer_launch<double, 2>(W, gam, out, N, G, step, Q, S, P, s_in, s_out, maps, st);
        else steer_launch<double, 1>(W, gam, out, N, G, step, Q, S, P, s_in, s_out, maps, st);
    }
    return hipGetLastError();
}

}  // namespace s2dw
