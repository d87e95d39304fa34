// Element functions of the small kernels (misc.hip): input padding, scaling coefficients and
// the final reduction of the synthesis, shared by the kernels and the persistent executor.
#pragma once

#include "kernels.h"

namespace s2dw {

// fpad = g_l(m) f_lm for m <= l (zero for l < m < Lp): the Wigner stage's rescaled recurrence
// takes the factor g here.  Element (m, l) of map z; f_lm of map z starts at z L^2.
__device__ __forceinline__ void pad_flm_elem(const double2 *flm, const double *g, double2 *fpad, int L, int Lp,
                                             size_t s_fpad, int m, int l, int z) {
    if (m >= Lp) return;
    flm += (size_t)z * L * L;
    fpad += (size_t)z * s_fpad;
    double2 v = make_double2(0.0, 0.0);
    if (m <= l) {
        const double2 f = flm[(size_t)l * l + l + m];
        const double c = g[(size_t)l * Lp + m];
        v = make_double2(c * f.x, c * f.y);
    }
    fpad[(size_t)l * Lp + m] = v;
}

// W^Phi_lm = sqrt(4 pi/(2l+1)) f_lm Phi_l0 (Eq. 31); Phi is real.  Element l^2 + m of map z.
__device__ __forceinline__ void scaling_elem(const double2 *flm, const double *phi, double2 *wphi, int L, int m, int l,
                                             int z) {
    if (m > 2 * l) return;
    const size_t i = (size_t)z * L * L + (size_t)l * l + m;
    const double c = sqrt(4.0 * 3.14159265358979323846 / (2.0 * l + 1.0)) * phi[l];
    const double2 f = flm[i];
    wphi[i] = make_double2(c * f.x, c * f.y);
}

// f_lm = fac_l g_l(m) sum_grp Fpart[grp][l][m] + sqrt((2l+1)/(4 pi)) W^Phi_lm Phi_l0   (Eq. 32,
// 41), m >= 0 (g_l(m): the factor the rescaled Wigner recurrence leaves out of the sums);
// f_{l,-m} = (-1)^m conj(f_lm).
// Fpart holds double2 (FP64 path) or float2 (mixed precision) partial sums; the final sum
// over the m' groups and the harmonic synthesis factor are applied in FP64.
template <class VC>
__device__ __forceinline__ void syn_final_elem(const VC *Fpart, size_t s_F, int nblk, int group, int Lmax,
                                               const double *fac, const double *gsc, const double2 *wphi,
                                               const double *phi, double2 *flm, int L, int Lp, int m, int l, int z) {
    if (m > l) return;
    Fpart += (size_t)z * s_F;
    flm += (size_t)z * L * L;
    if (wphi) wphi += (size_t)z * L * L;
    double fr = 0.0, fi = 0.0;
    // no wavelet coefficient reaches l >= Lmax; blocks starting above l hold no term of row l
    const int gmax = (l < Lmax && m < Lmax) ? min(nblk - 1, l / group) : -1;
    for (int g = 0; g <= gmax; ++g) {
        const VC v = Fpart[((size_t)g * L + l) * Lp + m];
        fr += (double)v.x;
        fi += (double)v.y;
    }
    const double cg = fac[l] * gsc[(size_t)l * Lp + m];
    fr *= cg;
    fi *= cg;
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

}  // namespace s2dw
