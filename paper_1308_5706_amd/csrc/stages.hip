// Launchers of the separation-of-variables stage kernels (stages_k.h): template dispatch
// over the transform size and the complex type, grids per stage.
#include "stages_k.h"

namespace s2dw {

// ------------------------------------------------------------------------------ launchers

#define S2DW_P_CASE(C, KER, PV, GRID, ARGS) \
    case PV: hipLaunchKernelGGL((KER<C, PV>), dim3(GRID, maps), dim3(PV / kRM), 0, st, ARGS); break;

#define S2DW_P_SWITCH_T(C, P, KER, GRID, ARGS)           \
    switch (P) {                                          \
        S2DW_P_CASE(C, KER, 32, GRID, ARGS)               \
        S2DW_P_CASE(C, KER, 64, GRID, ARGS)               \
        S2DW_P_CASE(C, KER, 128, GRID, ARGS)              \
        S2DW_P_CASE(C, KER, 256, GRID, ARGS)              \
        S2DW_P_CASE(C, KER, 512, GRID, ARGS)              \
        S2DW_P_CASE(C, KER, 1024, GRID, ARGS)             \
        S2DW_P_CASE(C, KER, 2048, GRID, ARGS)             \
        S2DW_P_CASE(C, KER, 4096, GRID, ARGS)             \
        S2DW_P_CASE(C, KER, 8192, GRID, ARGS)             \
        default: return hipErrorInvalidValue;             \
    }

#define S2DW_P_SWITCH(P, KER, GRID, ARGS)                                   \
    if (ARGS.f32) {                                                         \
        S2DW_P_SWITCH_T(float2, P, KER, GRID, ARGS)                          \
    } else {                                                                \
        S2DW_P_SWITCH_T(double2, P, KER, GRID, ARGS)                         \
    }

hipError_t launch_beta_fwd_fft(const StageArgs &a, int P, int maps, hipStream_t st) {
    if (t_rec) return rec_fft(PS_BETAF_FFT, a, a.f32, P, (long long)a.N * a.Lj, maps);
    S2DW_P_SWITCH(P, beta_fwd_fft_kernel, a.N * a.Lj, a)
    return hipGetLastError();
}

hipError_t launch_beta_fwd_pair(const StageArgs &a, int P, int maps, hipStream_t st) {
    if (t_rec) return rec_fft(PS_BETAF_PAIR, a, a.f32, P, (long long)a.N * ((a.Lj + 1) / 2), maps);
    S2DW_P_SWITCH(P, beta_fwd_pair_kernel, a.N * ((a.Lj + 1) / 2), a)
    return hipGetLastError();
}

hipError_t launch_alpha_fwd_fft(const StageArgs &a, int P, int maps, hipStream_t st) {
    if (t_rec) return rec_fft(PS_ALPHAF_FFT, a, a.f32, P, (long long)a.Nh * a.nb, maps);
    S2DW_P_SWITCH(P, alpha_fwd_fft_kernel, 8 * ((a.Nh * a.nb + 7) / 8), a)
    return hipGetLastError();
}

hipError_t launch_alpha_adj_fft(const StageArgs &a, int P, int maps, hipStream_t st) {
    if (t_rec) return rec_fft(PS_ALPHAA_FFT, a, a.f32, P, (long long)a.Nh * a.nb, maps);
    S2DW_P_SWITCH(P, alpha_adj_fft_kernel, 8 * ((a.Nh * a.nb + 7) / 8), a)
    return hipGetLastError();
}

bool pfa_length(int T) { return T == 2047 || T == 4095; }

// T = 2L - 1 in {2047, 4095}.  T = 4095 on eight-wave workgroups: the LDS of a column allows
// two workgroups per CU, so the wider form doubles the waves (measured at L = 2048, N = 4:
// the fused analysis alpha/gamma pass 1.76 -> 1.47 ms, the fused synthesis one 1.48 -> 1.37
// ms per step); T = 2047 keeps four waves (its alpha kernels ran 7 % slower with eight).
#define S2DW_PFA_LAUNCH(KER)                                                                         \
    {                                                                                                \
        if (t_rec) return hipErrorNotSupported;                                                      \
        const int T = 2 * a.L - 1;                                                                   \
        if (T != 2047 && T != 4095) return hipErrorInvalidValue;                                     \
        const int NC = T == 2047 ? pfa::Len2047::NC : pfa::Len4095::NC;                              \
        const int nwg = (a.Nh * a.nb + NC - 1) / NC;                                                 \
        const dim3 grid((unsigned)(8 * ((nwg + 7) / 8)), (unsigned)maps);                            \
        if (T == 2047) {                                                                             \
            if (a.f32) hipLaunchKernelGGL((KER<float2, pfa::Len2047>), grid, dim3(pfa::Len2047::NTH), 0, st, a); \
            else hipLaunchKernelGGL((KER<double2, pfa::Len2047>), grid, dim3(pfa::Len2047::NTH), 0, st, a); \
        } else {                                                                                     \
            if (a.f32) hipLaunchKernelGGL((KER<float2, pfa::Len4095T<512>>), grid, dim3(512), 0, st, a); \
            else hipLaunchKernelGGL((KER<double2, pfa::Len4095T<512>>), grid, dim3(512), 0, st, a); \
        }                                                                                            \
        return hipGetLastError();                                                                    \
    }

hipError_t launch_alpha_fwd_pfa(const StageArgs &a, int maps, hipStream_t st) S2DW_PFA_LAUNCH(alpha_fwd_pfa_kernel)

hipError_t launch_beta_fwd_pfa(const StageArgs &a, int maps, hipStream_t st) {
    if (t_rec) return hipErrorNotSupported;
    const int T = 2 * a.L - 1;
    if (T != 2047 && T != 4095) return hipErrorInvalidValue;
    const int NC = T == 2047 ? pfa::Len2047::NC : pfa::Len4095::NC;
    const dim3 grid((unsigned)((a.N * ((a.Lj + 1) / 2) + NC - 1) / NC), (unsigned)maps);
    // eight-wave workgroups at both lengths (measured: 0.58 -> 0.50 ms per step for the stage
    // at L = 1024, N = 8; 0.76 -> 0.61 ms at L = 2048, N = 4)
    if (T == 2047) {
        if (a.f32) hipLaunchKernelGGL((beta_fwd_pfa_kernel<float2, pfa::Len2047W>), grid, dim3(pfa::Len2047W::NTH), 0, st, a);
        else hipLaunchKernelGGL((beta_fwd_pfa_kernel<double2, pfa::Len2047W>), grid, dim3(pfa::Len2047W::NTH), 0, st, a);
    } else {
        using LW = pfa::Len4095T<512>;
        if (a.f32) hipLaunchKernelGGL((beta_fwd_pfa_kernel<float2, LW>), grid, dim3(LW::NTH), 0, st, a);
        else hipLaunchKernelGGL((beta_fwd_pfa_kernel<double2, LW>), grid, dim3(LW::NTH), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_beta_fwd_pfa_multi(const StageArgs &a, const BetaAdjScale *tab, int ns, int nwg, int maps,
                                     hipStream_t st) {
    if (t_rec) return hipErrorNotSupported;
    const int T = 2 * a.L - 1;
    if ((T != 2047 && T != 4095) || ns < 1 || nwg < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nwg, (unsigned)maps);
    if (T == 2047) {
        using LW = pfa::Len2047W;
        if (a.f32) hipLaunchKernelGGL((beta_fwd_pfa_multi_kernel<float2, LW>), grid, dim3(LW::NTH), 0, st, a, tab, ns);
        else hipLaunchKernelGGL((beta_fwd_pfa_multi_kernel<double2, LW>), grid, dim3(LW::NTH), 0, st, a, tab, ns);
    } else {
        using LW = pfa::Len4095T<512>;
        if (a.f32) hipLaunchKernelGGL((beta_fwd_pfa_multi_kernel<float2, LW>), grid, dim3(LW::NTH), 0, st, a, tab, ns);
        else hipLaunchKernelGGL((beta_fwd_pfa_multi_kernel<double2, LW>), grid, dim3(LW::NTH), 0, st, a, tab, ns);
    }
    return hipGetLastError();
}

hipError_t launch_alpha_adj_pfa(const StageArgs &a, int maps, hipStream_t st) S2DW_PFA_LAUNCH(alpha_adj_pfa_kernel)

// Orders n >= 0 whose transforms can wait in registers: at most 16 complex values per thread.
bool pfa_fused(int T, int Nh) {
    if (T == 2047) return Nh >= 1 && Nh <= 4;  // two orders per pass, 8 samples per thread
    if (T == 4095) return Nh >= 1 && Nh <= 2;  // one order per pass, 8 samples per thread (512)
    return false;
}

#define S2DW_FUSED_CASE(KER, LN, NH)                                                                     \
    case NH:                                                                                             \
        if (a.f32) hipLaunchKernelGGL((KER<float2, LN, NH>), grid, dim3(LN::NTH), 0, st, a);             \
        else hipLaunchKernelGGL((KER<double2, LN, NH>), grid, dim3(LN::NTH), 0, st, a);                  \
        break;

#define S2DW_FUSED_LAUNCH(KER)                                                                           \
    {                                                                                                    \
        if (t_rec) return hipErrorNotSupported;                                                          \
        const int T = 2 * a.L - 1;                                                                       \
        if (!pfa_fused(T, a.Nh) || a.G < 1 || a.nb < 1) return hipErrorInvalidValue;                     \
        const dim3 grid((unsigned)(8 * ((a.nb + 7) / 8)), (unsigned)maps);                               \
        if (T == 2047) {                                                                                 \
            switch (a.Nh) {                                                                              \
                S2DW_FUSED_CASE(KER, pfa::Len2047, 1)                                                    \
                S2DW_FUSED_CASE(KER, pfa::Len2047, 2)                                                    \
                S2DW_FUSED_CASE(KER, pfa::Len2047, 3)                                                    \
                S2DW_FUSED_CASE(KER, pfa::Len2047, 4)                                                    \
                default: return hipErrorInvalidValue;                                                    \
            }                                                                                            \
        } else {                                                                                         \
            switch (a.Nh) {                                                                              \
                S2DW_FUSED_CASE(KER, pfa::Len4095T<512>, 1)                                          \
                S2DW_FUSED_CASE(KER, pfa::Len4095T<512>, 2)                                          \
                default: return hipErrorInvalidValue;                                                    \
            }                                                                                            \
        }                                                                                                \
        return hipGetLastError();                                                                        \
    }

hipError_t launch_alpha_gamma_fwd_pfa(const StageArgs &a, int maps, hipStream_t st) S2DW_FUSED_LAUNCH(alpha_gamma_fwd_pfa_kernel)

hipError_t launch_gamma_alpha_adj_pfa(const StageArgs &a, int maps, hipStream_t st) S2DW_FUSED_LAUNCH(gamma_alpha_adj_pfa_kernel)

hipError_t launch_alpha_fwd_blk(const StageArgs &a, int P, int maps, hipStream_t st) {
    if (t_rec) return rec_fft(PS_ALPHAF_BLK, a, a.f32, P, (long long)a.Nh * a.nb, maps);
    S2DW_P_SWITCH(P, alpha_fwd_blk_kernel, 8 * ((a.Nh * a.nb + 7) / 8), a)
    return hipGetLastError();
}

hipError_t launch_alpha_adj_blk(const StageArgs &a, int P, int maps, hipStream_t st) {
    if (t_rec) return rec_fft(PS_ALPHAA_BLK, a, a.f32, P, (long long)a.Nh * a.nb, maps);
    S2DW_P_SWITCH(P, alpha_adj_blk_kernel, 8 * ((a.Nh * a.nb + 7) / 8), a)
    return hipGetLastError();
}

hipError_t launch_beta_adj_fft(const StageArgs &a, int P, int maps, hipStream_t st) {
    if (t_rec) return rec_fft(PS_BETAA_FFT, a, a.f32, P, (long long)a.K * ((a.Lj + 1) / 2), maps);
    if (P == 8192 && a.pcs) {  // T = 4095
        const dim3 grid((unsigned)(a.K * ((a.Lj + 1) / 2)), (unsigned)maps);
        if (a.f32) hipLaunchKernelGGL((beta_adj_fft_kernel<float2, 8192, true>), grid, dim3(8192 / kRM), 0, st, a);
        else hipLaunchKernelGGL((beta_adj_fft_kernel<double2, 8192, true>), grid, dim3(8192 / kRM), 0, st, a);
        return hipGetLastError();
    }
    S2DW_P_SWITCH(P, beta_adj_fft_kernel, a.K * ((a.Lj + 1) / 2), a)
    return hipGetLastError();
}

hipError_t launch_beta_adj_multi(const StageArgs &a, const BetaAdjScale *tab, int ns, int nwg, int P, int maps,
                                 hipStream_t st) {
    if (t_rec) return rec_fft(PS_BETAA_MULTI, BetaMultiArgs{a, tab, ns}, a.f32, P, nwg, maps);
#define S2DW_MULTI_CASE(C, PV)                                                                                \
    case PV:                                                                                                  \
        hipLaunchKernelGGL((beta_adj_multi_kernel<C, PV>), dim3(nwg, maps), dim3(PV / kRM), 0, st, a, tab, ns); \
        break;
#define S2DW_MULTI_SWITCH(C)                                                                    \
    switch (P) {                                                                                \
        S2DW_MULTI_CASE(C, 32) S2DW_MULTI_CASE(C, 64) S2DW_MULTI_CASE(C, 128)                    \
        S2DW_MULTI_CASE(C, 256) S2DW_MULTI_CASE(C, 512) S2DW_MULTI_CASE(C, 1024)                 \
        S2DW_MULTI_CASE(C, 2048) S2DW_MULTI_CASE(C, 4096) S2DW_MULTI_CASE(C, 8192)               \
        default: return hipErrorInvalidValue;                                                   \
    }
    if (P == 8192 && a.pcs) {  // T = 4095
        if (a.f32)
            hipLaunchKernelGGL((beta_adj_multi_kernel<float2, 8192, true>), dim3(nwg, maps), dim3(8192 / kRM), 0, st, a,
                               tab, ns);
        else
            hipLaunchKernelGGL((beta_adj_multi_kernel<double2, 8192, true>), dim3(nwg, maps), dim3(8192 / kRM), 0, st,
                               a, tab, ns);
    } else if (a.f32) {
        S2DW_MULTI_SWITCH(float2)
    } else {
        S2DW_MULTI_SWITCH(double2)
    }
#undef S2DW_MULTI_SWITCH
#undef S2DW_MULTI_CASE
    return hipGetLastError();
}

hipError_t launch_beta_adj_dh(const StageArgs &a, int P, int maps, hipStream_t st) {
    if (t_rec) return hipErrorNotSupported;
    S2DW_P_SWITCH(P, beta_adj_dh_kernel, a.K * a.Lj, a)
    return hipGetLastError();
}

#define S2DW_GAMMA_LAUNCH(KER, STAGE)                                                           \
    {                                                                                           \
        const size_t plane = (size_t)a.L * a.T;                                                 \
        if (t_rec) {                                                                            \
            const int V = plane % 2 == 0 ? 2 : 1;                                               \
            return rec_job(pkind(STAGE, a.f32, V), (long long)((plane / V + 255) / 256), maps, 256, a); \
        }                                                                                       \
        if (plane % 2 == 0) {                                                                   \
            const dim3 grid((unsigned)((plane / 2 + 255) / 256), maps);                               \
            if (a.f32) hipLaunchKernelGGL((KER<float2, 2>), grid, dim3(256), 0, st, a);         \
            else hipLaunchKernelGGL((KER<double2, 2>), grid, dim3(256), 0, st, a);              \
        } else {                                                                                \
            const dim3 grid((unsigned)((plane + 255) / 256), maps);                                   \
            if (a.f32) hipLaunchKernelGGL((KER<float2, 1>), grid, dim3(256), 0, st, a);         \
            else hipLaunchKernelGGL((KER<double2, 1>), grid, dim3(256), 0, st, a);              \
        }                                                                                       \
        return hipGetLastError();                                                               \
    }

hipError_t launch_gamma_fwd(const GammaArgs &a, int maps, hipStream_t st) S2DW_GAMMA_LAUNCH(gamma_fwd_kernel, PS_GAMMAF)

hipError_t launch_gamma_adj(const GammaArgs &a, int maps, hipStream_t st) S2DW_GAMMA_LAUNCH(gamma_adj_kernel, PS_GAMMAA)

hipError_t launch_gamma_alpha_adj(const GammaAlphaArgs &a, int maps, hipStream_t st) {
    if (a.Nh < 1 || a.Nh > kMaxK || a.Lj < 1 || a.Nh * (2 * a.Lj - 1) > 256 || a.T < 1 || a.nb < 1 || a.G < 1 ||
        a.G > 4 * a.Nh - 1 || maps < 1)
        return hipErrorInvalidValue;
    if (t_rec) return rec_job(pkind(PS_GAA, a.f32, a.Nh), a.nb, maps, 256, a);
    const dim3 grid((unsigned)a.nb, (unsigned)maps);
    switch (a.Nh * 2 + (a.f32 ? 1 : 0)) {
#define S2DW_GA_CASE(NH)                                                                                    \
    case 2 * NH: hipLaunchKernelGGL((gamma_alpha_adj_kernel<NH, double2>), grid, dim3(256), 0, st, a); break; \
    case 2 * NH + 1: hipLaunchKernelGGL((gamma_alpha_adj_kernel<NH, float2>), grid, dim3(256), 0, st, a); break;
        S2DW_GA_CASE(1)
        S2DW_GA_CASE(2)
        S2DW_GA_CASE(3)
        S2DW_GA_CASE(4)
        S2DW_GA_CASE(5)
        S2DW_GA_CASE(6)
        S2DW_GA_CASE(7)
        S2DW_GA_CASE(8)
#undef S2DW_GA_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_alpha_gamma_fwd(const AlphaGammaArgs &a, int maps, hipStream_t st) {
    if (a.Nh < 1 || a.Nh > kMaxK || a.Lj < 1 || 2 * a.Nh * a.Lj > kAlphaGammaCoeffs || a.T < 1 || a.nb < 1 || maps < 1)
        return hipErrorInvalidValue;
    const size_t plane = (size_t)a.nb * a.T;
    const size_t pair_bytes = a.f32 ? 8 : 16;
    const bool pair = a.T % 2 == 1 && plane % 2 == 0 && (maps == 1 || a.s_w % 2 == 0) &&
                      ((uintptr_t)a.wout % pair_bytes) == 0;
    const dim3 grid((unsigned)(((pair ? a.T / 2 + 1 : a.T) + 255) / 256), (unsigned)a.nb, (unsigned)maps);
    if (t_rec) return rec_job(pkind(PS_AGF, a.f32, a.Nh, pair ? 1 : 0), (long long)grid.x * a.nb, maps, 256, a);
    switch (a.Nh * 4 + (pair ? 2 : 0) + (a.f32 ? 1 : 0)) {
#define S2DW_AG_CASE(NH)                                                                               \
    case 4 * NH: hipLaunchKernelGGL((alpha_gamma_fwd_kernel<false, NH, double2>), grid, dim3(256), 0, st, a); break; \
    case 4 * NH + 1: hipLaunchKernelGGL((alpha_gamma_fwd_kernel<false, NH, float2>), grid, dim3(256), 0, st, a); break; \
    case 4 * NH + 2: hipLaunchKernelGGL((alpha_gamma_fwd_kernel<true, NH, double2>), grid, dim3(256), 0, st, a); break; \
    case 4 * NH + 3: hipLaunchKernelGGL((alpha_gamma_fwd_kernel<true, NH, float2>), grid, dim3(256), 0, st, a); break;
        S2DW_AG_CASE(1)
        S2DW_AG_CASE(2)
        S2DW_AG_CASE(3)
        S2DW_AG_CASE(4)
        S2DW_AG_CASE(5)
        S2DW_AG_CASE(6)
        S2DW_AG_CASE(7)
        S2DW_AG_CASE(8)
#undef S2DW_AG_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define S2DW_GAMMA_CX_LAUNCH(KER)                                                                 \
    {                                                                                             \
        if (t_rec) return hipErrorNotSupported;                                                   \
        const size_t plane = (size_t)a.L * a.T;                                                   \
        const dim3 grid((unsigned)((plane + 255) / 256), cmaps);                                  \
        if (a.f32) hipLaunchKernelGGL((KER<float2>), grid, dim3(256), 0, st, a);                  \
        else hipLaunchKernelGGL((KER<double2>), grid, dim3(256), 0, st, a);                       \
        return hipGetLastError();                                                                 \
    }

hipError_t launch_gamma_fwd_cx(const GammaArgs &a, int cmaps, hipStream_t st) S2DW_GAMMA_CX_LAUNCH(gamma_fwd_cx_kernel)

hipError_t launch_gamma_adj_cx(const GammaArgs &a, int cmaps, hipStream_t st) S2DW_GAMMA_CX_LAUNCH(gamma_adj_cx_kernel)

}  // namespace s2dw
