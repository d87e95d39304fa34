// Launchers of the Wigner-stage kernels (wigner_k.h) and the tile-shape options.
#include "wigner_k.h"

namespace s2dw {

// ------------------------------------------------------------------------------ launchers

template <int K, int R>
static hipError_t launch_fwd_k(const WigFwdArgs &a, int ntiles, int maps, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((wig_fwd_kernel<K, R>), dim3(ntiles, maps), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int K, int R>
static hipError_t launch_adj_k(const WigAdjArgs &a, int ntiles, int maps, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (a.f32) hipLaunchKernelGGL((wig_adj_kernel<K, R, float>), dim3(ntiles, maps), dim3(kAdjThreads), 0, st, a);
    else hipLaunchKernelGGL((wig_adj_kernel<K, R, double>), dim3(ntiles, maps), dim3(kAdjThreads), 0, st, a);
    return hipGetLastError();
}

// m' slots per wave: the accumulators take 16 R K registers, kept at or below 128
int wig_slots(int K) { return K >= 5 ? 1 : (K >= 2 ? 2 : 4); }

// Slot counts compiled for each number of carried orders K (the tile shapes the tuner may pick).
int wig_slot_options(int K, int *R) {
    if (K <= 1) {
        R[0] = 1, R[1] = 2, R[2] = 4;
        return 3;
    }
    if (K <= 4) {
        R[0] = 1, R[1] = 2;
        return 2;
    }
    R[0] = 1;
    return 1;
}

#define S2DW_WIG_SWITCH(FN)                                          \
    switch (K * 8 + R) {                                             \
        case 1 * 8 + 1: return FN<1, 1>(a, ntiles, maps, st);        \
        case 1 * 8 + 2: return FN<1, 2>(a, ntiles, maps, st);        \
        case 1 * 8 + 4: return FN<1, 4>(a, ntiles, maps, st);        \
        case 2 * 8 + 1: return FN<2, 1>(a, ntiles, maps, st);        \
        case 2 * 8 + 2: return FN<2, 2>(a, ntiles, maps, st);        \
        case 3 * 8 + 1: return FN<3, 1>(a, ntiles, maps, st);        \
        case 3 * 8 + 2: return FN<3, 2>(a, ntiles, maps, st);        \
        case 4 * 8 + 1: return FN<4, 1>(a, ntiles, maps, st);        \
        case 4 * 8 + 2: return FN<4, 2>(a, ntiles, maps, st);        \
        case 5 * 8 + 1: return FN<5, 1>(a, ntiles, maps, st);        \
        case 6 * 8 + 1: return FN<6, 1>(a, ntiles, maps, st);        \
        case 7 * 8 + 1: return FN<7, 1>(a, ntiles, maps, st);        \
        case 8 * 8 + 1: return FN<8, 1>(a, ntiles, maps, st);        \
        default: return hipErrorInvalidValue;                        \
    }

hipError_t launch_wig_fwd(const WigFwdArgs &a, int K, int R, int ntiles, int maps, hipStream_t st) {
    if (t_rec) return K <= 4 ? rec_job(pkind(PS_WIGF, 0, K, R), ntiles, maps, 256, a) : hipErrorNotSupported;
    S2DW_WIG_SWITCH(launch_fwd_k)
}

hipError_t launch_wig_adj(const WigAdjArgs &a, int K, int R, int ntiles, int maps, hipStream_t st) {
    if (t_rec) return K <= 4 ? rec_job(pkind(PS_WIGA, a.f32, K, R), ntiles, maps, 256, a) : hipErrorNotSupported;
    S2DW_WIG_SWITCH(launch_adj_k)
}

}  // namespace s2dw
