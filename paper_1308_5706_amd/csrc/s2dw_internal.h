// Internal declarations shared by the host side and the HIP kernels of the
// directional scale-discretized wavelet library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace s2dw {

constexpr int kMaxScales = 24;
constexpr int kMaxSegs = 64;
constexpr int kMaxK = 8;  // nonnegative n carried by the wavelets: ceil(N/2), N <= 16
constexpr int kMaxSteerAngles = 1 << 16;  // angles per steering call

// l-segments on which the set of active wavelet scales is constant.  At most one
// even and one odd scale is active on any l (supports of kappa^j and kappa^{j+2} are
// disjoint, Eq. 15), so a segment names the active scale of each parity slot.
struct SegTab {
    int n;
    int s0[kMaxSegs], s1[kMaxSegs];  // [s0, s1)
    int8_t je[kMaxSegs], jo[kMaxSegs];  // active even / odd scale, -1 if none
};

// Per-scale layout of the Wigner-stage workspaces.  Scale j has band-limit Lj (its
// kernel vanishes for l >= Lj); its arrays live on m, m' < Lj.
struct ScaleTab {
    int S;
    int Lj[kMaxScales];
    int64_t off[kMaxScales];   // offset of scale j in the U / V workspace (double2 units)
    int64_t boff[kMaxScales];  // offset of scale j in the beta-stage workspace (double2 units)
};

// Host-side harmonic tables of one parameter set (Sec. 2.2).
struct HostTables {
    int L = 0, N = 0, S = 0, K = 0;
    bool eta_imag = false;             // eta_N = i for even N (Eq. 11)
    std::vector<int> nk;               // nonnegative n with beta_(N,n) = 1, increasing
    std::vector<double> kappa;         // [S][L]  kappa^j(l)              (Eq. 15)
    std::vector<double> phi;           // [L]     Phi_l0                 (Eq. 16)
    std::vector<double> sig;           // [L][K]  |s_{l,n_k}|            (Eq. 11)
    std::vector<int> lo, hi;           // per scale: first / last l with kappa^j(l) > 0
};

// Builds kappa^j, Phi, s_ln for (L, N, lambda, J_min).  Returns false on bad input.
bool build_wavelet_tables(int L, int N, double lambda, int J_min, HostTables &t);
// Number of scales J_L(lambda) - J_min + 1; J_L(lambda) = ceil(log_lambda L).
int jmax_of(int L, double lambda);

// Delta = d(pi/2) recursion tables (see plan.cpp for the formulas).
struct DeltaTables {
    int L = 0, Lp = 0;
    std::vector<double> pq;      // [L][Lp][2]   per-column factors p_l(x), q_l(x)
    std::vector<double> uv;      // [Lp][L][2]   per-row factors u_l(x), v_l(x)
    std::vector<double> seed;    // [Lp][Lp]     Delta^{max(m',m)}_{m'm} (0 where it underflows)
    // The same recurrence for the rescaled values D_l = Delta^l_{m'm} / (g_l(m) h_l(m')),
    // with g_{l+1}(x) = q_l(x) g_{l-1}(x) from g_x = g_{x+1} = 1 and h_{l+1}(x) = v_l(x)
    // h_{l-1}(x) from h_x = h_{x+1} = 1: the Delta^{l-1} coefficient becomes 1,
    //   D_{l+1} = -(ut_l(m') pt_l(m)) D_l - D_{l-1},
    //   pt_l(x) = p_l(x) g_l(x)/g_{l+1}(x),  ut_l(x) = u_l(x) h_l(x)/h_{l+1}(x).
    std::vector<double> pt;      // [L][Lp]      pt_l(x)
    std::vector<double> ut;      // [Lp][L]      ut_l(x)
    std::vector<double> g;       // [L][Lp]      g_l(x), x <= l (0 elsewhere)
    std::vector<double> h;       // [Lp][L]      h_l(x), x <= l (0 elsewhere)
    std::vector<double> seedt;   // [Lp][Lp]     D at l0 = max(m',m) (0 where it underflows)
    std::vector<double> seedtm;  // [Lp][Lp]     its mantissa in [0.5, 1) with sign
    std::vector<int> seedte;     // [Lp][Lp]     its binary exponent
};
void build_delta_tables(int L, DeltaTables &d);

// Column table Delta^l_{m' n} for the K nonnegative wavelet n values, [Lp][L][K].
void build_delta_ncols(const DeltaTables &d, const std::vector<int> &nk, std::vector<double> &out);

}  // namespace s2dw
