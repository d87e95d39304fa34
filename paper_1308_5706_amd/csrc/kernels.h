// Kernel argument blocks and launchers of the wavelet library (device side).
#pragma once

#include "s2dw_internal.h"

#include <cstring>

namespace s2dw {

constexpr int kAdjWaves = 8;                 // waves per synthesis Wigner workgroup
constexpr int kAdjThreads = kAdjWaves * 64;

struct WigFwdArgs {
    // The l-recurrence runs on D_l = Delta^l_{m'm} / (g_l(m) h_l(m')) (rescaled so that its
    // Delta^{l-1} coefficient is 1: D_{l+1} = -(ut_l(m') pt_l(m)) D_l - D_{l-1}); g goes with
    // f_lm and h with the kb2 table.
    const double2 *fpad;   // [L][Lp]   g_l(m) f_lm for m <= l (0 elsewhere)
    const double *pq;      // [L][Lp]   pt_l(m)
    const double *uv;      // [Lp][L]   ut_l(m')
    const double *kb2;     // [Lp][L][2][K]  kappa^{j(slot,l)}(l) sigma_{l,n_k} Delta^l_{m' n_k} h_l(m')
    const double *seed;    // [Lp][Lp]  D at l0 = max(m',m)
    const double *seedm;   // [Lp][Lp]  its mantissa (extended-exponent variant)
    const int *seede;      // [Lp][Lp]  its exponent
    const int2 *tiles;     // (m0, m'0) per workgroup
    int nplain;            // workgroups [0, nplain) take plain tiles, the rest extended-exponent ones
    double2 *U;            // workspace; scale j at sc.off[j]: [N][Lj][Lj] = [n][m][m']
    size_t s_fpad, s_U;    // per-map strides (elements) of a batch; map = blockIdx.y
    int L, Lp, N, eoff;    // eoff = 3 when eta_N = i (conj(eta) = i^3), else 0
    int nk[kMaxK];
    SegTab seg;
    ScaleTab sc;
};

struct WigAdjArgs {
    const double *pq;      // as in WigFwdArgs; the partial sums come out divided by g_l(m)
    const double *uv;
    const void *kb2;       // double, or float if f32 (same layout as in WigFwdArgs)
    const double *seed;
    const double *seedm;
    const int *seede;
    const int2 *tiles;
    int nplain;
    const void *V;         // scale j at sc.off[j]: [K][2][Lj][Lj] = [k][P|Q][m][m'], double2 or float2
    void *Fpart;           // [L / group][L][Lp] partial sums over each m' group, double2 or float2
    size_t s_V, s_F;       // per-map strides (complex elements) of a batch; map = blockIdx.y
    int L, Lp, group, f32;
    SegTab seg;
    ScaleTab sc;
};

int wig_slots(int K);                        // default m' slots per wave for K carried orders
int wig_slot_options(int K, int *R);          // compiled slot counts for K (up to 3), returns how many
hipError_t launch_wig_fwd(const WigFwdArgs &a, int K, int R, int ntiles, int maps, hipStream_t st);
hipError_t launch_wig_adj(const WigAdjArgs &a, int K, int R, int ntiles, int maps, hipStream_t st);

// ---------------------------------------------------------------- beta / alpha / gamma stages
// Bluestein stages (stages.hip).  Layouts per scale j (Lj = band-limit of the scale,
// T = 2L - 1, nb beta rings, G gamma samples, Nh = ceil(N/2) orders n >= 0):
//   analysis:  U [N][Lj][Lj] = [n][m][m'] -> Ub [N][Lj][nb] = [n][m][b]
//              -> Y [Nh][nb][T] (alpha sums, n >= 0) -> W [G][nb][T] (gamma pass)
//   synthesis: W -> X [Nh][nb][T] (gamma pass) -> G [N][Lj][nb] = [n][m][b] (alpha sums)
//              -> V [K][2][Lj][Lj] = [k][P|Q][m][m']
struct StageArgs {
    // Arrays are double2 (FP64 path) or float2 (f32 = 1, mixed precision), except the
    // analysis beta input U, which is double2 in both.
    const void *in;
    void *out;
    const void *hh;        // FFT of the stage's chirp (or kernel) sequence, divided by P
    const void *hh2;       // FFT of the w(q) sequence (synthesis beta stage), divided by P
    const void *tw;        // e^{-2 pi i k/P}, k < P
    const void *csq;       // e^{i pi i^2/T}, i < T (alpha stages, T = 2L - 1), or i < nb (beta stages, T = Tb)
    const void *cpp;       // e^{i pi p(p+1)/T} at p + L - 1, |p| < L (T as for csq)
    const void *qw;        // Driscoll-Healy quadrature weights q_t, t < nb (real; synthesis beta stage)
    const void *eph;       // e^{2 pi i r/T}, r < T (blocked alpha stages)
    const void *pcs;       // constant tables of the prime-factor transforms of length T (pfa.h)
    // fused alpha and gamma passes (prime-factor transforms): W written (analysis) or read
    // (synthesis), [G][nb][T] per scale with per-map stride s_w real elements, and the gamma
    // factors tg [G][Nh] ((1 or 2) e^{i n gamma_g} for the analysis, e^{-i n gamma_g} for the synthesis)
    void *wout;
    const void *win;
    const void *tg;
    size_t s_w;
    int G;
    int nblk, B;           // blocked alpha stages: nblk blocks of B samples
    size_t s_in, s_out;    // per-map strides (complex elements) of a batch; map = blockIdx.y
    int L, nb, Lj, N, Nh, K, eta_imag, f32;  // nb: beta rings (L, or 2L on the Driscoll-Healy grid)
    int nk[kMaxK];
    double scale;
};
// Every launcher takes the number of maps of the batch (grid y).
hipError_t launch_beta_fwd_fft(const StageArgs &a, int P, int maps, hipStream_t st);
// Equiangular grid only: columns (n, m) and (n, m + 1) in one transform of size P >= 2Lj + 2L - 3.
hipError_t launch_beta_fwd_pair(const StageArgs &a, int P, int maps, hipStream_t st);
hipError_t launch_alpha_fwd_fft(const StageArgs &a, int P, int maps, hipStream_t st);
hipError_t launch_alpha_adj_fft(const StageArgs &a, int P, int maps, hipStream_t st);
hipError_t launch_alpha_fwd_blk(const StageArgs &a, int P, int maps, hipStream_t st);
// Direct prime-factor alpha transforms, T = 2L - 1 in {2047, 4095} (pcs: that length's tables).
bool pfa_length(int T);
hipError_t launch_alpha_fwd_pfa(const StageArgs &a, int maps, hipStream_t st);
hipError_t launch_alpha_adj_pfa(const StageArgs &a, int maps, hipStream_t st);
// Equiangular grid, T = 2L - 1 in {2047, 4095}: the two-column analysis beta transform as a
// prime-factor transform (eph: e^{2 pi i r/T}; pcs as above).
hipError_t launch_beta_fwd_pfa(const StageArgs &a, int maps, hipStream_t st);
// The alpha and gamma passes of a scale in one kernel with the prime-factor transforms (real
// signals): analysis Ub -> W, synthesis W -> G (scaled by a.scale); one beta ring per
// workgroup.  pfa_fused(T, Nh): whether the fused kernel serves length T with Nh orders n >= 0.
bool pfa_fused(int T, int Nh);
hipError_t launch_alpha_gamma_fwd_pfa(const StageArgs &a, int maps, hipStream_t st);
hipError_t launch_gamma_alpha_adj_pfa(const StageArgs &a, int maps, hipStream_t st);
hipError_t launch_alpha_adj_blk(const StageArgs &a, int P, int maps, hipStream_t st);
hipError_t launch_beta_adj_fft(const StageArgs &a, int P, int maps, hipStream_t st);
hipError_t launch_beta_adj_dh(const StageArgs &a, int P, int maps, hipStream_t st);
// One scale of a multi-scale beta launch: its first workgroup, band-limit, the offsets
// (elements) of its input and output in the stage arrays (synthesis: G and V; analysis: U and
// Ub), and, in the synthesis, its w(q) spectrum.
struct BetaAdjScale {
    int first, Lj;
    long long in_off, out_off;
    const void *hh2;
};
hipError_t launch_beta_adj_multi(const StageArgs &a, const BetaAdjScale *tab, int ns, int nwg, int P, int maps,
                                 hipStream_t st);
// The analysis beta stage of several scales at a prime-factor length T = 2L - 1 (2047, 4095).
hipError_t launch_beta_fwd_pfa_multi(const StageArgs &a, const BetaAdjScale *tab, int ns, int nwg, int maps,
                                     hipStream_t st);

struct GammaArgs {
    const void *win;       // W read (synthesis): double, or float if f32
    void *wout;            // W written (analysis)
    const void *in;        // Y (analysis): double2, or float2 if f32
    void *out;             // X (synthesis)
    const void *tg;        // [2N-1][Nh]: (1 or 2) e^{i n gamma_g} (analysis), e^{-i n gamma_g} (synthesis)
    size_t s_w, s_y;       // per-map strides of W (real elements; complex ones for the _cx kernels) and of
                           // Y / X (complex); map = blockIdx.y
    int L, T, G, Nh, f32;
};
hipError_t launch_gamma_fwd(const GammaArgs &a, int maps, hipStream_t st);
// Analysis alpha and gamma sums of one coarse scale in one pass (real signals): Ub
// [N][Lj][nb] (the beta stage's output, per-map stride s_in complex elements) -> W
// [G][nb][T] (per-map stride s_w real elements), both FP32 with f32; eph = e^{2 pi i r/T},
// r < T, and tg (as for the FP64 gamma pass) in FP64.
constexpr int kAlphaGammaCoeffs = 1024;  // 2 Nh Lj complex coefficients of a ring at most
struct AlphaGammaArgs {
    const void *in;
    void *wout;
    const void *tg;
    const void *eph;
    size_t s_in, s_w;
    int nb, T, Lj, N, Nh, G, f32;
};
hipError_t launch_alpha_gamma_fwd(const AlphaGammaArgs &a, int maps, hipStream_t st);
// Synthesis gamma and alpha quadratures of one coarse scale in one pass (real signals): W
// [G][nb][T] (per-map stride s_w real elements) -> G [N][Lj][nb] (per-map stride s_out
// complex elements), both FP32 with f32; tg = e^{-i n gamma_g} [G][Nh] and eph =
// e^{2 pi i r/T}, r < T, in FP64; scale = the product of the two quadrature weights.
// Nh (2Lj - 1) <= 256.
struct GammaAlphaArgs {
    const void *win;
    void *out;
    const void *tg;
    const void *eph;
    size_t s_w, s_out;
    int nb, T, Lj, N, Nh, G, f32;
    double scale;
};
hipError_t launch_gamma_alpha_adj(const GammaAlphaArgs &a, int maps, hipStream_t st);
hipError_t launch_gamma_adj(const GammaArgs &a, int maps, hipStream_t st);
// Complex signals: complex map z of W (s_w complex elements per map, (re, im) pairs) from /
// to the real maps 2z and 2z + 1 of Y / X; cmaps complex maps.
hipError_t launch_gamma_fwd_cx(const GammaArgs &a, int cmaps, hipStream_t st);
hipError_t launch_gamma_adj_cx(const GammaArgs &a, int cmaps, hipStream_t st);

// --------------------------------------------------------------------------------- misc

// maps: number of maps of a batch (grid z); f_lm, W^Phi_lm of map i at i L^2, workspaces at i s_*.
// The padded copy carries the factor g_l(m) ([L][Lp]) of the rescaled Wigner recurrence.
hipError_t launch_pad_flm(const double2 *flm, const double *g, double2 *fpad, int L, int Lp, size_t s_fpad, int maps,
                          hipStream_t st);
hipError_t launch_scaling(const double2 *flm, const double *phi, double2 *wphi, int L, int maps, hipStream_t st);
// Complex signals as two real ones: cmaps complex f_lm -> real maps 2z, 2z + 1 of fpad, and
// back: f = a + i b (+ the scaling part) from the syntheses of those maps (each L^2 at k s_fab).
hipError_t launch_pad_flm_complex(const double2 *flm, const double *g, double2 *fpad, int L, int Lp, size_t s_fpad,
                                  int cmaps, hipStream_t st);
hipError_t launch_merge_complex(const double2 *fab, size_t s_fab, const double2 *wphi, const double *phi,
                                double2 *flm, int L, int cmaps, hipStream_t st);
// g: the factor g_l(m) ([L][Lp]) the partial sums of the rescaled recurrence lack.
hipError_t launch_syn_final(const void *Fpart, size_t s_F, int f32, int nblk, int group, int Lmax, const double *fac,
                            const double *g, const double2 *wphi, const double *phi, double2 *flm, int L, int Lp,
                            int maps, hipStream_t st);
hipError_t launch_zero_words(void *p, size_t n, hipStream_t st);
hipError_t launch_to_f32(const double *src, float *dst, size_t n, hipStream_t st);
// W [maps][S][G][P] (gamma_g = g step) -> out [maps][S][Q][P] at the Q angles gam (device),
// P points per plane, map i of W at i s_in and of out at i s_out (elements); doubles, or
// floats if f32; G <= 31, maps <= 65535.
hipError_t launch_steer(const void *W, const double *gam, void *out, int f32, int N, int G, double step, int Q,
                        int S, size_t P, size_t s_in, size_t s_out, int maps, hipStream_t st);

// ------------------------------------------------------------ work-list recording
// The persistent executor (persist.hip) runs whole analyses or syntheses of many maps as one
// launch per direction.  Its work list is recorded from the ordinary launch sequence: while a
// Recorder is set on the calling thread (t_rec), each launcher of a stage the executor runs
// appends a job -- body kind, work items per map, threads per item, argument block --
// instead of launching, and every other launcher returns hipErrorNotSupported.

enum PStage : int {
    PS_PAD = 1, PS_SCALING, PS_ZERO, PS_WIGF, PS_BETAF_FFT, PS_BETAF_PAIR, PS_ALPHAF_FFT, PS_ALPHAF_BLK, PS_AGF,
    PS_GAMMAF, PS_GAMMAA, PS_GAA, PS_ALPHAA_FFT, PS_ALPHAA_BLK, PS_BETAA_FFT, PS_BETAA_MULTI, PS_WIGA, PS_SYNF,
};
// Body kind: stage, precision (1: FP32 stages), and two template parameters (log2 of the
// transform size, K and R of the Wigner stages, NH and the pairing of the direct passes).
constexpr int pkind(int stage, int f32, int a = 0, int b = 0) { return (stage << 20) | (f32 << 19) | (a << 8) | b; }
constexpr int pkind_stage(int k) { return k >> 20; }
constexpr int pkind_f32(int k) { return (k >> 19) & 1; }
constexpr int pkind_a(int k) { return (k >> 8) & 0x7ff; }
constexpr int pkind_b(int k) { return k & 0xff; }
constexpr int kPersistMaxP = 2048;  // largest transform of the executor (P / 8 <= 256 threads)

struct PadArgs {
    const double2 *flm;
    const double *g;
    double2 *fpad;
    int L, Lp;
    size_t s_fpad;
};
struct ScalingArgs {
    const double2 *flm;
    const double *phi;
    double2 *wphi;
    int L;
};
struct SynFinalArgs {
    const void *Fpart;
    size_t s_F;
    int nblk, group, Lmax, L, Lp;
    const double *fac, *g, *phi;
    const double2 *wphi;
    double2 *flm;
};
struct ZeroArgs {
    uint32_t *p;
    size_t n;
};
struct BetaMultiArgs {
    StageArgs a;
    const BetaAdjScale *tab;
    int ns;
};

struct RecJob {
    int kind = 0;
    long long gx = 0;  // work items (workgroups of the ordinary launch) per map
    int maps = 0;
    int nt = 256;      // threads per work item
    std::vector<unsigned char> args;
};
struct Recorder {
    std::vector<RecJob> jobs;
};
extern thread_local Recorder *t_rec;

template <class A>
hipError_t rec_job(int kind, long long gx, int maps, int nt, const A &a) {
    RecJob j;
    j.kind = kind;
    j.gx = gx;
    j.maps = maps;
    j.nt = nt;
    j.args.resize(sizeof(A));
    std::memcpy(j.args.data(), &a, sizeof(A));
    t_rec->jobs.push_back(std::move(j));
    return hipSuccess;
}
// The executor's tables (device).  Job j: nx work items per map, item i covering (256 / nt)
// rounds consecutive workgroups of the ordinary launch (gx per map); for map z it waits until
// every item of job prev (-1: none) has signalled counter ctr0 + z of that job.  The work is
// split into kPersistQueues ticket queues, each a list of entries (job, map) in dependency
// order, entry e of queue q taking tickets [item0, item0 + nx) of that queue.
struct PJob {
    int kind, gx, nt, rounds, nx, maps, prev, ctr0;
    unsigned long long arg;  // byte offset of the argument block
};
struct PEnt {
    int job, map, item0, pad_;
};
constexpr int kPersistQueues = 8;
struct PState {
    int ticket[kPersistQueues];
    int exited, error, pad_[2];
};
// The executor's two parts: 0 the Wigner stages (with the input padding and the final
// synthesis reduction), 1 the separation-of-variables stages; part of a body kind.
int persist_part(int kind);
// m' slots per wave of the executor's Wigner tiles for K carried orders.
int persist_slots(int K);
// Workers one launch may keep resident (occupancy x compute units) for direction dir (0
// analysis, 1 synthesis), part and precision f32; 0 when the query fails.
int persist_workers(int dir, int part, int f32);
// status (device, may be null): the launch's error word (1: a dependency wait ran out of
// polls); with status_or only a nonzero value is written.  wait_extra = 1 (tests only) makes
// every dependency wait unsatisfiable, so that each runs out after spin_limit polls.  chunk:
// tickets a worker takes at a time (>= 1).
// qoff[q] .. qoff[q + 1]: the entries of queue q; qn[q]: its tickets.
hipError_t launch_persist(int dir, int part, int f32, int workers, const PJob *jobs, const PEnt *ents,
                          const int *qoff, const int *qn, const unsigned char *args, int *ctr, int nctr,
                          PState *state, int *status, int spin_limit, int status_or, int wait_extra, int chunk,
                          hipStream_t st);

inline int log2_exact(int P) {
    int k = 0;
    while ((1 << k) < P) ++k;
    return (1 << k) == P ? k : -1;
}
// An FFT stage of size P: one work item per column, P / 8 threads.
template <class A>
hipError_t rec_fft(int stage, const A &a, int f32, int P, long long gx, int maps) {
    const int lg = log2_exact(P);
    if (lg < 5 || P > kPersistMaxP) return hipErrorNotSupported;
    return rec_job(pkind(stage, f32, lg), gx, maps, P / 8, a);
}

}  // namespace s2dw
