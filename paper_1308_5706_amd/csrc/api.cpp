// C ABI of the directional scale-discretized wavelet library: argument checks,
// per-parameter plans (tables, tile lists, workspaces) and the launch sequences.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <tuple>

#include "../../include/s2dw.h"
#include "kernels.h"

namespace s2dw {
namespace {

enum PlanKind { kWavelet = 0, kShtInverse = 1, kShtForward = 2 };

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Wigner tile shape of a plan (R m' slots per wave, the tile lists of both directions and
// the layout of the synthesis partial sums) and the maps per batched launch sequence.
// s2dw_autotune replaces it; every call copies it under g_mu when it starts and uses its
// copy throughout, so a call in flight on another stream keeps a consistent shape (tile
// lists are kept until the plan is freed).
struct Shape {
    int R = 0, group = 0, nblk = 0;
    const int2 *tiles_fwd = nullptr, *tiles_adj = nullptr;
    int nfwd_plain = 0, nfwd_x = 0, nadj_plain = 0, nadj_x = 0;
    size_t s_F = 0;                             // per-map partial-sum elements
    int chunk = 1;                              // maps per batched launch sequence (tunable)
    // the fused alpha and gamma kernels of the prime-factor lengths (tunable): 0 never,
    // 1 where they were measured faster than the two-pass form (fuse_fwd, fuse_adj),
    // 2 wherever they apply
    int fuse = 1;
};

struct Plan {
    int kind = 0, L = 0, N = 0, J_min = 0, S = 0, K = 0, Lp = 0, Lmax = 0;
    double lam = 2.0;
    HostTables ht;
    SegTab seg{};
    ScaleTab sc{};
    int eoff = 0;
    // sample grid of each scale: full resolution (band-limit L for every scale) or
    // multiresolution (the scale's own band-limit Lj); W of a map holds the scales back to back
    int grid = S2DW_GRID_MW;
    int Lg[kMaxScales] = {};                    // grid band-limit: alpha 2Lg - 1 samples
    int nb = 0, ng = 0;                         // beta rings and gamma samples of the (full) grid:
                                                // (L, 2N - 1), or (2L, N) on the Driscoll-Healy grid
    // Driscoll-Healy beta tables: chirps of Tb = 4L (csq t < 2L, cpp at p + L - 1, |p| < L) and
    // the quadrature weights q_t (Eq. 18); per scale the synthesis beta spectrum (size PE)
    double2 *dh_csq = nullptr, *dh_cpp = nullptr;
    double *dh_q = nullptr;
    float2 *dh_csqf = nullptr, *dh_cppf = nullptr;
    float *dh_qf = nullptr;
    std::vector<int> PE;
    std::vector<double2 *> hE;
    std::vector<float2 *> hEf;
    // the coarse scales j >= mj0 of the synthesis beta stage run in one launch (equiangular
    // full grid): their G arrays sit at goff[j] in the beta-stage workspace; mtab / mtabf
    // describe them to the kernel (mns scales, mnwg workgroups per map)
    int mj0 = -1, mns = 0, mnwg = 0;
    // the analysis beta stage of the same coarse scales in one launch at the prime-factor
    // lengths (their Ub arrays at goff[j]); atab describes them (ans scales, anwg workgroups)
    int ans = 0, anwg = 0;
    BetaAdjScale *atab = nullptr;
    size_t goff[kMaxScales] = {};
    BetaAdjScale *mtab = nullptr, *mtabf = nullptr;
    size_t woff[kMaxScales + 1] = {};           // element offset of scale j in the W of one map
    // chirp tables of one grid band-limit (length T = 2Lg - 1) and the spectrum of the first
    // synthesis beta convolution (transform size PD)
    struct GridTab {
        double2 *csq = nullptr, *cpp = nullptr, *hD1 = nullptr, *eph = nullptr;
        float2 *csqf = nullptr, *cppf = nullptr, *hD1f = nullptr, *ephf = nullptr;
        int PD = 0;
        // prime-factor transform tables of length T (when T is one of its lengths)
        double2 *pcs = nullptr;
        float2 *pcsf = nullptr;
        int npcs = 0;
    };
    std::map<int, GridTab> gt;
    // device tables
    double *pq = nullptr, *uv = nullptr;        // rescaled recurrence factors pt_l(m), ut_l(m')
    double *gsc = nullptr;                      // [L][Lp] g_l(m): D = Delta / (g_l(m) h_l(m'))
    double2 *tgf = nullptr, *tga = nullptr;     // gamma pass factors [2N-1][Nh]
    double *kb2 = nullptr, *seed = nullptr, *seedm = nullptr, *phi = nullptr, *fac = nullptr;
    int *seede = nullptr;
    Shape cur;                                  // current tile shape (guarded by g_mu)
    // tile lists per number R of m' slots per wave (the Wigner tile shape), built on demand
    struct TileSet {
        int2 *fwd = nullptr, *adj = nullptr;
        int nfwd_plain = 0, nfwd_x = 0, nadj_plain = 0, nadj_x = 0;
    };
    std::map<int, TileSet> tilesets;
    std::vector<int> seede_h;                   // start-value exponents [Lp][Lp] (host)
    // Bluestein stages: transform sizes and chirp spectra per scale, twiddles per size
    std::vector<int> PA, PB;                    // beta (analysis), alpha (both directions)
    // blocked alpha transforms (scales with few coefficients): nblk blocks of B samples, each
    // a convolution of size PBb; nblk = 0 where the single convolution of size PB is used
    std::vector<int> PBb, Bb, nblkb;
    std::vector<double2 *> hBb, hCb;
    std::vector<float2 *> hBbf, hCbf;
    std::vector<double2 *> hA, hB, hC, hD2;     // per scale (hD2 has the size PD of the scale's grid)
    std::map<int, double2 *> twP;               // e^{-2 pi i k/P}
    // FP32 copies of the stage tables for the mixed-precision path (built on first use)
    bool f32_ready = false;
    float2 *tgff = nullptr, *tgaf = nullptr;
    std::vector<float2 *> hAf, hBf, hCf, hD2f;
    std::map<int, float2 *> twPf;
    float *kb2f = nullptr;
    size_t n_kb2 = 0, n_tg = 0;
    int Nh = 0;                                 // orders n >= 0 carried: ceil(N/2)
    // per-map workspace sizes (complex elements; the partial sums' size is part of the shape)
    size_t s_fpad = 0, s_U = 0, s_Ub = 0, s_Y = 0;
    std::vector<void *> allocs;
    size_t dev_bytes = 0;
    // workspaces, one context per stream (calls on different streams may overlap)
    std::map<void *, std::unique_ptr<struct Work>> work;
    ~Plan();
};

// Workspace of one stream: room for `cap` maps of a batch, map i at i * Plan::s_* (the
// partial sums at i * Shape::s_F, room for cap * s_F elements).
struct Work {
    int cap = 0;
    size_t s_F = 0;
    double2 *fpad = nullptr, *U = nullptr, *Ub = nullptr, *Y = nullptr, *Fpart = nullptr;
    std::vector<void *> allocs;
    size_t bytes = 0;
    ~Work() {
        for (void *p : allocs) hipFree(p);
    }
};

Plan::~Plan() {
    work.clear();
    for (void *p : allocs) hipFree(p);
}

// ----------------------------------------------------------------------- stage timing
struct Prof {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec {
        const char *name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::map<std::string, std::pair<double, int64_t>> totals;
    std::set<std::string> only;  // stages timed while on; empty: every stage
};
Prof g_prof;

hipEvent_t prof_event() {
    if (g_prof.used == g_prof.pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_prof.pool.push_back(e);
    }
    return g_prof.pool[g_prof.used++];
}

// Set while the calling thread runs the entry point that allocates nothing: its launches
// record no timing events (creating one may allocate).
thread_local bool t_no_events = false;
}  // namespace
thread_local Recorder *t_rec = nullptr;  // work-list recording (persistent executor), kernels.h
namespace {

// Records events around one launch when timing is on.
struct Stage {
    hipStream_t st;
    hipEvent_t a = nullptr;
    const char *name;
    Stage(const char *n, hipStream_t s) : st(s), name(n) {
        if (!g_prof.on || t_no_events) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!g_prof.only.empty() && !g_prof.only.count(n)) return;
        a = prof_event();
        if (a) hipEventRecord(a, st);
    }
    ~Stage() {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        hipEvent_t b = prof_event();
        if (!b) return;
        hipEventRecord(b, st);
        g_prof.recs.push_back({name, a, b});
    }
};

void prof_collect() {
    for (auto &r : g_prof.recs) {
        float ms = 0.f;
        hipEventSynchronize(r.b);
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto &t = g_prof.totals[r.name];
            t.first += ms;
            t.second += 1;
        }
    }
    g_prof.recs.clear();
    g_prof.used = 0;
}

typedef std::tuple<int, int, int, double, int, int> PlanKey;
std::mutex g_mu;
std::map<PlanKey, std::unique_ptr<Plan>> g_plans;

template <typename T>
bool dalloc(Plan &pl, T *&p, size_t count) {
    p = nullptr;
    if (count == 0) count = 1;
    void *q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return false;
    pl.allocs.push_back(q);
    pl.dev_bytes += count * sizeof(T);
    p = (T *)q;
    return true;
}

template <typename T>
bool upload(Plan &pl, T *&p, const std::vector<T> &h) {
    if (!dalloc(pl, p, h.size())) return false;
    return hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

// Segments of [0, L) on which the active scales are fixed.
bool build_segments(const HostTables &t, SegTab &seg) {
    std::vector<int> b = {0, t.L};
    for (int j = 0; j < t.S; ++j)
        if (t.hi[j] >= t.lo[j]) {
            b.push_back(t.lo[j]);
            b.push_back(t.hi[j] + 1);
        }
    std::sort(b.begin(), b.end());
    b.erase(std::unique(b.begin(), b.end()), b.end());
    seg.n = 0;
    for (size_t i = 0; i + 1 < b.size(); ++i) {
        if (b[i] >= t.L) break;
        if (seg.n >= kMaxSegs) return false;
        int s0 = b[i], s1 = std::min(b[i + 1], t.L);
        int je = -1, jo = -1;
        for (int j = 0; j < t.S; ++j) {
            if (t.hi[j] < t.lo[j]) continue;
            if (t.lo[j] <= s0 && t.hi[j] >= s1 - 1) {
                int &slot = (j % 2 == 0) ? je : jo;
                if (slot >= 0) return false;  // two scales of one parity overlap
                slot = j;
            }
        }
        seg.s0[seg.n] = s0;
        seg.s1[seg.n] = s1;
        seg.je[seg.n] = (int8_t)je;
        seg.jo[seg.n] = (int8_t)jo;
        ++seg.n;
    }
    return true;
}

// Dispatch order of a tile list for L2 reuse.  Workgroups are handed to the 8 XCDs
// round-robin, so list position i runs on XCD (phase + i) mod 8.  The tiles of one m' group
// read the same m' rows of the wave-uniform tables (kappa sigma Delta, u, v) at every l;
// keeping a group on one XCD lets those rows come from that XCD's L2.  Groups go to the XCD
// with the least work so far (heaviest group first), each as a run of its tiles, heaviest
// first; positions whose XCD has no tile left take one from the fullest XCD.
std::vector<int2> xcd_order(const std::vector<std::pair<long, int2>> &tiles, int phase, bool mmajor = false) {
    std::map<int, std::vector<std::pair<long, int2>>> groups;  // by m'0
    for (const auto &e : tiles) groups[e.second.y].push_back(e);
    std::vector<std::pair<long, int>> gw;
    for (auto &g : groups) {
        std::stable_sort(g.second.begin(), g.second.end(),
                         [](const std::pair<long, int2> &u, const std::pair<long, int2> &v) { return u.first > v.first; });
        long w = 0;
        for (const auto &e : g.second) w += e.first;
        gw.push_back({w, g.first});
    }
    std::stable_sort(gw.begin(), gw.end(),
                     [](const std::pair<long, int> &u, const std::pair<long, int> &v) { return u.first > v.first; });
    std::vector<std::vector<int2>> bins(8);
    long load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (const auto &g : gw) {
        const int x = (int)(std::min_element(load, load + 8) - load);
        load[x] += g.first;
        for (const auto &e : groups[g.second]) bins[x].push_back(e.second);
    }
    // mmajor: each XCD takes its tiles m-tile by m-tile (then m' group), so that the workgroups
    // resident on it at one time share the per-lane columns (g f_lm and pt) of a few m-tiles
    // rather than the table rows of a few m' groups
    if (mmajor)
        for (auto &b : bins)
            std::stable_sort(b.begin(), b.end(),
                             [](const int2 &u, const int2 &v) { return u.x < v.x || (u.x == v.x && u.y < v.y); });
    std::vector<int2> out;
    size_t pos[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    while (out.size() < tiles.size()) {
        int x = (int)((phase + out.size()) % 8);
        if (pos[x] >= bins[x].size()) {
            size_t best = 0;
            for (int y = 0; y < 8; ++y)
                if (bins[y].size() - pos[y] > best) {
                    best = bins[y].size() - pos[y];
                    x = y;
                }
        }
        out.push_back(bins[x][pos[x]++]);
    }
    return out;
}

// Tile lists for the Wigner kernels: (m0, m'0) pairs in XCD-aware order (above); tiles holding
// a start value below 2^-1000 go to the extended-exponent list, launched after the others.
void build_tiles(const Plan &pl, const std::vector<int> &seede, int Lp, int mgroup, std::vector<int2> &plain,
                 std::vector<int2> &xn, bool mmajor = false) {
    std::vector<std::pair<long, int2>> a, b;
    const int L = pl.L, Lmax = pl.Lmax;
    for (int m0 = 0; m0 < Lmax; m0 += 64)
        for (int p0 = 0; p0 < Lmax; p0 += mgroup) {
            long work = Lmax - std::max(m0, p0);
            bool x = false;
            for (int mp = p0; mp < std::min(p0 + mgroup, L) && !x; ++mp)
                for (int m = m0; m < std::min(m0 + 64, L); ++m)
                    if (seede[(size_t)mp * Lp + m] < -1000) {
                        x = true;
                        break;
                    }
            (x ? b : a).push_back({work, make_int2(m0, p0)});
        }
    plain = xcd_order(a, 0, mmajor);
    xn = xcd_order(b, (int)(a.size() % 8), mmajor);
}

// Selects the Wigner tile shape: R m' slots per wave (the analysis workgroup covers 4R
// m', the synthesis one kAdjWaves R).  Tile lists are built once per R and kept.  Caller
// holds g_mu.  Calls in flight keep the shape they copied; a stream whose workspace is too
// small for the new partial-sum layout gets a larger one at its next call.
int set_slots(Plan &P, int R) {
    auto it = P.tilesets.find(R);
    if (it == P.tilesets.end()) {
        Plan::TileSet ts;
        std::vector<int2> pl_a, x_a, pl_s, x_s;
        // the analysis reads per-lane columns at every step, the synthesis does not: at large L
        // (32 m-tiles or more) its tiles go m-tile major (measured at L = 2048, N = 4: analysis
        // 2.55 -> 2.30 ms; at L = 1024 and for the synthesis the m' group order is faster)
        build_tiles(P, P.seede_h, P.Lp, 4 * R, pl_a, x_a, P.Lmax >= 1536);
        build_tiles(P, P.seede_h, P.Lp, kAdjWaves * R, pl_s, x_s);
        ts.nfwd_plain = (int)pl_a.size();
        ts.nfwd_x = (int)x_a.size();
        ts.nadj_plain = (int)pl_s.size();
        ts.nadj_x = (int)x_s.size();
        pl_a.insert(pl_a.end(), x_a.begin(), x_a.end());
        pl_s.insert(pl_s.end(), x_s.begin(), x_s.end());
        if (!upload(P, ts.fwd, pl_a) || !upload(P, ts.adj, pl_s)) return S2DW_E_NOMEM;
        it = P.tilesets.emplace(R, ts).first;
    }
    const Plan::TileSet &ts = it->second;
    Shape &sh = P.cur;
    sh.R = R;
    sh.tiles_fwd = ts.fwd;
    sh.tiles_adj = ts.adj;
    sh.nfwd_plain = ts.nfwd_plain;
    sh.nfwd_x = ts.nfwd_x;
    sh.nadj_plain = ts.nadj_plain;
    sh.nadj_x = ts.nadj_x;
    sh.group = kAdjWaves * R;
    sh.nblk = (P.L + sh.group - 1) / sh.group;
    sh.s_F = (size_t)sh.nblk * P.L * P.Lp;
    return S2DW_OK;
}

// The plan's current shape (copied under g_mu).
Shape shape_of(Plan &P) {
    std::lock_guard<std::mutex> lk(g_mu);
    return P.cur;
}

// Default maps per batched launch sequence: as many as fit 8 GiB of workspace, at most 64.
int default_chunk(const Plan &P) {
    const double per_map = 16.0 * (double)(P.s_fpad + P.s_U + P.s_Ub + P.s_Y + P.cur.s_F);
    return (int)std::max(1.0, std::min(64.0, std::floor(8.0 * (1ull << 30) / per_map)));
}

typedef long double ld;
const ld kPiL = 3.141592653589793238462643383279502884L;

// In-place radix-2 FFT in long double (host), X_k = sum_n x_n e^{-2 pi i n k/P}.
void host_fft(std::vector<ld> &re, std::vector<ld> &im) {
    const int P = (int)re.size();
    for (int i = 1, j = 0; i < P; ++i) {
        int bit = P >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            std::swap(re[i], re[j]);
            std::swap(im[i], im[j]);
        }
    }
    for (int len = 2; len <= P; len <<= 1) {
        for (int i = 0; i < P; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const ld a = -2.0L * kPiL * k / len;
                const ld c = cosl(a), sn = sinl(a);
                const int u = i + k, v = i + k + len / 2;
                const ld xr = re[v] * c - im[v] * sn, xi = re[v] * sn + im[v] * c;
                re[v] = re[u] - xr;
                im[v] = im[u] - xi;
                re[u] += xr;
                im[u] += xi;
            }
    }
}

int pow2_at_least(int n) {
    int p = 32;
    while (p < n) p <<= 1;
    return p;
}

// FFT of h'(i), i < len (zero beyond), divided by P and by `div`; h'(i) given by f(i).
template <typename F>
std::vector<double2> spectrum(int P, int len, ld div, F f) {
    std::vector<ld> re(P, 0.0L), im(P, 0.0L);
    for (int i = 0; i < len && i < P; ++i) {
        const std::pair<ld, ld> v = f(i);
        re[i] = v.first;
        im[i] = v.second;
    }
    host_fft(re, im);
    std::vector<double2> out(P);
    for (int i = 0; i < P; ++i) out[i] = make_double2((double)(re[i] / (P * div)), (double)(im[i] / (P * div)));
    return out;
}

// e^{sign i pi d^2 / T} with d^2 reduced exactly modulo 2T.
std::pair<ld, ld> chirp_val(long long d, int T, int sign) {
    const long long r = (d * d) % (2LL * T);
    const ld a = sign * kPiL * (ld)r / (ld)T;
    return {cosl(a), sinl(a)};
}

// Constant tables of the direct prime-factor transforms of length T (see pfa.h): cos and sin
// of 2 pi j/q for each factor q, and for T = 2047 the per-wave constants of the length-89
// stage.  Empty when T is not one of those lengths.
std::vector<double2> pfa_tables(int T) {
    auto cs = [](ld x) { return make_double2((double)cosl(x), (double)sinl(x)); };
    std::vector<double2> t;
    auto roots = [&](int q) {
        for (int j = 0; j < q; ++j) t.push_back(cs(2.0L * kPiL * j / q));
    };
    if (T == 2047) {
        roots(23);
        roots(89);
        // per wave of the length-89 stage, in its four-wave and eight-wave groupings
        const int H = 44;
        for (const auto &g : {std::make_pair(4, 11), std::make_pair(8, 6)})
            for (int w = 0; w < g.first; ++w)
                for (int r = 1; r <= H; ++r)
                    for (int kk = 0; kk < g.second; ++kk) {
                        const int k = 1 + w * g.second + kk;
                        t.push_back(cs(2.0L * kPiL * ((r * k) % 89) / 89));
                    }
    } else if (T == 4095) {
        roots(5);
        roots(7);
        roots(9);
        roots(13);
    }
    return t;
}

// Chirp tables of grid band-limit Lg (T = 2Lg - 1) and the spectrum of the first synthesis
// beta convolution, shared by the scales sampled on that grid.
int build_grid_tab(Plan &P, int Lg) {
    if (P.gt.count(Lg)) return S2DW_OK;
    Plan::GridTab g;
    const int M = 2 * Lg - 1;
    std::vector<double2> csq(M), cpp(M), eph(M);
    for (int r = 0; r < M; ++r) {
        const ld a = 2.0L * kPiL * (ld)r / (ld)M;
        eph[r] = make_double2((double)cosl(a), (double)sinl(a));
    }
    // chirps with the phase reduced exactly modulo 2T
    for (int i = 0; i < M; ++i) {
        const long long p = i - (Lg - 1);
        const long long r2 = ((long long)i * i) % (2LL * M), rp = ((p * (p + 1)) % (2LL * M) + 2LL * M) % (2LL * M);
        const ld a2 = kPiL * (ld)r2 / (ld)M, ap = kPiL * (ld)rp / (ld)M;
        csq[i] = make_double2((double)cosl(a2), (double)sinl(a2));
        cpp[i] = make_double2((double)cosl(ap), (double)sinl(ap));
    }
    g.PD = pow2_at_least(2 * M - 1);
    if (g.PD > 8192) return S2DW_E_UNSUPPORTED;
    auto hd1 = spectrum(g.PD, 2 * M - 1, (ld)M, [&](int i) { return chirp_val((long long)i - Lg - M + 2, M, +1); });
    if (!upload(P, g.csq, csq) || !upload(P, g.cpp, cpp) || !upload(P, g.hD1, hd1) || !upload(P, g.eph, eph))
        return S2DW_E_NOMEM;
    const std::vector<double2> pt = pfa_tables(M);
    if (!pt.empty()) {
        if (!upload(P, g.pcs, pt)) return S2DW_E_NOMEM;
        g.npcs = (int)pt.size();
    }
    P.gt[Lg] = g;
    return S2DW_OK;
}

int build_plan(int kind, int L, int N, double lam, int J_min, int grid, Plan *&out) {
    std::unique_ptr<Plan> pl(new (std::nothrow) Plan());
    if (!pl) return S2DW_E_NOMEM;
    pl->kind = kind;
    pl->grid = grid;
    pl->L = L;
    pl->N = N;
    pl->lam = lam;
    pl->J_min = J_min;
    HostTables &t = pl->ht;
    if (kind == kWavelet) {
        if (!build_wavelet_tables(L, N, lam, J_min, t)) return S2DW_E_ARG;
    } else {
        // a single pseudo-scale with n = 0 only: the spherical-harmonic transforms
        t.L = L;
        t.N = 1;
        t.S = 1;
        t.K = 1;
        t.eta_imag = false;
        t.nk = {0};
        t.kappa.assign(L, 1.0);
        if (kind == kShtInverse)
            for (int l = 0; l < L; ++l) t.kappa[l] = std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI));
        t.phi.assign(L, 0.0);
        t.sig.assign(L, 1.0);
        t.lo = {0};
        t.hi = {L - 1};
    }
    pl->S = t.S;
    pl->K = t.K;
    pl->eoff = t.eta_imag ? 3 : 0;
    if (!build_segments(t, pl->seg)) return S2DW_E_INTERNAL;
    pl->sc.S = t.S;
    int64_t off = 0, boff = 0;
    pl->Lmax = 0;
    for (int j = 0; j < t.S; ++j) {
        int Lj = t.hi[j] >= t.lo[j] ? t.hi[j] + 1 : 0;
        pl->sc.Lj[j] = Lj;
        pl->sc.off[j] = off;
        pl->sc.boff[j] = boff;
        off += (int64_t)std::max(t.N, 2 * t.K) * Lj * Lj;
        boff += (int64_t)t.N * L * Lj;
        pl->Lmax = std::max(pl->Lmax, Lj);
    }
    // Delta tables
    DeltaTables dt;
    build_delta_tables(L, dt);
    pl->Lp = dt.Lp;
    std::vector<double> ncol;
    build_delta_ncols(dt, t.nk, ncol);
    const int K = t.K, Lp = dt.Lp;
    // one record of padding at the end: the analysis kernel reads the entries of step l + 1
    // ahead of step l, also after the last step of the last row
    std::vector<double> kb2((size_t)Lp * L * 2 * K + 2 * K, 0.0);
    for (int mp = 0; mp < L; ++mp)
        for (int l = 0; l < L; ++l) {
            int si = 0;
            while (pl->seg.s1[si] <= l) ++si;
            const int js[2] = {pl->seg.je[si], pl->seg.jo[si]};
            for (int s = 0; s < 2; ++s) {
                if (js[s] < 0) continue;
                const double kap = t.kappa[(size_t)js[s] * L + l];
                // h_l(m') of the rescaled recurrence folded in (the g_l(m) side goes with f_lm)
                const double hh = dt.h[(size_t)mp * L + l];
                for (int k = 0; k < K; ++k)
                    kb2[(((size_t)mp * L + l) * 2 + s) * K + k] =
                        kap * t.sig[(size_t)l * K + k] * ncol[((size_t)mp * L + l) * K + k] * hh;
            }
        }
    Plan &P = *pl;
    const int M = 2 * L - 1;
    // sample grids and the W layout of one map
    const bool dh = grid == S2DW_GRID_DH;
    const int Gn = dh ? t.N : 2 * t.N - 1;
    P.nb = dh ? 2 * L : L;
    P.ng = Gn;
    {
        size_t wo = 0;
        for (int j = 0; j < t.S; ++j) {
            const size_t lg = P.Lg[j] = grid == S2DW_GRID_MW_MULTIRES ? P.sc.Lj[j] : L;
            const size_t rings = dh ? 2 * lg : lg;
            P.woff[j] = wo;
            wo += (size_t)Gn * rings * (lg > 0 ? 2 * lg - 1 : 0);
        }
        P.woff[t.S] = wo;
    }
    // gamma pass factors for the orders n >= 0, n = 2 ni - (N - 1), ni = N/2 + k, at
    // gamma_g = 2 pi g/(2N - 1) (equiangular) or pi g/N (Driscoll-Healy, Sec. 3.1)
    P.Nh = t.N - t.N / 2;
    std::vector<double2> tgf((size_t)Gn * P.Nh), tga((size_t)Gn * P.Nh);
    const int gper = dh ? 2 * Gn : Gn;  // gamma_g = 2 pi g/gper
    for (int g = 0; g < Gn; ++g)
        for (int k = 0; k < P.Nh; ++k) {
            const long long n = 2LL * (t.N / 2 + k) - (t.N - 1);
            const long long r = (n * g) % gper;
            const ld a = 2.0L * kPiL * (ld)r / (ld)gper;
            const ld f = n == 0 ? 1.0L : 2.0L;
            tgf[(size_t)g * P.Nh + k] = make_double2((double)(f * cosl(a)), (double)(f * sinl(a)));
            tga[(size_t)g * P.Nh + k] = make_double2((double)cosl(a), (double)-sinl(a));
        }
    std::vector<double> fac(L);
    for (int l = 0; l < L; ++l)
        fac[l] = kind == kShtForward ? std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) / (2.0 * M_PI)
                                     : (2.0 * l + 1.0) / (8.0 * M_PI * M_PI);
    P.n_kb2 = kb2.size();
    P.n_tg = tgf.size();
    dt.ut.resize(dt.ut.size() + 1, 0.0);  // one padding entry (as for kb2)
    bool ok = upload(P, P.pq, dt.pt) && upload(P, P.uv, dt.ut) && upload(P, P.gsc, dt.g) && upload(P, P.kb2, kb2) &&
              upload(P, P.seed, dt.seedt) && upload(P, P.seedm, dt.seedtm) && upload(P, P.seede, dt.seedte) &&
              upload(P, P.tgf, tgf) && upload(P, P.tga, tga) && upload(P, P.fac, fac) && upload(P, P.phi, t.phi);
    if (!ok) return S2DW_E_NOMEM;
    // tiles
    P.seede_h = dt.seedte;
    int rc_t = set_slots(P, wig_slots(K));
    if (rc_t != S2DW_OK) return rc_t;
    // Bluestein chirp spectra per scale, for the scale's grid band-limit Lg (T = 2Lg - 1;
    // see stages.hip for the convolution layouts)
    P.PA.assign(t.S, 0);
    P.PB.assign(t.S, 0);
    P.hA.assign(t.S, nullptr);
    P.hB.assign(t.S, nullptr);
    P.hC.assign(t.S, nullptr);
    P.hD2.assign(t.S, nullptr);
    std::vector<int> sizes;
    P.PE.assign(t.S, 0);
    P.hE.assign(t.S, nullptr);
    P.PBb.assign(t.S, 0);
    P.Bb.assign(t.S, 0);
    P.nblkb.assign(t.S, 0);
    P.hBb.assign(t.S, nullptr);
    P.hCb.assign(t.S, nullptr);
    const int Tb = dh ? 4 * L : 0;
    if (dh) {
        // Driscoll-Healy beta grid: chirps of Tb = 4L and the weights of Eq. 18
        std::vector<double2> csq(P.nb), cpp(2 * L - 1);
        std::vector<double> q(P.nb);
        for (int i = 0; i < P.nb; ++i) {
            const std::pair<ld, ld> c = chirp_val(i, Tb, +1);
            csq[i] = make_double2((double)c.first, (double)c.second);
            const ld th = kPiL * (2 * i + 1) / (ld)Tb;
            ld acc = 0.0L;
            for (int k = 0; k < L; ++k) acc += sinl((2 * k + 1) * th) / (2 * k + 1);
            q[i] = (double)(2.0L / L * sinl(th) * acc);
        }
        for (int i = 0; i < 2 * L - 1; ++i) {
            const long long p = i - (L - 1);
            const long long rp = ((p * (p + 1)) % (2LL * Tb) + 2LL * Tb) % (2LL * Tb);
            const ld a = kPiL * (ld)rp / (ld)Tb;
            cpp[i] = make_double2((double)cosl(a), (double)sinl(a));
        }
        if (!upload(P, P.dh_csq, csq) || !upload(P, P.dh_cpp, cpp) || !upload(P, P.dh_q, q)) return S2DW_E_NOMEM;
    }
    for (int j = 0; j < t.S; ++j) {
        const int Lj = P.sc.Lj[j];
        if (Lj == 0) continue;
        const int Lg = P.Lg[j], T = 2 * Lg - 1;
        int rc_g = build_grid_tab(P, Lg);
        if (rc_g != S2DW_OK) return rc_g;
        const int PD = P.gt[Lg].PD;
        const int nbj = dh ? P.nb : Lg, Tbj = dh ? Tb : T;  // beta rings and beta chirp length
        P.PA[j] = pow2_at_least(2 * Lj + nbj - 2);
        P.PB[j] = pow2_at_least(2 * Lj + T - 2);
        if (P.PA[j] > 8192 || P.PB[j] > 8192) return S2DW_E_UNSUPPORTED;
        sizes.push_back(PD);
        sizes.push_back(P.PA[j]);
        sizes.push_back(P.PB[j]);
        if (dh) {
            // synthesis beta sum: kernel e^{i pi d^2/Tb} at d = i - (Lj + nb - 2)
            P.PE[j] = pow2_at_least(nbj + 2 * Lj - 2);
            if (P.PE[j] > 8192) return S2DW_E_UNSUPPORTED;
            sizes.push_back(P.PE[j]);
            auto he = spectrum(P.PE[j], nbj + 2 * Lj - 2, 1.0L,
                               [&](int i) { return chirp_val((long long)i - (Lj + nbj - 2), Tb, +1); });
            if (!upload(P, P.hE[j], he)) return S2DW_E_NOMEM;
        }
        {
            // blocked alpha transforms: the cheapest of one convolution of size PB and nblk of
            // size Q in {512, 1024, 2048} over B = Q - 2Lj + 2 samples each (cost ~ count
            // Q log2 Q), taken when it saves at least 30% (measured: the looped short
            // convolutions reach about 0.1-0.2 less than this model predicts)
            auto cost = [](int Q) { return (double)Q * std::log2((double)Q); };
            double best = 0.7 * cost(P.PB[j]);
            for (int Q = 512; Q <= 2048; Q *= 2) {
                const int B = Q - 2 * Lj + 2;
                if (B < 64) continue;
                const int nbk = (T + B - 1) / B;
                if (nbk < 2) continue;
                if (nbk * cost(Q) < best) {
                    best = nbk * cost(Q);
                    P.PBb[j] = Q;
                    P.Bb[j] = B;
                    P.nblkb[j] = nbk;
                }
            }
            if (P.nblkb[j] > 1) {
                const int Q = P.PBb[j], B = P.Bb[j];
                sizes.push_back(Q);
                auto hb = spectrum(Q, 2 * Lj + B - 2, 1.0L,
                                   [&](int i) { return chirp_val((long long)i - Lj + 1, T, -1); });
                auto hc = spectrum(Q, 2 * Lj + B - 2, 1.0L,
                                   [&](int i) { return chirp_val((long long)i - Lj - B + 2, T, +1); });
                if (!upload(P, P.hBb[j], hb) || !upload(P, P.hCb[j], hc)) return S2DW_E_NOMEM;
            }
        }
        // the kernel's support covers nbj outputs, or all T ring positions where the analysis
        // beta stage transforms two columns at once (the two-column condition of run_inverse)
        const int na_out = (!dh && pow2_at_least(2 * Lj + 2 * Lg - 3) <= P.PA[j]) ? T : nbj;
        auto ha = spectrum(P.PA[j], 2 * Lj + na_out - 2, 1.0L,
                           [&](int i) { return chirp_val((long long)i - Lj + 1, Tbj, -1); });
        auto hb = spectrum(P.PB[j], 2 * Lj + T - 2, 1.0L,
                           [&](int i) { return chirp_val((long long)i - Lj + 1, T, -1); });
        auto hc = spectrum(P.PB[j], 2 * Lj + T - 2, 1.0L,
                           [&](int i) { return chirp_val((long long)i - Lj - T + 2, T, +1); });
        // the even part of w(q) = int_0^pi sin(b) e^{i q b} db, 2/(1 - q^2) at even q (its odd
        // part, +-i pi/2 at q = +-1, drops out of the folded sums of the paired columns, see
        // stages.hip), at q = Lj + Lg - 2 - i
        auto hd2 = spectrum(PD, T + 2 * Lj - 2, 1.0L, [&](int i) {
            const long long q = (long long)Lj + Lg - 2 - i;
            if (q % 2 == 0) return std::pair<ld, ld>(2.0L / (1.0L - (ld)q * (ld)q), 0.0L);
            return std::pair<ld, ld>(0.0L, 0.0L);
        });
        if (!upload(P, P.hA[j], ha) || !upload(P, P.hB[j], hb) || !upload(P, P.hC[j], hc) || !upload(P, P.hD2[j], hd2))
            return S2DW_E_NOMEM;
    }
    if (grid == S2DW_GRID_MW && kind == kWavelet) {
        // coarse scales (at most 256 order-column pairs each) at the end of the scale list, as many
        // as the beta-stage workspace holds side by side (sum of their Lj <= the largest Lj)
        int maxL = 0;
        for (int j = 0; j < t.S; ++j) maxL = std::max(maxL, P.sc.Lj[j]);
        int j0 = t.S, sumL = 0;
        while (j0 > 0 && P.K * ((P.sc.Lj[j0 - 1] + 1) / 2) <= 256 && sumL + P.sc.Lj[j0 - 1] <= maxL) sumL += P.sc.Lj[--j0];
        std::vector<BetaAdjScale> tab;
        size_t go = 0;
        int nwg = 0;
        for (int j = j0; j < t.S; ++j) {
            const int Lj = P.sc.Lj[j];
            if (Lj == 0) continue;
            P.goff[j] = go;
            tab.push_back(BetaAdjScale{nwg, Lj, (long long)go, (long long)P.sc.off[j], (const void *)P.hD2[j]});
            go += (size_t)t.N * Lj * L;
            nwg += P.K * ((Lj + 1) / 2);  // one workgroup per order and pair of columns (m, m + 1)
        }
        if (tab.size() >= 2) {
            if (!upload(P, P.mtab, tab)) return S2DW_E_NOMEM;
            P.mj0 = j0;
            P.mns = (int)tab.size();
            P.mnwg = nwg;
            if (pfa_length(2 * L - 1)) {
                const int NC = 2 * L - 1 == 2047 ? 2 : 1;  // column pairs per workgroup
                std::vector<BetaAdjScale> at;
                int anwg = 0;
                for (int j = j0; j < t.S; ++j) {
                    const int Lj = P.sc.Lj[j];
                    if (Lj == 0) continue;
                    at.push_back(BetaAdjScale{anwg, Lj, (long long)P.sc.off[j], (long long)P.goff[j], nullptr});
                    anwg += (t.N * ((Lj + 1) / 2) + NC - 1) / NC;
                }
                if (!upload(P, P.atab, at)) return S2DW_E_NOMEM;
                P.ans = (int)at.size();
                P.anwg = anwg;
            }
        }
    }
    for (int Psz : sizes) {
        if (P.twP.count(Psz)) continue;
        std::vector<double2> tw(Psz);
        for (int k = 0; k < Psz; ++k) {
            const ld a = -2.0L * kPiL * k / Psz;
            tw[k] = make_double2((double)cosl(a), (double)sinl(a));
        }
        double2 *d = nullptr;
        if (!upload(P, d, tw)) return S2DW_E_NOMEM;
        P.twP[Psz] = d;
    }
    // workspaces
    int maxLj = 0;
    for (int j = 0; j < t.S; ++j) maxLj = std::max(maxLj, P.sc.Lj[j]);
    P.s_fpad = (size_t)L * Lp;
    P.s_U = (size_t)std::max<int64_t>(off, 1);
    P.s_Ub = (size_t)t.N * P.nb * std::max(maxLj, 1);
    P.s_Y = (size_t)P.Nh * P.nb * M;
    P.cur.chunk = default_chunk(P);
    out = pl.release();
    return S2DW_OK;
}

// FP32 copy of a device table of n complex (or, with real = true, n real) FP64 values.
template <typename F>
bool f32_copy(Plan &P, F *&dst, const void *src, size_t n_values) {
    if (!dalloc(P, dst, n_values)) return false;
    const size_t words = n_values * sizeof(F) / sizeof(float);
    return launch_to_f32((const double *)src, (float *)dst, words, 0) == hipSuccess;
}

// Builds the FP32 table set of a plan (once; caller holds g_mu).
int ensure_f32(Plan &P) {
    if (P.f32_ready) return S2DW_OK;
    const int S = P.S;
    bool ok = f32_copy(P, P.tgff, P.tgf, P.n_tg) && f32_copy(P, P.tgaf, P.tga, P.n_tg) &&
              f32_copy(P, P.kb2f, P.kb2, P.n_kb2);
    for (auto &kv : P.gt) {
        if (!ok) break;
        const int T = 2 * kv.first - 1;
        Plan::GridTab &g = kv.second;
        ok = f32_copy(P, g.csqf, g.csq, T) && f32_copy(P, g.cppf, g.cpp, T) && f32_copy(P, g.hD1f, g.hD1, g.PD) &&
             f32_copy(P, g.ephf, g.eph, T);
        if (ok && g.pcs) ok = f32_copy(P, g.pcsf, g.pcs, g.npcs);
    }
    if (ok && P.grid == S2DW_GRID_DH)
        ok = f32_copy(P, P.dh_csqf, P.dh_csq, P.nb) && f32_copy(P, P.dh_cppf, P.dh_cpp, 2 * P.L - 1) &&
             f32_copy(P, P.dh_qf, P.dh_q, P.nb);
    P.hAf.assign(S, nullptr);
    P.hBf.assign(S, nullptr);
    P.hCf.assign(S, nullptr);
    P.hD2f.assign(S, nullptr);
    P.hEf.assign(S, nullptr);
    P.hBbf.assign(S, nullptr);
    P.hCbf.assign(S, nullptr);
    for (int j = 0; ok && j < S; ++j) {
        if (P.sc.Lj[j] == 0) continue;
        const int PD = P.gt[P.Lg[j]].PD;
        ok = f32_copy(P, P.hAf[j], P.hA[j], P.PA[j]) && f32_copy(P, P.hBf[j], P.hB[j], P.PB[j]) &&
             f32_copy(P, P.hCf[j], P.hC[j], P.PB[j]) && f32_copy(P, P.hD2f[j], P.hD2[j], PD);
        if (ok && P.hE[j]) ok = f32_copy(P, P.hEf[j], P.hE[j], P.PE[j]);
        if (ok && P.hBb[j])
            ok = f32_copy(P, P.hBbf[j], P.hBb[j], P.PBb[j]) && f32_copy(P, P.hCbf[j], P.hCb[j], P.PBb[j]);
    }
    if (ok && P.mj0 >= 0) {
        std::vector<BetaAdjScale> tab(P.mns);
        ok = hipMemcpy(tab.data(), P.mtab, sizeof(BetaAdjScale) * P.mns, hipMemcpyDeviceToHost) == hipSuccess;
        for (int i = 0, j = P.mj0; ok && j < P.S; ++j)
            if (P.sc.Lj[j] > 0) tab[i++].hh2 = P.hD2f[j];
        ok = ok && upload(P, P.mtabf, tab);
    }
    for (auto &kv : P.twP) {
        if (!ok) break;
        float2 *d = nullptr;
        ok = f32_copy(P, d, kv.second, kv.first);
        P.twPf[kv.first] = d;
    }
    if (!ok) return S2DW_E_NOMEM;
    if (hipStreamSynchronize(0) != hipSuccess) return S2DW_E_DEVICE;
    P.f32_ready = true;
    return S2DW_OK;
}

// The plan of these parameters if it was built before (and, with f32, its FP32 tables too),
// else null; builds nothing.
Plan *find_plan(int L, int N, double lam, int J_min, bool f32, int grid) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(PlanKey(kWavelet, L, N, lam, J_min, grid));
    if (it == g_plans.end()) return nullptr;
    if (f32 && !it->second->f32_ready) return nullptr;
    return it->second.get();
}

int get_plan(int kind, int L, int N, double lam, int J_min, Plan *&out, bool f32 = false, int grid = S2DW_GRID_MW) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (kind != kWavelet) grid = S2DW_GRID_MW;
    PlanKey key(kind, L, kind == kWavelet ? N : 1, kind == kWavelet ? lam : 0.0, kind == kWavelet ? J_min : 0, grid);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        out = it->second.get();
        return f32 ? ensure_f32(*out) : S2DW_OK;
    }
    Plan *p = nullptr;
    int rc = build_plan(kind, L, N, lam, J_min, grid, p);
    if (rc != S2DW_OK) return rc;
    g_plans[key].reset(p);
    out = p;
    return f32 ? ensure_f32(*out) : S2DW_OK;
}

template <typename T>
bool walloc(Work &w, T *&p, size_t count) {
    p = nullptr;
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
    w.allocs.push_back(q);
    w.bytes += count * sizeof(T);
    p = (T *)q;
    return true;
}

// The workspace of `stream` for a batch of `maps` maps with per-map partial sums of s_F
// elements (grown on demand: the first call on a stream, a larger batch or a larger
// partial-sum layout allocates; the old buffers are freed after that stream drains, and only
// calls on that stream use them).
int get_work(Plan &P, hipStream_t stream, int maps, size_t s_F, Work *&out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto &slot = P.work[(void *)stream];
    if (slot && slot->cap >= maps && slot->s_F >= s_F) {
        out = slot.get();
        return S2DW_OK;
    }
    if (slot) {
        if (hipStreamSynchronize(stream) != hipSuccess) return S2DW_E_DEVICE;
        slot.reset();
    }
    std::unique_ptr<Work> w(new (std::nothrow) Work());
    if (!w) return S2DW_E_NOMEM;
    const size_t n = (size_t)maps;
    if (!walloc(*w, w->fpad, n * P.s_fpad) || !walloc(*w, w->U, n * P.s_U) || !walloc(*w, w->Ub, n * P.s_Ub) ||
        !walloc(*w, w->Y, n * P.s_Y) || !walloc(*w, w->Fpart, n * s_F))
        return S2DW_E_NOMEM;
    w->cap = maps;
    w->s_F = s_F;
    slot = std::move(w);
    out = slot.get();
    return S2DW_OK;
}

int check_params(const s2dw_params *p) {
    if (!p) return S2DW_E_ARG;
    if (p->L < 2 || p->L > 4096) return S2DW_E_ARG;
    if (p->L > 2048) return S2DW_E_UNSUPPORTED;
    if (p->N < 1 || p->N > p->L || p->N > 2 * kMaxK) return S2DW_E_ARG;
    if (!(p->lambda > 1.0) || !std::isfinite(p->lambda)) return S2DW_E_ARG;
    int JL = jmax_of(p->L, p->lambda);
    if (p->J_min < 0 || p->J_min > JL || JL - p->J_min + 1 > kMaxScales) return S2DW_E_ARG;
    if (p->grid != S2DW_GRID_MW && p->grid != S2DW_GRID_MW_MULTIRES && p->grid != S2DW_GRID_DH) return S2DW_E_ARG;
    if (p->precision != S2DW_FP64 && p->precision != S2DW_MIXED) return S2DW_E_ARG;
    if (p->reality != 0 && p->reality != 1) return S2DW_E_ARG;
    return S2DW_OK;
}

bool aligned(const void *p) { return ((uintptr_t)p & 7u) == 0; }

// Grid band-limit of every scale of a valid parameter set (L for the full-resolution grid,
// the scale's own band-limit for the multiresolution one); host tables only, cached.
int grid_limits(const s2dw_params *p, std::vector<int> &Lg) {
    static std::map<std::tuple<int, int, double, int>, std::vector<int>> cache;
    std::vector<int> bl;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto key = std::make_tuple(p->L, p->N, p->lambda, p->J_min);
        auto it = cache.find(key);
        if (it != cache.end()) {
            bl = it->second;
        } else {
            HostTables t;
            if (!build_wavelet_tables(p->L, p->N, p->lambda, p->J_min, t)) return S2DW_E_ARG;
            for (int j = 0; j < t.S; ++j) bl.push_back(t.hi[j] >= t.lo[j] ? t.hi[j] + 1 : 0);
            cache[key] = bl;
        }
    }
    Lg.resize(bl.size());
    for (size_t j = 0; j < bl.size(); ++j) Lg[j] = p->grid == S2DW_GRID_MW_MULTIRES ? bl[j] : p->L;
    return S2DW_OK;
}

#define S2DW_CHECK_HIP(x)                               \
    do {                                                \
        if ((x) != hipSuccess) return S2DW_E_DEVICE;    \
    } while (0)

// Whether scale j of the analysis (synthesis) takes the fused prime-factor alpha and gamma
// kernel; the caller has checked that it applies (pfa_fused, real signals).  The default
// follows measurements at L = 1024, N = 8 and L = 2048, N = 4: the fused analysis kernel
// costs the same at every L_j and beats the two-pass form except on the scales with the
// blocked alpha transforms at T = 2047; the fused synthesis kernel wins at T = 4095, and at
// T = 2047 where it holds every order's gamma sums in registers (below 128 for them: not
// FP64 with more than two orders), else its second sweep over W costs more than it saves.
bool fuse_fwd(const Plan &P, const Shape &sh, int j, int T) {
    if (sh.fuse != 1) return sh.fuse == 2;
    return T == 4095 || P.nblkb[j] <= 1;
}
bool fuse_adj(const Plan &P, const Shape &sh, int f32, int T) {
    if (sh.fuse != 1) return sh.fuse == 2;
    return T == 4095 || f32 || P.Nh <= 2;
}

// Coarse scales of real signals take the fused alpha and gamma passes (the analysis one
// in both precisions: it computes in FP64 and reads and writes Ub and W in the plan's
// precision; the synthesis one in FP64) while Nh (2Lj - 1) stays within 9 G and 256 (the
// outputs of a ring in the synthesis pass, at most one per thread).  Nh (2Lj - 1) is the number of complex
// multiply-adds per sample, G the number of W values a sample writes or reads: the passes
// then cost little more than their W traffic, against a blocked alpha transform plus a
// gamma pass that also writes and reads Y or X (at L = 1024, N = 8, for Lj = 4, 8, 16:
// analysis 65-73 us per scale, synthesis 57-113 us, against about 130 us each).
bool direct_alpha_gamma(int Nh, int G, int Lj, bool cx) {
    const int terms = Nh * (2 * Lj - 1);
    return !cx && terms <= 9 * G && terms <= 256 && 2 * Nh * Lj <= kAlphaGammaCoeffs;
}

// Wigner-stage analysis + beta/alpha/gamma sums for a batch of `maps` maps: f_lm of map i at
// flm + i L^2, its W at W + i S (2N-1) L (2L-1) (elements of the W type).
// With cx (complex signals), flm holds maps / 2 complex signals, each run as the two real maps
// 2z, 2z + 1 (real and imaginary part on the sphere), and W holds maps / 2 complex arrays
// ((re, im) pairs, same per-map layout).
int run_inverse(Plan &P, const Shape &sh, Work &w, int maps, const double2 *flm, void *W, int f32, hipStream_t st,
                bool cx = false) {
    const int L = P.L;
    {
        Stage sg("pad", st);
        if (cx) S2DW_CHECK_HIP(launch_pad_flm_complex(flm, P.gsc, w.fpad, L, P.Lp, P.s_fpad, maps / 2, st));
        else S2DW_CHECK_HIP(launch_pad_flm(flm, P.gsc, w.fpad, L, P.Lp, P.s_fpad, maps, st));
    }
    WigFwdArgs a{};
    a.fpad = w.fpad;
    a.pq = P.pq;
    a.uv = P.uv;
    a.kb2 = P.kb2;
    a.seed = P.seed;
    a.seedm = P.seedm;
    a.seede = P.seede;
    a.U = w.U;
    a.s_fpad = P.s_fpad;
    a.s_U = P.s_U;
    a.L = L;
    a.Lp = P.Lp;
    a.N = P.ht.N;
    a.eoff = P.eoff;
    for (int k = 0; k < P.K; ++k) a.nk[k] = P.ht.nk[k];
    a.seg = P.seg;
    a.sc = P.sc;
    {
        Stage sg("wigner_fwd", st);
        a.tiles = sh.tiles_fwd;
        a.nplain = sh.nfwd_plain;
        S2DW_CHECK_HIP(launch_wig_fwd(a, P.K, sh.R, sh.nfwd_plain + sh.nfwd_x, maps, st));
    }
    const int N = P.ht.N;
    const size_t per_map = P.woff[P.S];  // elements of one W (complex ones with cx)
    const size_t ew = (f32 ? 4 : 8) * (cx ? 2 : 1);
    const int wmaps = cx ? maps / 2 : maps;
    for (int j = 0; j < P.S; ++j) {
        const int Lj = P.sc.Lj[j], Lg = P.Lg[j];
        const size_t per_scale = P.woff[j + 1] - P.woff[j];
        void *Wj = (char *)W + P.woff[j] * ew;
        if (Lj == 0) {
            for (int i = 0; i < wmaps; ++i)
                S2DW_CHECK_HIP(launch_zero_words((char *)Wj + per_map * ew * i, per_scale * ew / 4, st));
            continue;
        }
        const Plan::GridTab &gtab = P.gt[Lg];
        // coarse scales: the beta stage of all of them in one launch at the first, each scale's
        // Ub at goff[j]
        const bool bmerged = P.ans > 0 && j >= P.mj0 && gtab.pcs && P.grid == S2DW_GRID_MW;
        void *ubj = bmerged ? (f32 ? (void *)((float2 *)w.Ub + P.goff[j]) : (void *)(w.Ub + P.goff[j])) : (void *)w.Ub;
        StageArgs b{};
        b.f32 = f32;
        b.in = w.U + P.sc.off[j];
        b.out = w.Ub;
        b.s_in = P.s_U;
        b.s_out = P.s_Ub;
        b.hh = f32 ? (const void *)P.hAf[j] : P.hA[j];
        b.tw = f32 ? (const void *)P.twPf[P.PA[j]] : P.twP[P.PA[j]];
        const bool dh = P.grid == S2DW_GRID_DH;
        b.csq = dh ? (f32 ? (const void *)P.dh_csqf : P.dh_csq) : (f32 ? (const void *)gtab.csqf : gtab.csq);
        b.cpp = dh ? (f32 ? (const void *)P.dh_cppf : P.dh_cpp) : (f32 ? (const void *)gtab.cppf : gtab.cpp);
        b.L = Lg;
        b.nb = dh ? P.nb : Lg;
        b.Lj = Lj;
        b.N = N;
        b.Nh = P.Nh;
        {
            Stage sg("beta_fwd", st);
            // two columns per transform: as a prime-factor transform of length T where T is one
            // of its lengths, else as a chirp convolution where that needs no larger transform
            // than one column's (equiangular grid)
            if (bmerged) {
                if (j == P.mj0) {
                    StageArgs bm = b;
                    bm.in = w.U;
                    bm.eph = f32 ? (const void *)gtab.ephf : gtab.eph;
                    bm.pcs = f32 ? (const void *)gtab.pcsf : gtab.pcs;
                    S2DW_CHECK_HIP(launch_beta_fwd_pfa_multi(bm, P.atab, P.ans, P.anwg, maps, st));
                }
            } else if (!dh && gtab.pcs) {
                b.eph = f32 ? (const void *)gtab.ephf : gtab.eph;
                b.pcs = f32 ? (const void *)gtab.pcsf : gtab.pcs;
                S2DW_CHECK_HIP(launch_beta_fwd_pfa(b, maps, st));
            } else if (!dh && pow2_at_least(2 * Lj + 2 * Lg - 3) <= P.PA[j])
                S2DW_CHECK_HIP(launch_beta_fwd_pair(b, P.PA[j], maps, st));
            else
                S2DW_CHECK_HIP(launch_beta_fwd_fft(b, P.PA[j], maps, st));
        }
        if (direct_alpha_gamma(P.Nh, P.ng, Lj, cx)) {
            AlphaGammaArgs d{};
            d.in = ubj;
            d.wout = Wj;
            d.tg = P.tgf;
            d.eph = gtab.eph;
            d.s_in = P.s_Ub;
            d.s_w = per_map;
            d.nb = b.nb;
            d.T = 2 * Lg - 1;
            d.Lj = Lj;
            d.N = N;
            d.Nh = P.Nh;
            d.G = P.ng;
            d.f32 = f32;
            Stage sg("alpha_gamma_fwd", st);
            S2DW_CHECK_HIP(launch_alpha_gamma_fwd(d, maps, st));
            continue;
        }
        if (gtab.pcs && !cx && pfa_fused(2 * Lg - 1, P.Nh) && fuse_fwd(P, sh, j, 2 * Lg - 1)) {
            // the alpha and gamma passes in one prime-factor kernel, one beta ring per workgroup
            StageArgs d = b;
            d.in = ubj;
            d.s_in = P.s_Ub;
            d.pcs = f32 ? (const void *)gtab.pcsf : gtab.pcs;
            d.wout = Wj;
            d.s_w = per_map;
            d.tg = f32 ? (const void *)P.tgff : P.tgf;
            d.G = P.ng;
            Stage sg("alpha_gamma_fwd", st);
            S2DW_CHECK_HIP(launch_alpha_gamma_fwd_pfa(d, maps, st));
            continue;
        }
        StageArgs c = b;
        c.in = ubj;
        c.out = w.Y;
        c.s_in = P.s_Ub;
        c.s_out = P.s_Y;
        c.hh = f32 ? (const void *)P.hBf[j] : P.hB[j];
        c.tw = f32 ? (const void *)P.twPf[P.PB[j]] : P.twP[P.PB[j]];
        c.csq = f32 ? (const void *)gtab.csqf : gtab.csq;
        c.cpp = f32 ? (const void *)gtab.cppf : gtab.cpp;
        if (P.nblkb[j] > 1) {
            c.hh = f32 ? (const void *)P.hBbf[j] : P.hBb[j];
            c.tw = f32 ? (const void *)P.twPf[P.PBb[j]] : P.twP[P.PBb[j]];
            c.eph = f32 ? (const void *)gtab.ephf : gtab.eph;
            c.nblk = P.nblkb[j];
            c.B = P.Bb[j];
            Stage sg("alpha_fwd", st);
            S2DW_CHECK_HIP(launch_alpha_fwd_blk(c, P.PBb[j], maps, st));
        } else if (gtab.pcs) {
            c.pcs = f32 ? (const void *)gtab.pcsf : gtab.pcs;
            Stage sg("alpha_fwd", st);
            S2DW_CHECK_HIP(launch_alpha_fwd_pfa(c, maps, st));
        } else {
            Stage sg("alpha_fwd", st);
            S2DW_CHECK_HIP(launch_alpha_fwd_fft(c, P.PB[j], maps, st));
        }
        GammaArgs g{};
        g.wout = Wj;
        g.in = w.Y;
        g.s_w = per_map;
        g.s_y = P.s_Y;
        g.tg = f32 ? (const void *)P.tgff : P.tgf;
        g.L = b.nb;
        g.T = 2 * Lg - 1;
        g.G = P.ng;
        g.Nh = P.Nh;
        g.f32 = f32;
        {
            Stage sg("gamma_fwd", st);
            if (cx) S2DW_CHECK_HIP(launch_gamma_fwd_cx(g, wmaps, st));
            else S2DW_CHECK_HIP(launch_gamma_fwd(g, maps, st));
        }
    }
    return S2DW_OK;
}

// gamma/alpha/beta quadratures + Wigner-stage contraction for a batch: W -> f_lm (same
// per-map layout as run_inverse; wphi of map i at wphi + i L^2, or null).
// With cx, W holds maps / 2 complex arrays; real map 2z (2z + 1) is the real (imaginary) part
// of complex array z, and f_lm of real map k goes to flm + k L^2.
int run_forward(Plan &P, const Shape &sh, Work &w, int maps, const void *W, const double2 *wphi, double2 *flm,
                int f32, hipStream_t st, bool cx = false) {
    const int L = P.L, N = P.ht.N;
    const size_t per_map = P.woff[P.S];
    const size_t ew = (f32 ? 4 : 8) * (cx ? 2 : 1);
    for (int j = 0; j < P.S; ++j) {
        const int Lj = P.sc.Lj[j], Lg = P.Lg[j], M = 2 * Lg - 1;
        if (Lj == 0) continue;
        const Plan::GridTab &gtab = P.gt[Lg];
        const void *Wj = (const char *)W + P.woff[j] * ew;
        GammaArgs g{};
        g.win = Wj;
        g.out = w.Y;
        g.s_w = per_map;
        g.s_y = P.s_Y;
        const bool dh = P.grid == S2DW_GRID_DH;
        g.tg = f32 ? (const void *)P.tgaf : P.tga;
        g.L = dh ? P.nb : Lg;
        g.T = M;
        g.G = P.ng;
        g.Nh = P.Nh;
        g.f32 = f32;
        const bool merged = P.mj0 >= 0 && j >= P.mj0;  // synthesis beta stage in the coarse-scale launch
        void *gout = !merged ? (void *)w.Ub
                             : (f32 ? (void *)((float2 *)w.Ub + P.goff[j]) : (void *)(w.Ub + P.goff[j]));
        const double qscale = (2.0 * M_PI / M) * (2.0 * M_PI / P.ng);  // alpha and gamma quadrature weights
        // FP64 only: the fused pass computes in FP64 and is bound by its arithmetic at the
        // larger Lj, where the FP32 passes of the mixed path are cheaper
        const bool fused = direct_alpha_gamma(P.Nh, P.ng, Lj, cx) && !f32;
        const bool fused_pfa = !fused && gtab.pcs && !cx && pfa_fused(M, P.Nh) && fuse_adj(P, sh, f32, M);
        if (fused_pfa) {
            StageArgs d{};
            d.f32 = f32;
            d.win = Wj;
            d.s_w = per_map;
            d.tg = f32 ? (const void *)P.tgaf : P.tga;
            d.G = P.ng;
            d.out = gout;
            d.s_out = P.s_Ub;
            d.pcs = f32 ? (const void *)gtab.pcsf : gtab.pcs;
            d.L = Lg;
            d.nb = g.L;
            d.Lj = Lj;
            d.N = N;
            d.Nh = P.Nh;
            d.scale = qscale;
            Stage sg("gamma_alpha_adj", st);
            S2DW_CHECK_HIP(launch_gamma_alpha_adj_pfa(d, maps, st));
        } else if (fused) {
            GammaAlphaArgs d{};
            d.win = Wj;
            d.out = gout;
            d.tg = P.tga;
            d.eph = gtab.eph;
            d.s_w = per_map;
            d.s_out = P.s_Ub;
            d.nb = g.L;
            d.T = M;
            d.Lj = Lj;
            d.N = N;
            d.Nh = P.Nh;
            d.G = P.ng;
            d.scale = qscale;
            d.f32 = f32;
            Stage sg("gamma_alpha_adj", st);
            S2DW_CHECK_HIP(launch_gamma_alpha_adj(d, maps, st));
        } else {
            Stage sg("gamma_adj", st);
            if (cx) S2DW_CHECK_HIP(launch_gamma_adj_cx(g, maps / 2, st));
            else S2DW_CHECK_HIP(launch_gamma_adj(g, maps, st));
        }
        StageArgs c{};
        c.f32 = f32;
        c.in = w.Y;
        c.out = gout;
        c.s_in = P.s_Y;
        c.s_out = P.s_Ub;
        c.hh = f32 ? (const void *)P.hCf[j] : P.hC[j];
        c.tw = f32 ? (const void *)P.twPf[P.PB[j]] : P.twP[P.PB[j]];
        c.csq = f32 ? (const void *)gtab.csqf : gtab.csq;
        c.cpp = f32 ? (const void *)gtab.cppf : gtab.cpp;
        c.L = Lg;
        c.nb = g.L;
        c.Lj = Lj;
        c.N = N;
        c.Nh = P.Nh;
        c.K = P.K;
        c.scale = qscale;
        if (fused || fused_pfa) {
            // the alpha quadrature ran in the fused pass above
        } else if (P.nblkb[j] <= 1 && gtab.pcs) {
            StageArgs cp = c;
            cp.pcs = f32 ? (const void *)gtab.pcsf : gtab.pcs;
            Stage sg("alpha_adj", st);
            S2DW_CHECK_HIP(launch_alpha_adj_pfa(cp, maps, st));
        } else if (P.nblkb[j] > 1) {
            StageArgs cb = c;
            cb.hh = f32 ? (const void *)P.hCbf[j] : P.hCb[j];
            cb.tw = f32 ? (const void *)P.twPf[P.PBb[j]] : P.twP[P.PBb[j]];
            cb.eph = f32 ? (const void *)gtab.ephf : gtab.eph;
            cb.nblk = P.nblkb[j];
            cb.B = P.Bb[j];
            Stage sg("alpha_adj", st);
            S2DW_CHECK_HIP(launch_alpha_adj_blk(cb, P.PBb[j], maps, st));
        } else {
            Stage sg("alpha_adj", st);
            S2DW_CHECK_HIP(launch_alpha_adj_fft(c, P.PB[j], maps, st));
        }
        if (merged) continue;
        StageArgs v = c;
        v.in = w.Ub;
        v.s_in = P.s_Ub;
        // V of scale j starts sc.off[j] complex elements into the workspace (the synthesis
        // Wigner kernel indexes it with the same element type); per-map stride s_U elements
        v.out = f32 ? (void *)((float2 *)w.U + P.sc.off[j]) : (void *)(w.U + P.sc.off[j]);
        v.s_out = P.s_U;
        for (int k = 0; k < P.K; ++k) v.nk[k] = P.ht.nk[k];
        v.eta_imag = P.ht.eta_imag ? 1 : 0;
        if (dh) {
            v.csq = f32 ? (const void *)P.dh_csqf : P.dh_csq;
            v.cpp = f32 ? (const void *)P.dh_cppf : P.dh_cpp;
            v.qw = f32 ? (const void *)P.dh_qf : P.dh_q;
            v.hh = f32 ? (const void *)P.hEf[j] : P.hE[j];
            v.tw = f32 ? (const void *)P.twPf[P.PE[j]] : P.twP[P.PE[j]];
            Stage sg("beta_adj", st);
            S2DW_CHECK_HIP(launch_beta_adj_dh(v, P.PE[j], maps, st));
        } else {
            v.hh = f32 ? (const void *)gtab.hD1f : gtab.hD1;
            v.hh2 = f32 ? (const void *)P.hD2f[j] : P.hD2[j];
            v.eph = f32 ? (const void *)gtab.ephf : gtab.eph;
            v.pcs = f32 ? (const void *)gtab.pcsf : gtab.pcs;
            v.tw = f32 ? (const void *)P.twPf[gtab.PD] : P.twP[gtab.PD];
            Stage sg("beta_adj", st);
            S2DW_CHECK_HIP(launch_beta_adj_fft(v, gtab.PD, maps, st));
        }
    }
    if (P.mj0 >= 0) {
        const Plan::GridTab &gtab = P.gt[L];
        StageArgs v{};
        v.f32 = f32;
        v.in = w.Ub;
        v.out = w.U;
        v.s_in = P.s_Ub;
        v.s_out = P.s_U;
        v.csq = f32 ? (const void *)gtab.csqf : gtab.csq;
        v.cpp = f32 ? (const void *)gtab.cppf : gtab.cpp;
        v.hh = f32 ? (const void *)gtab.hD1f : gtab.hD1;
        v.tw = f32 ? (const void *)P.twPf[gtab.PD] : P.twP[gtab.PD];
        v.eph = f32 ? (const void *)gtab.ephf : gtab.eph;
        v.pcs = f32 ? (const void *)gtab.pcsf : gtab.pcs;
        v.L = L;
        v.nb = L;
        v.N = N;
        v.Nh = P.Nh;
        v.K = P.K;
        for (int k = 0; k < P.K; ++k) v.nk[k] = P.ht.nk[k];
        v.eta_imag = P.ht.eta_imag ? 1 : 0;
        Stage sg("beta_adj", st);
        S2DW_CHECK_HIP(launch_beta_adj_multi(v, f32 ? P.mtabf : P.mtab, P.mns, P.mnwg, gtab.PD, maps, st));
    }
    WigAdjArgs a{};
    a.pq = P.pq;
    a.uv = P.uv;
    a.kb2 = f32 ? (const void *)P.kb2f : P.kb2;
    a.seed = P.seed;
    a.seedm = P.seedm;
    a.seede = P.seede;
    a.V = w.U;
    a.Fpart = w.Fpart;
    a.s_V = P.s_U;
    a.s_F = sh.s_F;
    a.L = L;
    a.Lp = P.Lp;
    a.group = sh.group;
    a.f32 = f32;
    a.seg = P.seg;
    a.sc = P.sc;
    {
        Stage sg("wigner_adj", st);
        a.tiles = sh.tiles_adj;
        a.nplain = sh.nadj_plain;
        S2DW_CHECK_HIP(launch_wig_adj(a, P.K, sh.R, sh.nadj_plain + sh.nadj_x, maps, st));
    }
    {
        Stage sg("syn_final", st);
        S2DW_CHECK_HIP(launch_syn_final(w.Fpart, sh.s_F, f32, sh.nblk, sh.group, P.Lmax, P.fac, P.gsc, wphi, P.phi, flm,
                                        L, P.Lp, maps, st));
    }
    return S2DW_OK;
}

// ------------------------------------------------------------------ persistent executor
// The work list of a persistent batch is recorded from run_inverse / run_forward (kernels.h),
// one parameter set ("group") at a time, with a shape of its own: Wigner tiles of
// persist_slots(K) m' slots and four-wave synthesis workgroups (m' groups of 4R).  Each group
// has its own workspaces (count maps), held by the program.

struct PGroup {
    Plan *P = nullptr;
    int count = 0;
    const void *flm = nullptr;
    void *W = nullptr, *wphi = nullptr;
};

struct PProgram {
    struct Part {
        PJob *jobs = nullptr;
        PEnt *ents = nullptr;
        int *qoff = nullptr, *qn = nullptr;
        unsigned char *args = nullptr;
        int *ctr = nullptr;
        PState *state = nullptr;
        int njobs = 0, nitems = 0, nctr = 0, workers = 0, chunk = 1;
    };
    int dir = 0, f32 = 0;
    Part part[2];
    std::vector<std::unique_ptr<Work>> works;
    std::vector<void *> allocs;
    ~PProgram() {
        for (void *q : allocs) hipFree(q);
    }
    template <class T>
    bool alloc(T *&p, size_t count) {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
        allocs.push_back(q);
        p = (T *)q;
        return true;
    }
};

std::map<std::string, std::unique_ptr<PProgram>> g_programs;  // under g_mu
int g_spin_limit = 0;                                           // 0: the default bound
int g_wait_extra = 0;                                           // 1: waits never satisfied (tests)

constexpr int kDefaultSpinLimit = 1 << 24;  // polls of about 0.2 us: a few seconds

// The persistent shape of a plan (caller holds g_mu): tiles built once and kept.
int persist_shape(Plan &P, Shape &sh) {
    const int R = persist_slots(P.K);
    const int key = -R;  // tile sets of the persistent shape, beside the ordinary ones
    auto it = P.tilesets.find(key);
    if (it == P.tilesets.end()) {
        Plan::TileSet ts;
        std::vector<int2> pl_a, x_a, pl_s, x_s;
        build_tiles(P, P.seede_h, P.Lp, 4 * R, pl_a, x_a);
        build_tiles(P, P.seede_h, P.Lp, 4 * R, pl_s, x_s);
        ts.nfwd_plain = (int)pl_a.size();
        ts.nfwd_x = (int)x_a.size();
        ts.nadj_plain = (int)pl_s.size();
        ts.nadj_x = (int)x_s.size();
        pl_a.insert(pl_a.end(), x_a.begin(), x_a.end());
        pl_s.insert(pl_s.end(), x_s.begin(), x_s.end());
        if (!upload(P, ts.fwd, pl_a) || !upload(P, ts.adj, pl_s)) return S2DW_E_NOMEM;
        it = P.tilesets.emplace(key, ts).first;
    }
    const Plan::TileSet &ts = it->second;
    sh = P.cur;
    sh.R = R;
    sh.tiles_fwd = ts.fwd;
    sh.tiles_adj = ts.adj;
    sh.nfwd_plain = ts.nfwd_plain;
    sh.nfwd_x = ts.nfwd_x;
    sh.nadj_plain = ts.nadj_plain;
    sh.nadj_x = ts.nadj_x;
    sh.group = 4 * R;
    sh.nblk = (P.L + sh.group - 1) / sh.group;
    sh.s_F = (size_t)sh.nblk * P.L * P.Lp;
    sh.fuse = 0;
    return S2DW_OK;
}

// Records the launch sequence of every group and lays out the program's two parts.
int build_program(PProgram &pr, int dir, int f32, const std::vector<PGroup> &gs, hipStream_t st) {
    pr.dir = dir;
    pr.f32 = f32;
    std::vector<std::vector<RecJob>> rec(gs.size());
    for (size_t g = 0; g < gs.size(); ++g) {
        Plan &P = *gs[g].P;
        Shape sh;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            int rc = persist_shape(P, sh);
            if (rc != S2DW_OK) return rc;
        }
        std::unique_ptr<Work> w(new (std::nothrow) Work());
        if (!w) return S2DW_E_NOMEM;
        const size_t n = (size_t)gs[g].count;
        if (!walloc(*w, w->fpad, n * P.s_fpad) || !walloc(*w, w->U, n * P.s_U) || !walloc(*w, w->Ub, n * P.s_Ub) ||
            !walloc(*w, w->Y, n * P.s_Y) || !walloc(*w, w->Fpart, n * sh.s_F))
            return S2DW_E_NOMEM;
        w->cap = gs[g].count;
        w->s_F = sh.s_F;
        Recorder R;
        t_rec = &R;
        t_no_events = true;
        int rc;
        if (dir == 0) {
            rc = run_inverse(P, sh, *w, gs[g].count, (const double2 *)gs[g].flm, gs[g].W, f32, st);
            if (rc == S2DW_OK && gs[g].wphi &&
                launch_scaling((const double2 *)gs[g].flm, P.phi, (double2 *)gs[g].wphi, P.L, gs[g].count, st) !=
                    hipSuccess)
                rc = S2DW_E_DEVICE;
        } else {
            rc = run_forward(P, sh, *w, gs[g].count, gs[g].W, (const double2 *)gs[g].wphi, (double2 *)gs[g].flm, f32,
                             st);
        }
        t_rec = nullptr;
        t_no_events = false;
        // while recording, a failed launch is a stage the executor does not run
        if (rc != S2DW_OK) return rc == S2DW_E_DEVICE ? S2DW_E_UNSUPPORTED : rc;
        rec[g] = std::move(R.jobs);
        pr.works.push_back(std::move(w));
    }
    for (int part = 0; part < 2; ++part) {
        // the part's jobs of every group, with their position in the group's sequence; each job
        // of a full batch (maps = count) depends on the group's previous such job in the part,
        // the others (per-map clears of empty scales) on nothing
        struct E {
            int g, pos;
            const RecJob *j;
        };
        std::vector<E> es;
        for (size_t g = 0; g < gs.size(); ++g) {
            int pos = 0;
            for (const RecJob &j : rec[g])
                if (persist_part(j.kind) == part) es.push_back({(int)g, pos++, &j});
        }
        std::stable_sort(es.begin(), es.end(), [](const E &a, const E &b) { return a.pos < b.pos; });
        std::vector<int> last(gs.size(), -1);
        std::vector<PJob> jobs(es.size());
        std::vector<unsigned char> args;
        std::vector<double> work(gs.size(), 0.0);  // per map of each group: threads x workgroups
        int ctr0 = 0;
        long long nitems = 0;
        for (size_t i = 0; i < es.size(); ++i) {
            const RecJob &r = *es[i].j;
            const int g = es[i].g;
            PJob &J = jobs[i];
            const bool main = r.maps == gs[g].count;
            J.kind = r.kind;
            if (r.gx < 1 || r.gx > (1 << 30) || r.nt < 1 || r.nt > 256 || 256 % r.nt) return S2DW_E_UNSUPPORTED;
            J.gx = (int)r.gx;
            J.nt = r.nt;
            const int per = 256 / r.nt;
            const int wg = (J.gx + per - 1) / per;  // worker rounds per map
            // at least four worker rounds per item (the fixed costs of an item: its ticket, its
            // entry, the wait and the signal of its run), at most 256 items per map and job
            J.rounds = std::max((wg + 255) / 256, std::min(wg, 4));
            J.nx = (wg + J.rounds - 1) / J.rounds;
            J.maps = r.maps;
            J.prev = main ? last[g] : -1;
            if (main) last[g] = (int)i;
            J.ctr0 = ctr0;
            while (args.size() % 16) args.push_back(0);
            J.arg = args.size();
            args.insert(args.end(), r.args.begin(), r.args.end());
            ctr0 += J.maps;
            nitems += (long long)J.nx * J.maps;
            if (main) work[g] += (double)r.gx * r.nt;
        }
        if (nitems > (1 << 30)) return S2DW_E_UNSUPPORTED;
        // maps to queues, heaviest first to the least loaded (every map's jobs in one queue)
        std::vector<std::vector<int>> qof(gs.size());
        {
            std::vector<std::pair<double, std::pair<int, int>>> ms;
            for (size_t g = 0; g < gs.size(); ++g) {
                qof[g].assign(gs[g].count, 0);
                for (int z = 0; z < gs[g].count; ++z) ms.push_back({work[g], {(int)g, z}});
            }
            std::stable_sort(ms.begin(), ms.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
            double load[kPersistQueues] = {};
            for (const auto &m : ms) {
                const int q = (int)(std::min_element(load, load + kPersistQueues) - load);
                load[q] += m.first;
                qof[m.second.first][m.second.second] = q;
            }
        }
        // entries of each queue in job order (jobs with one map but a larger batch, the
        // per-map clears of empty scales, go to queue 0)
        std::vector<std::vector<PEnt>> qe(kPersistQueues);
        std::vector<int> qitems(kPersistQueues, 0);
        for (size_t i = 0; i < es.size(); ++i) {
            const int g = es[i].g;
            const PJob &J = jobs[i];
            for (int z = 0; z < J.maps; ++z) {
                const int q = J.maps == gs[g].count ? qof[g][z] : 0;
                qe[q].push_back(PEnt{(int)i, z, qitems[q], 0});
                qitems[q] += J.nx;
            }
        }
        std::vector<PEnt> ents;
        std::vector<int> qoff(kPersistQueues + 1, 0);
        for (int q = 0; q < kPersistQueues; ++q) {
            qoff[q] = (int)ents.size();
            ents.insert(ents.end(), qe[q].begin(), qe[q].end());
        }
        qoff[kPersistQueues] = (int)ents.size();
        PProgram::Part &pt = pr.part[part];
        pt.njobs = (int)jobs.size();
        pt.nitems = (int)nitems;
        pt.nctr = ctr0;
        if (pt.njobs == 0) continue;
        pt.workers = std::min(persist_workers(dir, part, f32), pt.nitems);
        if (pt.workers < 1) return S2DW_E_DEVICE;
        // tickets per fetch: small, so that a map's runs spread over many workers
        pt.chunk = std::max(1, std::min(4, pt.nitems / (128 * pt.workers)));
        if (!pr.alloc(pt.jobs, jobs.size()) || !pr.alloc(pt.ents, ents.size()) ||
            !pr.alloc(pt.qoff, kPersistQueues + 1) || !pr.alloc(pt.qn, kPersistQueues) ||
            !pr.alloc(pt.args, args.size()) || !pr.alloc(pt.ctr, pt.nctr) || !pr.alloc(pt.state, 1))
            return S2DW_E_NOMEM;
        if (hipMemcpy(pt.jobs, jobs.data(), jobs.size() * sizeof(PJob), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pt.ents, ents.data(), ents.size() * sizeof(PEnt), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pt.qoff, qoff.data(), qoff.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pt.qn, qitems.data(), qitems.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pt.args, args.data(), args.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(pt.ctr, 0, (size_t)pt.nctr * sizeof(int)) != hipSuccess ||
            hipMemset(pt.state, 0, sizeof(PState)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            return S2DW_E_DEVICE;
    }
    return S2DW_OK;
}

// One persistent batch: checks the groups, finds or builds its program, launches the parts.
int run_persistent(int dir, const s2dw_group *groups, int32_t ngroups, int32_t *status, hipStream_t st) {
    if (!groups || ngroups < 1) return S2DW_E_ARG;
    const int f32 = groups[0].params.precision == S2DW_MIXED ? 1 : 0;
    std::vector<PGroup> gs;
    std::string key((const char *)&dir, sizeof dir);
    key.append((const char *)&st, sizeof st);
    for (int32_t g = 0; g < ngroups; ++g) {  // every group checked before any device work
        const s2dw_group &e = groups[g];
        int rc = check_params(&e.params);
        if (rc != S2DW_OK) return rc;
        if (e.count < 1 || !e.flm || !e.W || !aligned(e.flm) || !aligned(e.W) || (e.Wphi_lm && !aligned(e.Wphi_lm)))
            return S2DW_E_ARG;
        if ((e.params.precision == S2DW_MIXED ? 1 : 0) != f32) return S2DW_E_ARG;
    }
    for (int32_t g = 0; g < ngroups; ++g)
        if (groups[g].params.reality != 1 || groups[g].params.grid != S2DW_GRID_MW || groups[g].params.N > 8)
            return S2DW_E_UNSUPPORTED;
    for (int32_t g = 0; g < ngroups; ++g) {
        const s2dw_group &e = groups[g];
        PGroup pg;
        int rc = get_plan(kWavelet, e.params.L, e.params.N, e.params.lambda, e.params.J_min, pg.P, f32 != 0, e.params.grid);
        if (rc != S2DW_OK) return rc;
        pg.count = e.count;
        pg.flm = e.flm;
        pg.W = e.W;
        pg.wphi = e.Wphi_lm;
        gs.push_back(pg);
        const uintptr_t kv[5] = {(uintptr_t)pg.P, (uintptr_t)pg.count, (uintptr_t)pg.flm, (uintptr_t)pg.W,
                                 (uintptr_t)pg.wphi};
        key.append((const char *)kv, sizeof kv);
    }
    PProgram *pr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_programs.find(key);
        if (it != g_programs.end()) pr = it->second.get();
    }
    if (!pr) {
        std::unique_ptr<PProgram> np(new (std::nothrow) PProgram());
        if (!np) return S2DW_E_NOMEM;
        int rc = build_program(*np, dir, f32, gs, st);
        if (rc != S2DW_OK) return rc;
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_programs.find(key);
        if (it != g_programs.end()) pr = it->second.get();  // built meanwhile by another thread: keep that one
        else pr = (g_programs[key] = std::move(np)).get();
    }
    int spin, extra;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        spin = g_spin_limit > 0 ? g_spin_limit : kDefaultSpinLimit;
        extra = g_wait_extra;
    }
    // analysis: Wigner part, then the separation-of-variables part; synthesis the reverse
    const int order[2] = {dir == 0 ? 0 : 1, dir == 0 ? 1 : 0};
    int launched = 0;
    for (int k = 0; k < 2; ++k) {
        const PProgram::Part &pt = pr->part[order[k]];
        if (pt.njobs == 0) continue;
        Stage sg(order[k] == 0 ? "persist_wigner" : "persist_sov", st);
        S2DW_CHECK_HIP(launch_persist(dir, order[k], f32, pt.workers, pt.jobs, pt.ents, pt.qoff, pt.qn, pt.args,
                                      pt.ctr, pt.nctr, pt.state, status, spin, launched > 0 ? 1 : 0, extra, pt.chunk,
                                      st));
        ++launched;
    }
    return S2DW_OK;
}

}  // namespace
}  // namespace s2dw

namespace s2dw {

// Fixed device scratch of s2dw_analysis_noalloc (the stage workspaces of one call): one copy
// per GPU, held until the process ends.  In host code the name is only a stand-in for the
// device symbol; its device address comes from hipGetSymbolAddress (per device, below).
// File-scope array with external linkage: a `static` one keeps a local binding in the
// device code object, outside its dynamic symbol table, and the runtime cannot resolve
// it by name.
__device__ __align__(256) double2 scratch[S2DW_NOALLOC_SCRATCH_BYTES / sizeof(double2)];

namespace {

std::mutex g_scratch_mu;
std::map<int, double2 *> g_scratch;  // device -> device address of that device's scratch

// The scratch of the current device, looked up once per device (with that device current).
int scratch_of_current_device(double2 *&out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return S2DW_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        out = it->second;
        return S2DW_OK;
    }
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return S2DW_E_DEVICE;
    g_scratch[dev] = (double2 *)ptr;
    out = (double2 *)ptr;
    return S2DW_OK;
}

}  // namespace
}  // namespace s2dw

using namespace s2dw;

extern "C" {

int s2dw_num_scales(const s2dw_params *p, int32_t *S) {
    if (!p || !S || p->L < 2 || !(p->lambda > 1.0) || !std::isfinite(p->lambda)) return S2DW_E_ARG;
    int JL = jmax_of(p->L, p->lambda);
    if (p->J_min < 0 || p->J_min > JL) return S2DW_E_ARG;
    *S = JL - p->J_min + 1;
    return S2DW_OK;
}

int s2dw_grid_shape(const s2dw_params *p, int32_t shape[3]) {
    if (!p || !shape || p->L < 2 || p->N < 1) return S2DW_E_ARG;
    const bool dh = p->grid == S2DW_GRID_DH;
    shape[0] = dh ? p->N : 2 * p->N - 1;
    shape[1] = dh ? 2 * p->L : p->L;
    shape[2] = 2 * p->L - 1;
    return S2DW_OK;
}

int s2dw_scale_grid(const s2dw_params *p, int32_t j, int32_t shape[3], uint64_t *offset) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    std::vector<int> Lg;
    rc = grid_limits(p, Lg);
    if (rc != S2DW_OK) return rc;
    if (j < 0 || j >= (int32_t)Lg.size()) return S2DW_E_ARG;
    const bool dh = p->grid == S2DW_GRID_DH;
    const uint64_t G = dh ? p->N : 2 * (uint64_t)p->N - 1, rf = dh ? 2 : 1;
    uint64_t off = 0;
    for (int32_t i = 0; i < j; ++i) off += G * rf * Lg[i] * (Lg[i] > 0 ? 2 * (uint64_t)Lg[i] - 1 : 0);
    if (shape) {
        shape[0] = (int32_t)G;
        shape[1] = (int32_t)(rf * Lg[j]);
        shape[2] = Lg[j] > 0 ? 2 * Lg[j] - 1 : 0;
    }
    if (offset) *offset = off;
    return S2DW_OK;
}

int s2dw_wavelet_bytes(const s2dw_params *p, uint64_t *bytes) {
    if (!bytes) return S2DW_E_ARG;
    const uint64_t el = (p && p->precision == S2DW_MIXED ? 4 : 8) * (p && p->reality == 0 ? 2 : 1);
    if (p && p->grid == S2DW_GRID_MW_MULTIRES) {
        int rc = check_params(p);
        if (rc != S2DW_OK) return rc;
        std::vector<int> Lg;
        rc = grid_limits(p, Lg);
        if (rc != S2DW_OK) return rc;
        uint64_t n = 0;
        for (int l : Lg) n += (2 * (uint64_t)p->N - 1) * l * (l > 0 ? 2 * (uint64_t)l - 1 : 0);
        *bytes = n * el;
        return S2DW_OK;
    }
    int32_t S = 0;
    int rc = s2dw_num_scales(p, &S);
    if (rc != S2DW_OK) return rc;
    if (p->N < 1) return S2DW_E_ARG;
    int32_t sh[3];
    rc = s2dw_grid_shape(p, sh);
    if (rc != S2DW_OK) return rc;
    *bytes = (uint64_t)S * sh[0] * sh[1] * sh[2] * el;
    return S2DW_OK;
}

int s2dw_analysis_batched(const s2dw_params *p, int32_t count, const double *flm, void *W, double *Wphi_lm,
                          void *stream) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    if (count < 1 || !flm || !W || !aligned(flm) || !aligned(W) || (Wphi_lm && !aligned(Wphi_lm))) return S2DW_E_ARG;
    Plan *P = nullptr;
    const int f32 = p->precision == S2DW_MIXED ? 1 : 0;
    rc = get_plan(kWavelet, p->L, p->N, p->lambda, p->J_min, P, f32 != 0, p->grid);
    if (rc != S2DW_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const bool cx = p->reality == 0;
    const int per = cx ? 2 : 1;  // real maps per signal
    const Shape sh = shape_of(*P);
    const int chunk = std::max(1, std::min<int>(count, sh.chunk / per));
    Work *w = nullptr;
    rc = get_work(*P, st, chunk * per, sh.s_F, w);
    if (rc != S2DW_OK) return rc;
    const size_t L2 = (size_t)p->L * p->L;
    const size_t wmap = P->woff[P->S] * (f32 ? 4 : 8) * per;
    for (int i0 = 0; i0 < count; i0 += chunk) {
        const int n = std::min(chunk, count - i0);
        rc = run_inverse(*P, sh, *w, n * per, (const double2 *)flm + L2 * i0, (char *)W + wmap * i0, f32, st, cx);
        if (rc != S2DW_OK) return rc;
        if (Wphi_lm) {
            Stage sg("scaling", st);
            S2DW_CHECK_HIP(launch_scaling((const double2 *)flm + L2 * i0, P->phi, (double2 *)Wphi_lm + L2 * i0, p->L,
                                          n, st));
        }
    }
    return S2DW_OK;
}

int s2dw_synthesis_batched(const s2dw_params *p, int32_t count, const void *W, const double *Wphi_lm,
                           double *flm_out, void *stream) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    if (count < 1 || !W || !flm_out || !aligned(W) || !aligned(flm_out) || (Wphi_lm && !aligned(Wphi_lm)))
        return S2DW_E_ARG;
    Plan *P = nullptr;
    const int f32 = p->precision == S2DW_MIXED ? 1 : 0;
    rc = get_plan(kWavelet, p->L, p->N, p->lambda, p->J_min, P, f32 != 0, p->grid);
    if (rc != S2DW_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const bool cx = p->reality == 0;
    const int per = cx ? 2 : 1;
    const Shape sh = shape_of(*P);
    const int chunk = std::max(1, std::min<int>(count, sh.chunk / per));
    Work *w = nullptr;
    rc = get_work(*P, st, chunk * per, sh.s_F, w);
    if (rc != S2DW_OK) return rc;
    const size_t L2 = (size_t)p->L * p->L;
    const size_t wmap = P->woff[P->S] * (f32 ? 4 : 8) * per;
    for (int i0 = 0; i0 < count; i0 += chunk) {
        const int n = std::min(chunk, count - i0);
        const double2 *wphi = Wphi_lm ? (const double2 *)Wphi_lm + L2 * i0 : nullptr;
        if (!cx) {
            rc = run_forward(*P, sh, *w, n, (const char *)W + wmap * i0, wphi, (double2 *)flm_out + L2 * i0, f32, st);
            if (rc != S2DW_OK) return rc;
            continue;
        }
        // the real and imaginary parts' syntheses land in the (free) padded-input workspace,
        // map k at k L^2, and are combined with the scaling part
        rc = run_forward(*P, sh, *w, 2 * n, (const char *)W + wmap * i0, nullptr, w->fpad, f32, st, true);
        if (rc != S2DW_OK) return rc;
        Stage sg("syn_final", st);
        S2DW_CHECK_HIP(launch_merge_complex(w->fpad, L2, wphi, P->phi, (double2 *)flm_out + L2 * i0, p->L, n, st));
    }
    return S2DW_OK;
}

int s2dw_autotune(const s2dw_params *p, int32_t count, void *stream, int32_t *slots, int32_t *chunk) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    if (count < 1) return S2DW_E_ARG;
    Plan *P = nullptr;
    const int f32 = p->precision == S2DW_MIXED ? 1 : 0;
    rc = get_plan(kWavelet, p->L, p->N, p->lambda, p->J_min, P, f32 != 0, p->grid);
    if (rc != S2DW_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamSynchronize(st) != hipSuccess) return S2DW_E_DEVICE;
    int cmax = 1;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        cmax = std::min<int>(count, std::max(default_chunk(*P), 1));
    }
    // probe buffers (zero coefficients: the kernels have no data-dependent control flow)
    const size_t L2 = (size_t)p->L * p->L;
    const size_t wmap = P->woff[P->S] * (f32 ? 4 : 8) * (p->reality == 0 ? 2 : 1);
    void *fin = nullptr, *wbuf = nullptr, *fout = nullptr;
    if (hipMalloc(&fin, 16 * L2 * cmax) != hipSuccess) return S2DW_E_NOMEM;
    if (hipMalloc(&wbuf, wmap * cmax) != hipSuccess || hipMalloc(&fout, 16 * L2 * cmax) != hipSuccess) {
        hipFree(fin);
        if (wbuf) hipFree(wbuf);
        return S2DW_E_NOMEM;
    }
    hipMemset(fin, 0, 16 * L2 * cmax);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    s2dw_params q = *p;
    // seconds per map of a round trip with tile shape R, batch chunk c and fusion form fu
    auto trial = [&](int R, int c, int fu, double &sec) -> int {
        {
            std::lock_guard<std::mutex> lk(g_mu);
            int r2 = set_slots(*P, R);
            if (r2 != S2DW_OK) return r2;
            P->cur.chunk = c;
            P->cur.fuse = fu;
        }
        for (int it = 0; it < 3; ++it) {
            if (it == 1) hipEventRecord(e0, st);
            int r2 = s2dw_analysis_batched(&q, c, (const double *)fin, wbuf, nullptr, st);
            if (r2 == S2DW_OK) r2 = s2dw_synthesis_batched(&q, c, wbuf, nullptr, (double *)fout, st);
            if (r2 != S2DW_OK) return r2;
        }
        hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) return S2DW_E_DEVICE;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        sec = ms * 1e-3 / (2.0 * c);
        return S2DW_OK;
    };
    int Ropt[3];
    const int nR = wig_slot_options(P->K, Ropt);
    int bestR = shape_of(*P).R, bestC = cmax, bestF = 1;
    double best = 1e30;
    for (int i = 0; i < nR && rc == S2DW_OK; ++i) {
        double sec = 0;
        rc = trial(Ropt[i], cmax, 1, sec);
        if (rc == S2DW_OK && sec < best) {
            best = sec;
            bestR = Ropt[i];
        }
    }
    // the alpha and gamma forms, where the fused prime-factor kernels apply (T = 2047, 4095)
    const auto gfull = P->gt.find(P->L);
    if (gfull != P->gt.end() && gfull->second.pcs && p->reality != 0 && pfa_fused(2 * P->L - 1, P->Nh)) {
        for (int fu = 0; fu <= 2 && rc == S2DW_OK; fu += 2) {
            double sec = 0;
            rc = trial(bestR, cmax, fu, sec);
            if (rc == S2DW_OK && sec < best) {
                best = sec;
                bestF = fu;
            }
        }
    }
    best = 1e30;
    for (int c = 1; c <= cmax && rc == S2DW_OK; c *= 2) {
        double sec = 0;
        rc = trial(bestR, c, bestF, sec);
        if (rc == S2DW_OK && sec < best * 0.97) {  // a larger batch must win by 3%
            best = sec;
            bestC = c;
        }
    }
    if (rc == S2DW_OK && cmax & (cmax - 1)) {  // the largest chunk when it is not a power of two
        double sec = 0;
        rc = trial(bestR, cmax, bestF, sec);
        if (rc == S2DW_OK && sec < best * 0.97) bestC = cmax;
    }
    hipStreamSynchronize(st);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(fin);
    hipFree(wbuf);
    hipFree(fout);
    if (rc != S2DW_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        rc = set_slots(*P, bestR);
        P->cur.chunk = bestC;
        P->cur.fuse = bestF;
    }
    if (slots) *slots = bestR;
    if (chunk) *chunk = bestC;
    return rc;
}

int s2dw_analysis_persistent(const s2dw_group *groups, int32_t ngroups, int32_t *status, void *stream) {
    return run_persistent(0, groups, ngroups, status, (hipStream_t)stream);
}

int s2dw_synthesis_persistent(const s2dw_group *groups, int32_t ngroups, int32_t *status, void *stream) {
    return run_persistent(1, groups, ngroups, status, (hipStream_t)stream);
}

int s2dw_persistent_wait_bound(int32_t polls, int32_t never_satisfied) {
    if (polls < 0 || (never_satisfied != 0 && never_satisfied != 1)) return S2DW_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    g_spin_limit = polls;
    g_wait_extra = never_satisfied;
    return S2DW_OK;
}

int s2dw_get_tuning(const s2dw_params *p, int32_t *slots, int32_t *chunk, int32_t *fuse) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    Plan *P = nullptr;
    rc = get_plan(kWavelet, p->L, p->N, p->lambda, p->J_min, P, p->precision == S2DW_MIXED, p->grid);
    if (rc != S2DW_OK) return rc;
    const Shape sh = shape_of(*P);
    if (slots) *slots = sh.R;
    if (chunk) *chunk = sh.chunk;
    if (fuse) *fuse = sh.fuse;
    return S2DW_OK;
}

int s2dw_set_tuning(const s2dw_params *p, int32_t slots, int32_t chunk, int32_t fuse) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    if (chunk < 1 || fuse < 0 || fuse > 2) return S2DW_E_ARG;
    Plan *P = nullptr;
    rc = get_plan(kWavelet, p->L, p->N, p->lambda, p->J_min, P, p->precision == S2DW_MIXED, p->grid);
    if (rc != S2DW_OK) return rc;
    int Ropt[3];
    const int nR = wig_slot_options(P->K, Ropt);
    if (std::find(Ropt, Ropt + nR, (int)slots) == Ropt + nR) return S2DW_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    rc = set_slots(*P, slots);
    if (rc != S2DW_OK) return rc;
    P->cur.chunk = chunk;
    P->cur.fuse = fuse;
    return S2DW_OK;
}

int s2dw_workspace_bytes(const s2dw_params *p, int32_t count, uint64_t *bytes) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    if (count < 1 || !bytes) return S2DW_E_ARG;
    Plan *P = nullptr;
    rc = get_plan(kWavelet, p->L, p->N, p->lambda, p->J_min, P, p->precision == S2DW_MIXED, p->grid);
    if (rc != S2DW_OK) return rc;
    const Shape sh = shape_of(*P);
    const uint64_t per_map = 16ull * (P->s_fpad + P->s_U + P->s_Ub + P->s_Y + sh.s_F);
    const int per = p->reality == 0 ? 2 : 1;  // real maps per signal
    *bytes = per_map * per * (uint64_t)std::min<int>(count, std::max(sh.chunk / per, 1));
    return S2DW_OK;
}

int s2dw_cache_bytes(uint64_t *bytes) {
    if (!bytes) return S2DW_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    uint64_t b = 0;
    for (auto &kv : g_plans) {
        b += kv.second->dev_bytes;
        for (auto &w : kv.second->work)
            if (w.second) b += w.second->bytes;
    }
    *bytes = b;
    return S2DW_OK;
}

int s2dw_analysis(const s2dw_params *p, const double *flm, void *W, double *Wphi_lm, void *stream) {
    return s2dw_analysis_batched(p, 1, flm, W, Wphi_lm, stream);
}

int s2dw_analysis_noalloc(const s2dw_params *p, const double *flm, void *W, double *Wphi_lm, void *stream) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    if (!flm || !W || !aligned(flm) || !aligned(W) || (Wphi_lm && !aligned(Wphi_lm))) return S2DW_E_ARG;
    const int f32 = p->precision == S2DW_MIXED ? 1 : 0;
    Plan *P = find_plan(p->L, p->N, p->lambda, p->J_min, f32 != 0, p->grid);
    if (!P) return S2DW_E_ARG;  // the plan must have been built by an allocating call
    const bool cx = p->reality == 0;
    const int per = cx ? 2 : 1;  // real maps of the signal
    const size_t per_map = P->s_fpad + P->s_U + P->s_Ub + P->s_Y;  // complex elements
    if ((size_t)per * per_map * sizeof(double2) > S2DW_NOALLOC_SCRATCH_BYTES) return S2DW_E_UNSUPPORTED;
    double2 *base = nullptr;
    rc = scratch_of_current_device(base);
    if (rc != S2DW_OK) return rc;
    Work w;  // views into the scratch (owns nothing)
    w.cap = per;
    w.fpad = base;
    w.U = w.fpad + (size_t)per * P->s_fpad;
    w.Ub = w.U + (size_t)per * P->s_U;
    w.Y = w.Ub + (size_t)per * P->s_Ub;
    const Shape sh = shape_of(*P);
    hipStream_t st = (hipStream_t)stream;
    t_no_events = true;
    rc = run_inverse(*P, sh, w, per, (const double2 *)flm, W, f32, st, cx);
    if (rc == S2DW_OK && Wphi_lm && launch_scaling((const double2 *)flm, P->phi, (double2 *)Wphi_lm, p->L, 1, st) !=
                                        hipSuccess)
        rc = S2DW_E_DEVICE;
    t_no_events = false;
    return rc;
}

int s2dw_synthesis(const s2dw_params *p, const void *W, const double *Wphi_lm, double *flm_out, void *stream) {
    return s2dw_synthesis_batched(p, 1, W, Wphi_lm, flm_out, stream);
}

int s2dw_scaling(const s2dw_params *p, const double *flm, double *Wphi_lm, double *Wphi_map, void *stream) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    if (!flm || !aligned(flm) || (Wphi_lm && !aligned(Wphi_lm)) || (Wphi_map && !aligned(Wphi_map))) return S2DW_E_ARG;
    if (Wphi_map && p->reality == 0) return S2DW_E_UNSUPPORTED;  // the sphere maps are real
    if (!Wphi_lm && !Wphi_map) return S2DW_OK;
    Plan *P = nullptr;
    rc = get_plan(kWavelet, p->L, p->N, p->lambda, p->J_min, P, false, p->grid);
    if (rc != S2DW_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    Work *w = nullptr;
    rc = get_work(*P, st, 1, shape_of(*P).s_F, w);
    if (rc != S2DW_OK) return rc;
    double2 *wphi = (double2 *)Wphi_lm;
    if (!wphi) wphi = w->fpad;  // scratch: L*Lp >= L*L complex
    S2DW_CHECK_HIP(launch_scaling((const double2 *)flm, P->phi, wphi, p->L, 1, st));
    if (Wphi_map) {
        Plan *Q = nullptr;
        rc = get_plan(kShtInverse, p->L, 1, 0.0, 0, Q);
        if (rc != S2DW_OK) return rc;
        Work *wq = nullptr;
        const Shape shq = shape_of(*Q);
        rc = get_work(*Q, st, 1, shq.s_F, wq);
        if (rc != S2DW_OK) return rc;
        rc = run_inverse(*Q, shq, *wq, 1, wphi, Wphi_map, 0, st);
    }
    return rc;
}

int s2dw_steer(const s2dw_params *p, int32_t count, const void *W, int32_t n_gamma, const double *gamma, void *out,
               void *stream) {
    int rc = check_params(p);
    if (rc != S2DW_OK) return rc;
    if (count < 1 || n_gamma < 0 || n_gamma > kMaxSteerAngles) return S2DW_E_ARG;
    if (n_gamma == 0) return S2DW_OK;
    if (!W || !gamma || !out || !aligned(W) || !aligned(gamma) || !aligned(out)) return S2DW_E_ARG;
    std::vector<int> Lg;
    rc = grid_limits(p, Lg);
    if (rc != S2DW_OK) return rc;
    const bool dh = p->grid == S2DW_GRID_DH;
    const int S = (int)Lg.size(), G = dh ? p->N : 2 * p->N - 1, rf = dh ? 2 : 1;
    // gamma samples: gamma_g = 2 pi g/(2N-1), or pi g/N on the Driscoll-Healy grid; in both
    // cases the interpolation weight is 1/G (z_n = 1/N on the paper's grid, Eq. 10)
    const double step = dh ? M_PI / p->N : 2.0 * M_PI / G;
    const int f32 = p->precision == S2DW_MIXED;
    const size_t es = f32 ? 4 : 8;
    // complex coefficients (complex signals): (re, im) pairs steer as one plane of twice the size
    const size_t cf = p->reality == 0 ? 2 : 1;
    // element offsets of each scale in one map of W and of out
    std::vector<size_t> oin(S + 1, 0), oout(S + 1, 0);
    for (int j = 0; j < S; ++j) {
        const size_t pl = cf * rf * Lg[j] * (Lg[j] > 0 ? 2 * Lg[j] - 1 : 0);
        oin[j + 1] = oin[j] + G * pl;
        oout[j + 1] = oout[j] + (size_t)n_gamma * pl;
    }
    hipStream_t st = (hipStream_t)stream;
    Stage sg("steer", st);
    for (int32_t i = 0; i < count; i += 65535) {
        const int maps = std::min<int32_t>(65535, count - i);
        const char *Wi = (const char *)W + i * oin[S] * es;
        char *Oi = (char *)out + i * oout[S] * es;
        if (p->grid != S2DW_GRID_MW_MULTIRES) {  // one plane size: all scales in one launch
            S2DW_CHECK_HIP(launch_steer(Wi, gamma, Oi, f32, p->N, G, step, n_gamma, S,
                                        cf * rf * p->L * (2 * p->L - 1), oin[S], oout[S], maps, st));
            continue;
        }
        for (int j = 0; j < S; ++j) {
            if (Lg[j] == 0) continue;
            S2DW_CHECK_HIP(launch_steer(Wi + oin[j] * es, gamma, Oi + oout[j] * es, f32, p->N, G, step, n_gamma, 1,
                                        cf * Lg[j] * (2 * Lg[j] - 1), oin[S], oout[S], maps, st));
        }
    }
    return S2DW_OK;
}

int s2dw_sht_forward(const s2dw_params *p, const double *f_map, double *flm, void *stream) {
    if (!p || p->L < 2 || p->L > 4096 || !f_map || !flm || !aligned(f_map) || !aligned(flm)) return S2DW_E_ARG;
    if (p->L > 2048) return S2DW_E_UNSUPPORTED;
    Plan *Q = nullptr;
    int rc = get_plan(kShtForward, p->L, 1, 0.0, 0, Q);
    if (rc != S2DW_OK) return rc;
    Work *w = nullptr;
    const Shape sh = shape_of(*Q);
    rc = get_work(*Q, (hipStream_t)stream, 1, sh.s_F, w);
    if (rc != S2DW_OK) return rc;
    return run_forward(*Q, sh, *w, 1, f_map, nullptr, (double2 *)flm, 0, (hipStream_t)stream);
}

int s2dw_sht_inverse(const s2dw_params *p, const double *flm, double *f_map, void *stream) {
    if (!p || p->L < 2 || p->L > 4096 || !f_map || !flm || !aligned(f_map) || !aligned(flm)) return S2DW_E_ARG;
    if (p->L > 2048) return S2DW_E_UNSUPPORTED;
    Plan *Q = nullptr;
    int rc = get_plan(kShtInverse, p->L, 1, 0.0, 0, Q);
    if (rc != S2DW_OK) return rc;
    Work *w = nullptr;
    const Shape sh = shape_of(*Q);
    rc = get_work(*Q, (hipStream_t)stream, 1, sh.s_F, w);
    if (rc != S2DW_OK) return rc;
    return run_inverse(*Q, sh, *w, 1, (const double2 *)flm, f_map, 0, (hipStream_t)stream);
}

int s2dw_wavelet_tables(const s2dw_params *p, double *kappa, double *phi, double *s_ln) {
    if (!p || p->L < 2 || p->L > 4096 || p->N < 1 || p->N > p->L || p->N > 2 * kMaxK) return S2DW_E_ARG;
    HostTables t;
    if (!build_wavelet_tables(p->L, p->N, p->lambda, p->J_min, t)) return S2DW_E_ARG;
    const int L = p->L, N = p->N;
    if (kappa) memcpy(kappa, t.kappa.data(), sizeof(double) * t.kappa.size());
    if (phi) memcpy(phi, t.phi.data(), sizeof(double) * L);
    if (s_ln) {
        memset(s_ln, 0, sizeof(double) * 2 * (size_t)L * (2 * N - 1));
        for (int l = 0; l < L; ++l)
            for (int k = 0; k < t.K; ++k) {
                const double v = t.sig[(size_t)l * t.K + k];
                for (int sg = -1; sg <= 1; sg += 2) {
                    const int n = sg * t.nk[k];
                    double *o = s_ln + 2 * ((size_t)l * (2 * N - 1) + n + N - 1);
                    o[t.eta_imag ? 1 : 0] = v;  // eta_N = i for even N (Eq. 11)
                    if (n == 0) break;
                }
            }
    }
    return S2DW_OK;
}

int s2dw_profile(int enable) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    prof_collect();
    g_prof.totals.clear();
    g_prof.on = enable != 0;
    return S2DW_OK;
}

int s2dw_profile_stages(const char *names) {
    static const char *const known[] = {"pad",       "wigner_fwd",      "beta_fwd",  "alpha_fwd",
                                        "gamma_fwd", "alpha_gamma_fwd", "gamma_adj", "gamma_alpha_adj",
                                        "alpha_adj", "beta_adj",        "wigner_adj", "syn_final",
                                        "scaling",   "steer",           "persist_wigner", "persist_sov"};
    std::set<std::string> sel;
    if (names) {
        const std::string all(names);
        size_t i = 0;
        while (i <= all.size()) {
            size_t j = all.find(',', i);
            if (j == std::string::npos) j = all.size();
            const std::string w = all.substr(i, j - i);
            if (!w.empty()) {
                bool ok = false;
                for (const char *k : known) ok = ok || w == k;
                if (!ok) return S2DW_E_ARG;
                sel.insert(w);
            }
            i = j + 1;
        }
    }
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.only.swap(sel);
    return S2DW_OK;
}

int s2dw_profile_read(s2dw_stage_time *out, int32_t max, int32_t *n) {
    if (!n || (max > 0 && !out)) return S2DW_E_ARG;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    prof_collect();
    int i = 0;
    for (auto &kv : g_prof.totals) {
        if (i < max) {
            memset(out[i].name, 0, sizeof(out[i].name));
            strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
            out[i].ms = kv.second.first;
            out[i].count = kv.second.second;
        }
        ++i;
    }
    *n = i;
    return S2DW_OK;
}

const char *s2dw_strerror(int code) {
    switch (code) {
        case S2DW_OK: return "ok";
        case S2DW_E_ARG: return "invalid argument";
        case S2DW_E_NOMEM: return "out of memory";
        case S2DW_E_DEVICE: return "HIP call failed";
        case S2DW_E_UNSUPPORTED: return "not supported";
        case S2DW_E_INTERNAL: return "internal error";
        default: return "unknown status";
    }
}

void s2dw_release_caches(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_plans.empty() || !g_programs.empty()) hipDeviceSynchronize();
    g_programs.clear();  // they point into the plans' tables
    g_plans.clear();
}

}  // extern "C"
