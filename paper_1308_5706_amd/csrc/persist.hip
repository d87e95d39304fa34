// Persistent executor: the whole analysis (or synthesis) of many maps, of several parameter
// sets at once, as two launches per direction: one runs the Wigner stages (with the input
// padding of the analysis and the final reduction of the synthesis), the other the
// separation-of-variables stages, each with the register budget of its own kernels.
//
// The work list is the ordinary launch sequence of every parameter set, recorded (kernels.h):
// each launch becomes a job whose workgroups ("work items") the executor runs as device
// functions.  The maps are spread over 8 ticket queues (each map's work in one queue); a
// queue lists (job, map) entries in dependency order.  A launch of `workers` workgroups of
// 256 threads stays resident; each worker takes tickets in increasing order from its home
// queue and, once that is exhausted, from the others in turn; it finds the ticket's entry,
// waits until the job it depends on has finished for the same map, runs the item and
// signals the job's counter for that map.  Every dependency lies in the same queue with
// smaller tickets; a ticket is only taken by a running worker, and the smallest unfinished
// ticket of a queue never waits on an unfinished one, so the launch drains whatever the
// number of resident workers.
//
// Within a parameter set a job depends on the job before it (the launch order of the
// ordinary path, per map); the parameter sets are independent, and their jobs interleave by
// position in their sequences so that every set's maps move through the stages together.
// A worker takes `chunk` consecutive tickets at a time and runs them in order; consecutive
// tickets of one job and map form a run, which waits once for its dependency and signals once
// (the count of its items) when it ends, before the next run waits (so the ordering argument
// above still holds).  Visibility between workgroups: at the end of a run every wave waits
// for its stores (vmcnt 0), a barrier follows, and one thread releases at agent scope and
// adds the count; the waiting thread polls with atomic loads and acquires at agent scope
// (the caches it invalidates are the ones the workgroup shares), and a barrier follows.
//
// Work items of the FFT stages take P / 8 threads; a worker runs 256 / (P / 8) of them side by
// side, each with its own LDS column.  Past the end of a job the extra columns repeat its last
// one: the same values written to the same places.
//
// Every wait is bounded (spin_limit polls): a wait that runs out sets the error word, and
// from then on workers skip the waits and the items' work (still signalling) so that the
// launch drains.  wait_extra = 1 makes every wait unsatisfiable (tests of that path).  The
// last worker to leave copies the error word to *status (if given; with status_or only a
// nonzero one, so that a second launch keeps the first one's error) and clears the ticket,
// exit and error words and every counter, so that the next launch (or graph replay) starts
// from zero.
#include "misc_k.h"
#include "stages_k.h"
#include "wigner_k.h"

namespace s2dw {

static_assert(S2DW_FFT_RADIX == 8, "the recorded FFT work items take P / 8 threads");

namespace {

constexpr int kPersistThreads = 256;
constexpr int kPersistAW = kPersistThreads / 64;  // waves of the synthesis Wigner items
constexpr int kMaxNH = 4;                          // orders n >= 0 of the direct fused passes (N <= 8)
constexpr int kVmcnt0 = 0x0F70;                    // s_waitcnt vmcnt(0) (gfx9 encoding; expcnt, lgkmcnt not waited)

constexpr int cmax(int a, int b) { return a > b ? a : b; }
// LDS of a worker: the FFT columns (256 threads' worth: padded(2048) elements of the largest
// complex type), the synthesis Wigner window, the direct fused passes' tables
constexpr int kPersistLds =
    cmax(cmax(fft::padded(kPersistMaxP) * (int)sizeof(double2), kPersistAW * 8 * 64 * 2 * (int)sizeof(double)),
         cmax(kAlphaGammaCoeffs * (int)sizeof(double2), (kMaxNH + 2) * 256 * (int)sizeof(double2)));

// The argument block of a job, read through the constant address space (as kernel
// arguments are): the loads are scalar and may be repeated wherever the compiler likes.
template <class T>
__device__ __forceinline__ const T &job_args(const unsigned char *ap) {
    typedef const __attribute__((address_space(4))) T *cptr;
    return *(const T *)(cptr)(ap);
}

// The FFT work item of size P: 256 / NT columns side by side, the extra ones past gx repeating
// the last column.
template <class C, int P, class F>
__device__ __forceinline__ void fft_item(int vb0, int gx, int tid, unsigned char *lds, F f) {
    constexpr int NT = P / 8;
    const int sub = tid / NT, lt = tid - sub * NT;
    int vb = vb0 + sub;
    if (vb >= gx) vb = gx - 1;
    f(vb, lt, (C *)lds + sub * fft::padded(P));
}

#define S2DW_PERSIST_P(CALL)  \
    switch (ka) {             \
        case 5: CALL(32) break; \
        case 6: CALL(64) break; \
        case 7: CALL(128) break; \
        case 8: CALL(256) break; \
        case 9: CALL(512) break; \
        case 10: CALL(1024) break; \
        case 11: CALL(2048) break; \
        default: break;       \
    }

// The Wigner tile shapes of the executor (persist_slots: the ordinary kernels' defaults).
#define S2DW_PERSIST_KR(CALL) \
    switch (ka * 8 + kb) {    \
        case 12: CALL(1, 4) break; \
        case 18: CALL(2, 2) break; \
        case 26: CALL(3, 2) break; \
        case 34: CALL(4, 2) break; \
        default: break;       \
    }

// Work item: workgroups vb0 .. of map by of the job (kind, argument block ap, gx per map).
// PART 0: the Wigner stages (with the input padding and the final synthesis reduction);
// PART 1: the separation-of-variables stages.
template <class C, int DIR, int PART>
__device__ __forceinline__ void persist_item(int kind, const unsigned char *ap, int vb0, int gx, int by, int tid,
                                             unsigned char *lds) {
    const int stage = pkind_stage(kind), ka = pkind_a(kind), kb = pkind_b(kind);
    if constexpr (DIR == 0 && PART == 0) {
        switch (stage) {
            case PS_PAD: {
                const PadArgs &p = job_args<PadArgs>(ap);
                const int gx0 = (p.Lp + 255) / 256;
                pad_flm_elem(p.flm, p.g, p.fpad, p.L, p.Lp, p.s_fpad, (vb0 % gx0) * 256 + tid, vb0 / gx0, by);
                break;
            }
            case PS_WIGF: {
                const WigFwdArgs &a = job_args<WigFwdArgs>(ap);
#define S2DW_WF(K, R)                                                     \
    if (vb0 < a.nplain) wig_fwd_body<K, R, false>(a, vb0, by, tid);       \
    else wig_fwd_body<K, R, true>(a, vb0, by, tid);
                S2DW_PERSIST_KR(S2DW_WF)
#undef S2DW_WF
                break;
            }
            default: break;
        }
    } else if constexpr (DIR == 0) {
        switch (stage) {
            case PS_BETAF_FFT: {
                const StageArgs &a = job_args<StageArgs>(ap);
#define S2DW_BF(PV) \
    fft_item<C, PV>(vb0, gx, tid, lds, [&](int vb, int lt, C *buf) { beta_fwd_fft_body<C, PV>(a, vb, by, lt, buf); });
                S2DW_PERSIST_P(S2DW_BF)
#undef S2DW_BF
                break;
            }
            case PS_BETAF_PAIR: {
                const StageArgs &a = job_args<StageArgs>(ap);
#define S2DW_BP(PV) \
    fft_item<C, PV>(vb0, gx, tid, lds, [&](int vb, int lt, C *buf) { beta_fwd_pair_body<C, PV>(a, vb, by, lt, buf); });
                S2DW_PERSIST_P(S2DW_BP)
#undef S2DW_BP
                break;
            }
            case PS_ALPHAF_FFT: {
                const StageArgs &a = job_args<StageArgs>(ap);
#define S2DW_AF(PV) \
    fft_item<C, PV>(vb0, gx, tid, lds, [&](int vb, int lt, C *buf) { alpha_fwd_fft_body<C, PV>(a, vb, by, lt, buf); });
                S2DW_PERSIST_P(S2DW_AF)
#undef S2DW_AF
                break;
            }
            case PS_ALPHAF_BLK: {
                const StageArgs &a = job_args<StageArgs>(ap);
#define S2DW_AB(PV)                                                                                               \
    if constexpr (fft::Plan<PV, 8>::NPASS >= 2)                                                                  \
        fft_item<C, PV>(vb0, gx, tid, lds, [&](int vb, int lt, C *buf) { alpha_fwd_blk_body<C, PV>(a, vb, by, lt, buf); });
                S2DW_PERSIST_P(S2DW_AB)
#undef S2DW_AB
                break;
            }
            case PS_AGF: {
                const AlphaGammaArgs &a = job_args<AlphaGammaArgs>(ap);
                const int gx0 = ((kb ? a.T / 2 + 1 : a.T) + 255) / 256;
                const int bx = vb0 % gx0, b = vb0 / gx0;
                double2 *cs = (double2 *)lds;
#define S2DW_AG(NH)                                                             \
    case NH:                                                                    \
        if (kb) alpha_gamma_fwd_body<true, NH, C>(a, bx, b, by, tid, cs);       \
        else alpha_gamma_fwd_body<false, NH, C>(a, bx, b, by, tid, cs);         \
        break;
                switch (ka) {
                    S2DW_AG(1)
                    S2DW_AG(2)
                    S2DW_AG(3)
                    S2DW_AG(4)
                    default: break;
                }
#undef S2DW_AG
                break;
            }
            case PS_GAMMAF: {
                const GammaArgs &a = job_args<GammaArgs>(ap);
                if (ka == 2) gamma_fwd_body<C, 2>(a, vb0, by, tid);
                else gamma_fwd_body<C, 1>(a, vb0, by, tid);
                break;
            }
            case PS_SCALING: {
                const ScalingArgs &p = job_args<ScalingArgs>(ap);
                const int gx0 = (2 * p.L - 1 + 255) / 256;
                scaling_elem(p.flm, p.phi, p.wphi, p.L, (vb0 % gx0) * 256 + tid, vb0 / gx0, by);
                break;
            }
            case PS_ZERO: {
                const ZeroArgs &p = job_args<ZeroArgs>(ap);
                for (size_t i = (size_t)vb0 * 256 + tid; i < p.n; i += (size_t)gx * 256) p.p[i] = 0u;
                break;
            }
            default: break;
        }
    } else if constexpr (PART == 1) {
        switch (stage) {
            case PS_GAMMAA: {
                const GammaArgs &a = job_args<GammaArgs>(ap);
                if (ka == 2) gamma_adj_body<C, 2>(a, vb0, by, tid);
                else gamma_adj_body<C, 1>(a, vb0, by, tid);
                break;
            }
            case PS_GAA: {
                const GammaAlphaArgs &a = job_args<GammaAlphaArgs>(ap);
                double2(*xs)[256] = (double2(*)[256])lds;
#define S2DW_GA(NH) \
    case NH: gamma_alpha_adj_body<NH, C>(a, vb0, by, tid, xs, xs + NH); break;
                switch (ka) {
                    S2DW_GA(1)
                    S2DW_GA(2)
                    S2DW_GA(3)
                    S2DW_GA(4)
                    default: break;
                }
#undef S2DW_GA
                break;
            }
            case PS_ALPHAA_FFT: {
                const StageArgs &a = job_args<StageArgs>(ap);
#define S2DW_AA(PV) \
    fft_item<C, PV>(vb0, gx, tid, lds, [&](int vb, int lt, C *buf) { alpha_adj_fft_body<C, PV>(a, vb, by, lt, buf); });
                S2DW_PERSIST_P(S2DW_AA)
#undef S2DW_AA
                break;
            }
            case PS_ALPHAA_BLK: {
                const StageArgs &a = job_args<StageArgs>(ap);
#define S2DW_AJ(PV) \
    fft_item<C, PV>(vb0, gx, tid, lds, [&](int vb, int lt, C *buf) { alpha_adj_blk_body<C, PV>(a, vb, by, lt, buf); });
                S2DW_PERSIST_P(S2DW_AJ)
#undef S2DW_AJ
                break;
            }
            case PS_BETAA_FFT: {
                const StageArgs &a = job_args<StageArgs>(ap);
#define S2DW_BA(PV)                                                                                     \
    fft_item<C, PV>(vb0, gx, tid, lds, [&](int vb, int lt, C *buf) {                                   \
        beta_adj_body<C, PV, false, true>(a, buf, vb, a.Lj, (const C *)a.in + by * a.s_in,              \
                                          (C *)a.out + by * a.s_out, (const C *)a.hh2, lt);                   \
    });
                S2DW_PERSIST_P(S2DW_BA)
#undef S2DW_BA
                break;
            }
            case PS_BETAA_MULTI: {
                const BetaMultiArgs &m = job_args<BetaMultiArgs>(ap);
#define S2DW_BM(PV)                                                                                \
    fft_item<C, PV>(vb0, gx, tid, lds, [&](int vb, int lt, C *buf) {                              \
        beta_adj_multi_body<C, PV, false, true>(m.a, m.tab, m.ns, vb, by, lt, buf);               \
    });
                S2DW_PERSIST_P(S2DW_BM)
#undef S2DW_BM
                break;
            }
            default: break;
        }
    } else {
        switch (stage) {
            case PS_WIGA: {
                using VT = real_t<C>;
                const WigAdjArgs &a = job_args<WigAdjArgs>(ap);
                VT *win = (VT *)lds;
#define S2DW_WA(K, R)                                                                          \
    if (vb0 < a.nplain) wig_adj_body<K, R, false, VT, kPersistAW>(a, win, vb0, by, tid);       \
    else wig_adj_body<K, R, true, VT, kPersistAW>(a, win, vb0, by, tid);
                S2DW_PERSIST_KR(S2DW_WA)
#undef S2DW_WA
                break;
            }
            case PS_SYNF: {
                const SynFinalArgs &p = job_args<SynFinalArgs>(ap);
                const int gx0 = (p.L + 255) / 256;
                syn_final_elem((const C *)p.Fpart, p.s_F, p.nblk, p.group, p.Lmax, p.fac, p.g, p.wphi, p.phi, p.flm,
                               p.L, p.Lp, (vb0 % gx0) * 256 + tid, vb0 / gx0, by);
                break;
            }
            default: break;
        }
    }
}

// Two workers per CU for the Wigner part (the register budget of its tile shapes, as in the
// ordinary kernels), three for the others (168 registers for the union of their bodies:
// measured 63.5 ms for the 256-map batch against 66.6 ms with four workers and 128).
template <class C, int DIR, int PART>
__global__ void __launch_bounds__(kPersistThreads, PART == 0 ? 2 : 3) persist_kernel(const PJob *__restrict__ jobs,
                                                                  const PEnt *__restrict__ ents,
                                                                  const int *__restrict__ qoff,
                                                                  const int *__restrict__ qn,
                                                                  const unsigned char *__restrict__ args, int *ctr,
                                                                  int nctr, PState *state, int *status, int spin_limit,
                                                                  int status_or, int wait_extra, int chunk) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[kPersistLds];
    __shared__ int s_ticket, s_err, s_last;
    const int tid = threadIdx.x;
    // The end of a run of n items of one job and map: every wave waits for its stores, then
    // one agent-scope release and the count.
    auto signal = [&](int c, int n) {
        __builtin_amdgcn_s_waitcnt(kVmcnt0);
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_s_waitcnt(kVmcnt0);
            __hip_atomic_fetch_add(ctr + c, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    // the home queue first (workgroups of one queue share an XCD: q = blockIdx mod 8), then the
    // others in turn; a worker leaves after finding every queue exhausted in a row
    int q = blockIdx.x % kPersistQueues, empty = 0, e = -1;  // e: entry cursor in queue q (-1: not placed)
    for (;;) {
        if (tid == 0) s_ticket = __hip_atomic_fetch_add(&state->ticket[q], chunk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int t0 = __builtin_amdgcn_readfirstlane(s_ticket);  // uniform: job and item fields go to SGPRs
        __syncthreads();                                          // s_ticket is read before it is rewritten
        const int nq = qn[q];
        if (t0 >= nq) {
            if (++empty == kPersistQueues) break;
            q = (q + 1) % kPersistQueues;
            e = -1;
            continue;
        }
        empty = 0;
        const int t1 = min(t0 + chunk, nq), eend = qoff[q + 1];
        if (e < 0) {  // the last entry of the queue starting at or before t0 (binary search)
            int lo = qoff[q], hi = eend;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (ents[mid].item0 <= t0) lo = mid;
                else hi = mid;
            }
            e = lo;
        }
        int run_job = -1, run_by = -1, run_n = 0;
        for (int t = t0; t < t1; ++t) {
            while (e + 1 < eend && ents[e + 1].item0 <= t) ++e;
            const PEnt E = ents[e];
            const int j = E.job, by = E.map, ix = t - E.item0;
            const PJob J = jobs[j];
            if (j != run_job || by != run_by) {
                // a new run: signal the last one (an item of this chunk may wait for it), then wait
                // for this one's dependency
                if (run_n) signal(jobs[run_job].ctr0 + run_by, run_n);
                run_job = j;
                run_by = by;
                run_n = 0;
                if (tid == 0) {
                    // no wait once a wait has run out: the rest of the launch only drains
                    if (J.prev >= 0 && !__hip_atomic_load(&state->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        const PJob Q = jobs[J.prev];
                        int *c = ctr + Q.ctr0 + by;
                        const int need = Q.nx + wait_extra;  // wait_extra = 1 (tests only): never satisfied
                        int polls = 0;
                        while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                            if (++polls > spin_limit) {
                                __hip_atomic_store(&state->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                break;
                            }
                            __builtin_amdgcn_s_sleep(8);
                        }
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                    s_err = __hip_atomic_load(&state->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __syncthreads();
            }
            if (!__builtin_amdgcn_readfirstlane(s_err)) {
                const int per = kPersistThreads / J.nt;  // workgroups of the ordinary launch side by side
                for (int k = 0; k < J.rounds; ++k) {
                    const int vb0 = (ix * J.rounds + k) * per;
                    if (vb0 >= J.gx) break;
                    persist_item<C, DIR, PART>(J.kind, args + J.arg, vb0, J.gx, by, tid, lds);
                    __syncthreads();
                }
            }
            ++run_n;
        }
        if (run_n) signal(jobs[run_job].ctr0 + run_by, run_n);
    }
    // leave; the last worker resets the state for the next launch
    if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int e = __hip_atomic_fetch_add(&state->exited, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = e == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (s_last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (int i = tid; i < nctr; i += kPersistThreads) ctr[i] = 0;
        if (tid == 0) {
            const int err = __hip_atomic_load(&state->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (status && (err || !status_or)) *status = err;
            state->error = 0;
            for (int k = 0; k < kPersistQueues; ++k) state->ticket[k] = 0;
            state->exited = 0;
        }
    }
}

template <class C, int DIR, int PART>
int workers_of() {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_kernel<C, DIR, PART>, kPersistThreads, 0) !=
        hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

}  // namespace

int persist_part(int kind) {
    const int s = pkind_stage(kind);
    return (s == PS_PAD || s == PS_WIGF || s == PS_WIGA || s == PS_SYNF) ? 0 : 1;
}

int persist_slots(int K) { return K <= 1 ? 4 : 2; }

int persist_workers(int dir, int part, int f32) {
#define S2DW_PW(D, PT) return f32 ? workers_of<float2, D, PT>() : workers_of<double2, D, PT>()
    if (dir == 0) {
        if (part == 0) S2DW_PW(0, 0);
        S2DW_PW(0, 1);
    }
    if (part == 0) S2DW_PW(1, 0);
    S2DW_PW(1, 1);
#undef S2DW_PW
}

hipError_t launch_persist(int dir, int part, int f32, int workers, const PJob *jobs, const PEnt *ents,
                          const int *qoff, const int *qn, const unsigned char *args, int *ctr, int nctr,
                          PState *state, int *status, int spin_limit, int status_or, int wait_extra, int chunk,
                          hipStream_t st) {
    if (workers < 1 || chunk < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)workers), block(kPersistThreads);
#define S2DW_PL(C, D, PT)                                                                                    \
    hipLaunchKernelGGL((persist_kernel<C, D, PT>), grid, block, 0, st, jobs, ents, qoff, qn, args, ctr, nctr, state, \
                       status, spin_limit, status_or, wait_extra, chunk)
    const int sel = dir * 4 + part * 2 + (f32 ? 1 : 0);
    switch (sel) {
        case 0: S2DW_PL(double2, 0, 0); break;
        case 1: S2DW_PL(float2, 0, 0); break;
        case 2: S2DW_PL(double2, 0, 1); break;
        case 3: S2DW_PL(float2, 0, 1); break;
        case 4: S2DW_PL(double2, 1, 0); break;
        case 5: S2DW_PL(float2, 1, 0); break;
        case 6: S2DW_PL(double2, 1, 1); break;
        case 7: S2DW_PL(float2, 1, 1); break;
        default: return hipErrorInvalidValue;
    }
#undef S2DW_PL
    return hipGetLastError();
}

}  // namespace s2dw
