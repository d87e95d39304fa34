/*
 * s2dw.h -- C ABI of the MI355X directional scale-discretized wavelet
 * transform on the sphere (McEwen, Vandergheynst & Wiaux, "On the
 * computation of directional scale-discretized wavelet transforms on the
 * sphere", SPIE 2013).
 *
 * The problem statement the arguments follow (Sec. 2): a signal f on the
 * sphere, band-limited at L (f_lm = 0 for l >= L), is given by its
 * spherical-harmonic coefficients f_lm.  Wavelets Psi^j (Eq. 7) with
 * azimuthal band-limit N (Eq. 8), dilation parameter lambda > 1 (Eq. 12)
 * and scales j = 0..J, J = J_L(lambda) - J_min with J_L(lambda) =
 * ceil(log_lambda L), give wavelet coefficients W^j(alpha, beta, gamma)
 * on the rotation group (Eq. 1, computed through Eq. 20) and scaling
 * coefficients W^Phi (Eq. 3, 31).  Synthesis (Eq. 4, computed through
 * Eq. 32-41) recovers f_lm exactly.
 *
 * Conventions
 *  - Complex arrays are interleaved (re, im) doubles.
 *  - f_lm and the harmonic scaling coefficients W^Phi_lm: L*L complex,
 *    index l*l + l + m, -l <= m <= l.
 *  - Wavelet coefficients W: real, [S][2N-1][L][2L-1] = [j][gamma_g][beta_b]
 *    [alpha_a] with alpha fastest, on the equiangular grid
 *        alpha_a = 2 pi a/(2L-1),  beta_b = pi (2b+1)/(2L-1) (b < L),
 *        gamma_g = 2 pi g/(2N-1).
 *    Scale index j = 0 is the highest-frequency wavelet (the paper's
 *    footnote to Eq. 15); S = J + 1.  Elements are doubles for
 *    S2DW_FP64 and floats for S2DW_MIXED.
 *  - Multiresolution layout (grid = S2DW_GRID_MW_MULTIRES): the kernel of
 *    scale j vanishes for l >= L_j = min(L, ceil(L lambda^(1-j))) (Eq. 14-15),
 *    so W^j is band-limited at L_j and needs no finer grid (the closing
 *    remarks of Sec. 3.2); it is sampled on the equiangular grid of band-limit
 *    L_j (alpha 2L_j-1, beta L_j, gamma 2N-1) and the scales are stored back to
 *    back: W = [W^0 (2N-1)xL_0x(2L_0-1)][W^1 ...]...  s2dw_scale_grid gives each
 *    scale's shape and offset.  Analysis and synthesis stay exact.
 *  - Driscoll-Healy layout (grid = S2DW_GRID_DH), the discretisation of
 *    Sec. 3.1: W real [S][N][2L][2L-1] = [j][gamma_g][beta_t][alpha_a] with
 *        alpha_a = 2 pi a/(2L-1),  beta_t = pi (2t+1)/(4L) (t < 2L),
 *        gamma_g = pi g/N (g < N, the N base orientations on [0, pi)).
 *    Synthesis integrates beta with the quadrature weights of Eq. 17-18 and
 *    gamma with weight 2 pi z_n, z_n = 1/N (Eq. 39); both directions are exact.
 *  - Sphere maps: real [L][2L-1] = [theta_b][phi_a] on the same beta/alpha
 *    samples.
 *  - Real signals (reality = 1): f_{l,-m} = (-1)^m conj(f_lm), which makes W
 *    real.  The library reads f_lm for m >= 0 only and writes all m on output.
 *  - Complex signals (reality = 0): all f_lm are read and written; W is
 *    complex, stored as (re, im) pairs (doubles, or floats for S2DW_MIXED) in
 *    the same layout.  A complex signal runs through the real path as its real
 *    and imaginary parts on the sphere (Eq. 1 is linear in f), two real maps in
 *    the same kernel launches, so it costs two real transforms.
 *
 * Memory and execution
 *  - Every data pointer is a DEVICE pointer owned by the caller (usually a
 *    torch tensor's data_ptr); the library never frees or keeps it past the
 *    call.  Pointers must be 8-byte aligned.
 *  - stream is a hipStream_t (NULL = the legacy default stream).  Every
 *    call is asynchronous on it; results are ready when the stream is.
 *  - The library owns per-parameter plans (tables + workspace) in a cache
 *    that s2dw_release_caches() frees.  The first call with new parameters
 *    builds the plan on the host and uploads it (it synchronises the
 *    stream once).  Workspaces are per stream: the first call on a stream
 *    (or a larger batch) allocates them, and calls on different streams may
 *    overlap.  Calls on one stream from several host threads must be
 *    serialised by the caller.
 *  - Graph capture: after a first call with the same parameters and stream
 *    (which builds the plan and allocates the stream's workspace), the
 *    batched and single-map calls launch kernels only and can be captured.
 *    A captured graph holds the workspace's addresses: it stays valid until a
 *    later call on the same stream needs a larger workspace (more maps, or a
 *    larger tile shape chosen by s2dw_autotune) or s2dw_release_caches runs.
 *
 * Errors: every function returns S2DW_OK (0) or a negative code.  Argument
 * errors are found before any device work and leave outputs untouched.
 * HIP launch failures return S2DW_E_DEVICE; asynchronous device faults show
 * up at the caller's next synchronisation.  No C++ exception crosses the ABI.
 */
#ifndef S2DW_H
#define S2DW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    S2DW_OK = 0,
    S2DW_E_ARG = -1,         /* invalid argument (value, null or misaligned pointer) */
    S2DW_E_NOMEM = -2,       /* device or host allocation failed */
    S2DW_E_DEVICE = -3,      /* a HIP call failed */
    S2DW_E_UNSUPPORTED = -4, /* valid but not implemented (e.g. the sphere map of complex scaling coefficients) */
    S2DW_E_INTERNAL = -5
};

enum {
    S2DW_GRID_MW = 0,          /* every scale on the grid of band-limit L: alpha 2L-1, beta L
                                  (incl. pi), gamma 2N-1 */
    S2DW_GRID_MW_MULTIRES = 1, /* scale j on the grid of its own band-limit L_j (see below) */
    S2DW_GRID_DH = 2           /* the paper's own grid (Sec. 3.1): alpha 2L-1, beta 2L, gamma N
                                  on [0, pi) (see below) */
};
enum { S2DW_FP64 = 0, S2DW_MIXED = 1 };

typedef struct s2dw_params {
    int32_t L;         /* harmonic band-limit, 2 <= L <= 4096 */
    int32_t N;         /* azimuthal band-limit of the wavelets, 1 <= N <= min(L, 16) (Eq. 8) */
    double lambda;     /* dilation parameter, finite and > 1 (Eq. 12) */
    int32_t J_min;     /* 0 <= J_min <= J_L(lambda); scales j = 0..J_L(lambda) - J_min */
    int32_t grid;      /* S2DW_GRID_MW, S2DW_GRID_MW_MULTIRES or S2DW_GRID_DH */
    int32_t precision; /* S2DW_FP64, or S2DW_MIXED: W stored as floats; the beta, gamma and
                          alpha stages of both directions and the m'-sum of the synthesis
                          contraction (Eq. 34) computed and accumulated in FP32; the
                          Delta recursion, the analysis l-sum (Eq. 27) and the final
                          harmonic synthesis (Eq. 32) stay FP64.  Error against the FP64
                          result: about 1e-6 relative (tests bound it by 1e-5). */
    int32_t reality;   /* 1: real signal (real W), 0: complex signal (complex W) */
} s2dw_params;

/* Number of wavelet scales S = J_L(lambda) - J_min + 1 (Sec. 2.2). */
int s2dw_num_scales(const s2dw_params *p, int32_t *S);

/* Grid shape {n_gamma, n_beta, n_alpha} of one scale: {2N-1, L, 2L-1}, or {N, 2L, 2L-1}
 * for S2DW_GRID_DH (the finest scale for S2DW_GRID_MW_MULTIRES). */
int s2dw_grid_shape(const s2dw_params *p, int32_t shape[3]);

/* Bytes of the wavelet-coefficient array W of one map (all S scales, either layout). */
int s2dw_wavelet_bytes(const s2dw_params *p, uint64_t *bytes);

/* Sample grid of scale j: shape {2N-1, L_j, 2L_j-1} ({2N-1, L, 2L-1} for S2DW_GRID_MW,
 * {N, 2L, 2L-1} for S2DW_GRID_DH) and the element offset of W^j in the W of one map.
 * Host-only; shape or offset may be NULL. */
int s2dw_scale_grid(const s2dw_params *p, int32_t j, int32_t shape[3], uint64_t *offset);

/*
 * Wavelet analysis (Eq. 20 by the factoring of rotations, Eq. 25-30).
 *   flm      in : L*L complex, real-signal symmetric.
 *   W        out: [S][2N-1][L][2L-1] real (double or float, see precision).
 *   Wphi_lm  out: L*L complex harmonic scaling coefficients (Eq. 31), or NULL.
 */
int s2dw_analysis(const s2dw_params *p, const double *flm, void *W, double *Wphi_lm, void *stream);

/*
 * Wavelet analysis that allocates nothing, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments and results as s2dw_analysis (bitwise), one map.  The stage workspaces
 * live in a fixed device scratch of S2DW_NOALLOC_SCRATCH_BYTES that every GPU the library
 * runs on holds until the process ends; the call makes no hipMalloc or hipFree, and
 * records no stage-timing events.
 *  - The plan of p must exist: build it first with any call that allocates (for example
 *    s2dw_workspace_bytes, or s2dw_analysis, with the same parameters and precision);
 *    otherwise S2DW_E_ARG.
 *  - Parameters whose workspace exceeds the scratch return S2DW_E_UNSUPPORTED (about
 *    L <= 256 at N = 8; s2dw_workspace_bytes, which also counts the synthesis's partial
 *    sums, is an upper bound).
 *  - All calls on one GPU share its scratch: calls that overlap in time on one GPU (on
 *    different streams or from different host threads) race and give wrong results.  The
 *    scratch keeps the last call's contents; every call writes what it reads first.
 */
#define S2DW_NOALLOC_SCRATCH_BYTES (64ull << 20)
int s2dw_analysis_noalloc(const s2dw_params *p, const double *flm, void *W, double *Wphi_lm, void *stream);

/*
 * Wavelet synthesis (Eq. 4 through Eq. 32-41, with exact quadrature on the
 * equiangular grid).
 *   W        in : [S][2N-1][L][2L-1] real.
 *   Wphi_lm  in : L*L complex scaling coefficients, or NULL for the wavelet part only.
 *   flm_out  out: L*L complex.
 */
int s2dw_synthesis(const s2dw_params *p, const void *W, const double *Wphi_lm, double *flm_out, void *stream);

/*
 * Batched forms: `count` maps with the same parameters in contiguous arrays, map i at
 *   flm + i L*L complex, W + i S (2N-1) L (2L-1) elements, Wphi_lm + i L*L complex.
 * The maps run through the same kernel launches (the map index is a grid dimension), in
 * chunks of maps whose size the plan holds (see s2dw_autotune).  Each map's result is
 * bitwise the one of the single-map call.  The calls launch kernels only (no memset
 * nodes), so after a first call with the same parameters and stream, which allocates the
 * stream's workspace, they can be captured in a HIP graph.
 */
int s2dw_analysis_batched(const s2dw_params *p, int32_t count, const double *flm, void *W, double *Wphi_lm,
                          void *stream);
int s2dw_synthesis_batched(const s2dw_params *p, int32_t count, const void *W, const double *Wphi_lm,
                           double *flm_out, void *stream);

/*
 * Steering (steerability of the wavelet coefficients, Eq. 9-10): wavelet coefficients
 * at arbitrary third Euler angles gamma from the grid samples.  The wavelets carry only
 * the orders n with |n| < N and n = N-1 (mod 2) (Eq. 11), so W^j(alpha, beta, .) is a
 * trigonometric polynomial with those frequencies, fixed exactly by its 2N-1 samples:
 *     W(alpha, beta, gamma) = sum_g z(gamma - gamma_g) W(alpha, beta, gamma_g),
 *     z(delta) = 1/(2N-1) sum_{n carried} cos(n delta).
 * On the Driscoll-Healy grid the samples are the paper's N base orientations
 * gamma_g = pi g/N and z(delta) = 1/N sum_{n carried} cos(n delta) (z_n = 1/N).  Exact up
 * to rounding for W produced by the analysis; other input is first projected onto the
 * carried orders.
 *   count    number of maps, >= 1 (W and out hold count maps back to back).
 *   W        in : [count][S][2N-1][L][2L-1] real, doubles (S2DW_FP64) or floats (S2DW_MIXED);
 *                 with S2DW_GRID_MW_MULTIRES, count maps of the multiresolution layout.
 *   n_gamma  number of angles, 0 <= n_gamma <= 65536 (0: nothing is done).
 *   gamma    in : n_gamma angles in radians, any real values, DEVICE array of doubles.
 *   out      out: [count][S][n_gamma][L][2L-1] (multiresolution: per scale [n_gamma][L_j]
 *                 [2L_j-1], scales back to back), same element type as W; must not overlap W.
 * Only the kernel launch is asynchronous; no workspace, so it can be captured.
 */
int s2dw_steer(const s2dw_params *p, int32_t count, const void *W, int32_t n_gamma, const double *gamma, void *out,
               void *stream);

/*
 * Autotuner: times round trips (analysis + synthesis) of zero-filled probe maps on
 * `stream` for each compiled Wigner tile shape (m' slots per wave, 1, 2 or 4 depending on
 * the number of carried orders), for the alpha and gamma forms where the prime-factor
 * kernels apply (see s2dw_set_tuning), and for batch chunks 1, 2, 4, ... up to min(count,
 * what fits 8 GiB of workspace), keeps the fastest per map in the plan of p, and reports the
 * tile shape and chunk (s2dw_get_tuning reports all three).
 * Synchronises the stream; allocates probe buffers.  slots and chunk may be NULL.
 * Calls of the same plan on other streams may run meanwhile: each call uses the tile
 * shape it found when it started, and no other stream's workspace is freed.  Results
 * change only by rounding between tile shapes.
 */
int s2dw_autotune(const s2dw_params *p, int32_t count, void *stream, int32_t *slots, int32_t *chunk);

/*
 * Persistent batched form (many maps, several parameter sets, all scales): the analysis or
 * the synthesis of every group's batch as two launches of a persistent executor -- one for
 * the Wigner stages (Sec. 3.2-3.3, Eq. 27 and 34; with the input padding of the analysis and
 * the final sum of Eq. 32/41 of the synthesis), one for the beta, alpha and gamma stages
 * (Eq. 29-31 and 35-40; with the scaling coefficients of Eq. 31).  The stages of every map run
 * as work items of CU-resident workgroups that take them from a device work list in
 * dependency order, so that maps of all groups move through the stages together and no
 * per-stage launch is left.  Results equal those of s2dw_analysis_batched /
 * s2dw_synthesis_batched of each group up to rounding (the executor's Wigner tiles have their
 * own shape).
 *   groups[g].params: L, N, lambda, J_min, precision of group g; every group must have the
 *                     same precision, reality = 1, grid = S2DW_GRID_MW and N <= 8, and every
 *                     transform of its stages must be of size 2048 or less (L <= 512);
 *                     otherwise S2DW_E_UNSUPPORTED (other groups: s2dw_*_batched)
 *   groups[g].count:  maps of the group (>= 1)
 *   groups[g].flm:    [count][L^2] complex f_lm: input of the analysis, output of the synthesis
 *   groups[g].W:      [count][S][2N-1][L][2L-1] wavelet coefficients (doubles, or floats with
 *                     S2DW_MIXED): output of the analysis, input of the synthesis
 *   groups[g].Wphi_lm: [count][L^2] complex scaling coefficients (analysis output, synthesis
 *                     input), or NULL (analysis: not computed; synthesis: taken as zero)
 *   status:           device int32 (may be NULL): after the call's work, 0, or 1 if a wait of
 *                     the executor for a dependency ran past its bound (then the results are
 *                     not valid; the executor still finishes and clears its state)
 * All pointers are device memory, 8-byte aligned; arrays of different groups must not
 * overlap.  The first call with a given list (groups, buffers, stream) records its work list,
 * allocates its workspaces and uploads them (synchronously); later calls with the same list
 * only launch, so they can be captured in a graph.  The program is held until
 * s2dw_release_caches.  Calls of one program must not overlap (same stream: they don't).
 */
typedef struct s2dw_group {
    s2dw_params params;
    int32_t count;
    void *flm;
    void *W;
    void *Wphi_lm;
} s2dw_group;
int s2dw_analysis_persistent(const s2dw_group *groups, int32_t ngroups, int32_t *status, void *stream);
int s2dw_synthesis_persistent(const s2dw_group *groups, int32_t ngroups, int32_t *status, void *stream);
/* The bound of the executor's dependency waits, in polls of about 0.2 us (0: the default,
 * about three seconds), and, for tests of the bounded-wait path only, never_satisfied = 1:
 * every wait then runs out (status 1, results not valid) while the launches still finish.
 * S2DW_E_ARG if polls < 0 or never_satisfied is not 0 or 1. */
int s2dw_persistent_wait_bound(int32_t polls, int32_t never_satisfied);

/*
 * The tuning of the plan of p (built on first use): the Wigner tile shape (m' slots per
 * wave), the maps per batched launch sequence, and the form of the alpha and gamma passes
 * at the prime-factor lengths T = 2L - 1 of 2047 and 4095 (real signals): 0 two passes
 * (alpha transform, then gamma sum), 2 one fused kernel per scale wherever it applies, 1 the
 * default, fused where it was measured faster.  s2dw_autotune also times forms 0 and 2.
 * s2dw_set_tuning applies stored results (e.g. an earlier s2dw_autotune's) without timing:
 * S2DW_E_ARG for a slot count that is not compiled for the plan's carried orders, chunk < 1
 * or fuse outside 0..2.  Calls already running keep the tuning they started with; results
 * change only by rounding between tunings.  Outputs may be NULL.
 */
int s2dw_get_tuning(const s2dw_params *p, int32_t *slots, int32_t *chunk, int32_t *fuse);
int s2dw_set_tuning(const s2dw_params *p, int32_t slots, int32_t chunk, int32_t fuse);

/*
 * Device memory queries for admission control (serving):
 *   s2dw_workspace_bytes: bytes of the workspace one stream holds for a batch of `count`
 *     maps with parameters p (builds the plan of p on first use);
 *   s2dw_cache_bytes: bytes held now by all plans (tables) and stream workspaces.
 */
int s2dw_workspace_bytes(const s2dw_params *p, int32_t count, uint64_t *bytes);
int s2dw_cache_bytes(uint64_t *bytes);

/*
 * Scaling coefficients (Eq. 3, 31): W^Phi_lm = sqrt(4 pi/(2l+1)) f_lm Phi_l0.
 *   Wphi_lm  out: L*L complex, or NULL.
 *   Wphi_map out: real [L][2L-1] sphere map of the scaling coefficients
 *                 (the inverse spherical-harmonic transform of W^Phi), or NULL
 *                 (real signals only: S2DW_E_UNSUPPORTED for reality = 0).
 */
int s2dw_scaling(const s2dw_params *p, const double *flm, double *Wphi_lm, double *Wphi_map, void *stream);

/*
 * Forward spherical-harmonic transform of a real band-limited map sampled on
 * the equiangular grid [L][2L-1] (exact; the precondition of Sec. 3.1 that
 * f_lm be computed by a sampling theorem).  Only p->L is used.
 */
int s2dw_sht_forward(const s2dw_params *p, const double *f_map, double *flm, void *stream);

/* Inverse spherical-harmonic transform onto the equiangular grid [L][2L-1]. */
int s2dw_sht_inverse(const s2dw_params *p, const double *flm, double *f_map, void *stream);

/*
 * The harmonic wavelet tables of p (Sec. 2.2), written to HOST memory:
 *   kappa  [S][L]  kernel kappa^j(l) (Eq. 14-15), or NULL
 *   phi    [L]     scaling function Phi_l0 (Eq. 16), or NULL
 *   s_ln   [L][2N-1] complex directionality s_ln (Eq. 11), index n + N - 1, or NULL
 * Psi^j_ln = kappa^j(l) s_ln (Eq. 7).  Needs no GPU.
 */
int s2dw_wavelet_tables(const s2dw_params *p, double *kappa, double *phi, double *s_ln);

/*
 * Stage timing.  While enabled, each launch sequence records a HIP event on the
 * caller's stream before and after every kernel, so the time between the two is
 * that kernel's device time.  s2dw_profile(1) enables and clears the totals,
 * s2dw_profile(0) disables.  s2dw_profile_read waits for the recorded events and
 * fills up to max entries (host memory) with per-stage totals since the last clear;
 * *n receives the number of stages.  Names: pad, wigner_fwd, beta_fwd, alpha_fwd,
 * gamma_fwd, alpha_gamma_fwd (analysis; the last is the fused alpha and gamma pass that
 * the coarse scales of real signals take), gamma_adj, gamma_alpha_adj (its synthesis
 * counterpart, FP64), alpha_adj, beta_adj, wigner_adj, syn_final (synthesis), scaling,
 * steer.
 */
typedef struct s2dw_stage_time {
    char name[24];
    double ms;      /* summed device time */
    int64_t count;  /* launches */
} s2dw_stage_time;
int s2dw_profile(int enable);
int s2dw_profile_read(s2dw_stage_time *out, int32_t max, int32_t *n);

/*
 * Restricts stage timing to the named stages: names is a comma-separated list of the
 * stage names above (host string, read during the call); NULL or "" times every stage
 * (the default).  Each timed launch costs two event records on the stream, which the
 * device executes between kernels, so timing only the stage of interest keeps the
 * timed sequence close to an untimed one.  Returns S2DW_E_ARG, and keeps the previous
 * selection, if a name is not a stage name.  Needs no GPU.
 */
int s2dw_profile_stages(const char *names);

/* Human-readable text of a status code. */
const char *s2dw_strerror(int code);

/* Free every cached plan (tables and workspaces). Synchronises the device. */
void s2dw_release_caches(void);

#ifdef __cplusplus
}
#endif

#endif /* S2DW_H */
