/*
 * orc.c -- CPU reference ("oracle") for the directional scale-discretized
 * wavelet transform on the sphere (McEwen, Vandergheynst & Wiaux, "On the
 * computation of directional scale-discretized wavelet transforms on the
 * sphere", SPIE 2013).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain reference that the GPU
 * library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, table or
 * helper with the GPU library and never calls it.
 *
 * What it computes, and from which passage:
 *   - Wigner small-d functions d^l_{mn}(beta) (Sec. 3.2, Eq. 24) with the
 *     convention d^l_{mn}(beta) = <l m| exp(-i beta J_y) |l n>, from the
 *     closed-form value at l0 = max(|m|,|n|) (Wigner's explicit sum, which
 *     has a single term there) and the textbook three-term recurrence in l.
 *     Both run in long double (64-bit mantissa, 15-bit exponent), so edge
 *     values down to 2^-4096 neither underflow nor lose digits.
 *   - The inverse Wigner transform on a separable grid (Eq. 22; with the
 *     analysis coefficients of Eq. 21 it is the wavelet analysis, Eq. 20):
 *        out(a,b,g) = sum_l sum_m sum_n c^l_{mn} e^{i m alpha_a} d^l_{mn}(beta_b) e^{i n gamma_g}
 *     summed over l first, then n, then m, each as a plain direct sum.
 *   - The forward Wigner transform (Eq. 23 / Eq. 33) of samples on the
 *     equiangular grid alpha_a = 2 pi a/(2L-1), beta_b = pi(2b+1)/(2L-1)
 *     (b < L), gamma_g = 2 pi g/(2N-1), by quadrature: the uniform rules in
 *     alpha (Eq. 19) and gamma, and in beta the unique trigonometric
 *     polynomial of degree <= L-1 through the samples extended to the full
 *     circle with the parity (-1)^{m+n}, integrated against
 *     sin(beta) d^l_{mn}(beta) over [0, pi] by a Gauss-Legendre rule in beta
 *     with enough nodes (4L+16) that the integral of this entire integrand is
 *     converged to rounding (the nodes and weights, sin(beta) included, come
 *     from the caller).
 *   - The same forward transform on the paper's Driscoll-Healy grid
 *     (Sec. 3.1, Eq. 17-18; gamma on [0, pi) with weight 2 pi z_n, Eq. 39).
 *
 * Complex arrays are interleaved (re, im) doubles.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

static const ld PI_L = 3.141592653589793238462643383279502884L;

static int iabs_(int x) { return x < 0 ? -x : x; }
static int imax_(int a, int b) { return a > b ? a : b; }
static int pmod_(long long x, long long m) { long long r = x % m; return (int)(r < 0 ? r + m : r); }

/* sqrt(binomial(2a, a+k)) for 0 <= |k| <= a, as a product of ratios. */
static ld sqrt_binom_center(int a, int k)
{
    int kk = iabs_(k);
    ld c = 1.0L;
    /* C(2a, a+kk) = prod_{i=1}^{a-kk} (a+kk+i)/i */
    for (int i = 1; i <= a - kk; ++i) c *= (ld)(a + kk + i) / (ld)i;
    return sqrtl(c);
}

/* d^{l0}_{mn}(beta) at l0 = max(|m|,|n|): the single surviving term of
 * Wigner's explicit sum.  ch = cos(beta/2), sh = sin(beta/2). */
static ld wigner_edge(int m, int n, ld ch, ld sh)
{
    int l0 = imax_(iabs_(m), iabs_(n));
    if (iabs_(m) >= iabs_(n)) {
        if (m == l0) {
            /* d^l_{l n} = (-1)^{l-n} sqrt(C(2l, l+n)) cos^{l+n} sin^{l-n} */
            ld v = sqrt_binom_center(l0, n) * powl(ch, l0 + n) * powl(sh, l0 - n);
            return ((l0 - n) & 1) ? -v : v;
        }
        /* m = -l0: d^l_{-l n} = sqrt(C(2l, l+n)) cos^{l-n} sin^{l+n} */
        return sqrt_binom_center(l0, n) * powl(ch, l0 - n) * powl(sh, l0 + n);
    }
    if (n == l0) {
        /* d^l_{m l} = sqrt(C(2l, l+m)) cos^{l+m} sin^{l-m} */
        return sqrt_binom_center(l0, m) * powl(ch, l0 + m) * powl(sh, l0 - m);
    }
    /* n = -l0: d^l_{m,-l} = (-1)^{l+m} sqrt(C(2l, l+m)) cos^{l-m} sin^{l+m} */
    {
        ld v = sqrt_binom_center(l0, m) * powl(ch, l0 - m) * powl(sh, l0 + m);
        return ((l0 + m) & 1) ? -v : v;
    }
}

/* d^l_{mn}(beta) for l = 0..L-1 (zero for l < max(|m|,|n|)).
 * Three-term recurrence in l (e.g. Varshalovich et al. 1989, Sec. 4.8):
 *   l sqrt(((l+1)^2-m^2)((l+1)^2-n^2)) d^{l+1}
 *     = (2l+1)(l(l+1) cos(beta) - m n) d^l - (l+1) sqrt((l^2-m^2)(l^2-n^2)) d^{l-1}. */
static void wigner_run(int L, int m, int n, ld cb, ld ch, ld sh, ld *d)
{
    int l0 = imax_(iabs_(m), iabs_(n));
    for (int l = 0; l < L && l < l0; ++l) d[l] = 0.0L;
    if (l0 >= L) return;
    d[l0] = wigner_edge(m, n, ch, sh);
    ld mm = (ld)m * m, nn = (ld)n * n, mn = (ld)m * n;
    for (int l = l0; l + 1 < L; ++l) {
        if (l == 0) { d[1] = cb * d[0]; continue; } /* m = n = 0: P_1 */
        ld fl = (ld)l;
        ld prev = (l > l0) ? d[l - 1] : 0.0L;
        ld a = (2.0L * fl + 1.0L) * (fl * (fl + 1.0L) * cb - mn);
        ld b = (fl + 1.0L) * sqrtl((fl * fl - mm) * (fl * fl - nn));
        ld den = fl * sqrtl(((fl + 1.0L) * (fl + 1.0L) - mm) * ((fl + 1.0L) * (fl + 1.0L) - nn));
        d[l + 1] = (a * d[l] - b * prev) / den;
    }
}

/* Exported for the tests: d^l_{mn}(beta), l < L, as doubles. */
void orc_wigner_d(int L, int m, int n, double beta, double *out)
{
    ld *d = (ld *)malloc(sizeof(ld) * (size_t)L);
    ld b = (ld)beta;
    wigner_run(L, m, n, cosl(b), cosl(b / 2.0L), sinl(b / 2.0L), d);
    for (int l = 0; l < L; ++l) out[l] = (double)d[l];
    free(d);
}

/* Same, returning long double values split as (hi, lo) doubles so that the
 * tests can see digits beyond double precision. */
void orc_wigner_d_ext(int L, int m, int n, double beta, double *hi, double *lo)
{
    ld *d = (ld *)malloc(sizeof(ld) * (size_t)L);
    ld b = (ld)beta;
    wigner_run(L, m, n, cosl(b), cosl(b / 2.0L), sinl(b / 2.0L), d);
    for (int l = 0; l < L; ++l) { hi[l] = (double)d[l]; lo[l] = (double)(d[l] - (ld)hi[l]); }
    free(d);
}

/* Coefficient c^l_{mn} for scale s, in one of two modes:
 *   separable: c = f_{lm} conj(Psi^s_{ln})  (Eq. 20, analysis)
 *   general:   c = cgen[s][l][m+L-1][ni]     (any Wigner expansion, Eq. 22) */
typedef struct {
    int L, nn, S;
    const double *flm;  /* [l*l+l+m] complex */
    const double *psi;  /* [s][l][ni] complex */
    const double *cgen; /* [s][l][m+L-1][ni] complex */
} coef_src;

static void coef_get(const coef_src *c, int s, int l, int m, int ni, ld *re, ld *im)
{
    if (c->cgen) {
        size_t M = 2 * (size_t)c->L - 1;
        size_t idx = (((size_t)s * c->L + l) * M + (size_t)(m + c->L - 1)) * c->nn + ni;
        *re = c->cgen[2 * idx];
        *im = c->cgen[2 * idx + 1];
        return;
    }
    size_t fi = (size_t)l * l + l + m;
    ld fr = c->flm[2 * fi], fim = c->flm[2 * fi + 1];
    size_t pi = ((size_t)s * c->L + l) * c->nn + ni;
    ld pr = c->psi[2 * pi], pim = -c->psi[2 * pi + 1]; /* conj(Psi) */
    *re = fr * pr - fim * pim;
    *im = fr * pim + fim * pr;
}

/*
 * Inverse Wigner transform on a separable grid:
 *   out[s][g][b][a] = sum_{l<L} sum_{|m|<=l} sum_{ni} c^l_{m n_ni} e^{i m alpha_a} d^l_{m n}(beta_b) e^{i n gamma_g}
 * with alpha_a = 2 pi a / na (a < na), gamma_g = 2 pi g / mg (g < ng), beta_b = betas[b].
 * out is complex [S][ng][nb][na].
 */
static int inverse_core(const coef_src *src, const int *nlist, int nb, const double *betas,
                        int na, int ng, int mg, double *out, int nthreads)
{
    int L = src->L, nn = src->nn, S = src->S;
    int M = 2 * L - 1;
    double *ea = (double *)malloc(sizeof(double) * 2 * (size_t)na);
    double *eg = (double *)malloc(sizeof(double) * 2 * (size_t)mg);
    if (!ea || !eg) { free(ea); free(eg); return -1; }
    for (int k = 0; k < na; ++k) {
        ld t = 2.0L * PI_L * (ld)k / (ld)na;
        ea[2 * k] = (double)cosl(t); ea[2 * k + 1] = (double)sinl(t);
    }
    for (int k = 0; k < mg; ++k) {
        ld t = 2.0L * PI_L * (ld)k / (ld)mg;
        eg[2 * k] = (double)cosl(t); eg[2 * k + 1] = (double)sinl(t);
    }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int b = 0; b < nb; ++b) {
        ld beta = (ld)betas[b];
        ld cb = cosl(beta), ch = cosl(beta / 2.0L), sh = sinl(beta / 2.0L);
        ld *d = (ld *)malloc(sizeof(ld) * (size_t)L);
        double *G = (double *)calloc((size_t)S * nn * M * 2, sizeof(double));
        double *H = (double *)malloc(sizeof(double) * (size_t)M * 2);
        if (!d || !G || !H) {
#pragma omp atomic write
            err = -1;
            free(d); free(G); free(H);
            continue;
        }
        /* G[s][ni][m] = sum_l c^l_{mn} d^l_{mn}(beta) */
        for (int ni = 0; ni < nn; ++ni) {
            int n = nlist[ni];
            for (int m = -(L - 1); m <= L - 1; ++m) {
                int l0 = imax_(iabs_(m), iabs_(n));
                if (l0 >= L) continue;
                wigner_run(L, m, n, cb, ch, sh, d);
                for (int s = 0; s < S; ++s) {
                    ld ar = 0.0L, ai = 0.0L;
                    for (int l = l0; l < L; ++l) {
                        ld cr, ci;
                        coef_get(src, s, l, m, ni, &cr, &ci);
                        ar += cr * d[l];
                        ai += ci * d[l];
                    }
                    size_t gi = ((size_t)s * nn + ni) * M + (size_t)(m + L - 1);
                    G[2 * gi] = (double)ar;
                    G[2 * gi + 1] = (double)ai;
                }
            }
        }
        /* H_m = sum_n G_{mn} e^{i n gamma_g};  out_a = sum_m H_m e^{i m alpha_a} */
        for (int s = 0; s < S; ++s) {
            for (int g = 0; g < ng; ++g) {
                for (int mi = 0; mi < M; ++mi) {
                    double hr = 0.0, hi = 0.0;
                    for (int ni = 0; ni < nn; ++ni) {
                        size_t gi = ((size_t)s * nn + ni) * M + mi;
                        int k = pmod_((long long)nlist[ni] * g, mg);
                        double wr = eg[2 * k], wi = eg[2 * k + 1];
                        hr += G[2 * gi] * wr - G[2 * gi + 1] * wi;
                        hi += G[2 * gi] * wi + G[2 * gi + 1] * wr;
                    }
                    H[2 * mi] = hr; H[2 * mi + 1] = hi;
                }
                for (int a = 0; a < na; ++a) {
                    double sr = 0.0, si = 0.0;
                    for (int mi = 0; mi < M; ++mi) {
                        int m = mi - (L - 1);
                        int k = pmod_((long long)m * a, na);
                        double wr = ea[2 * k], wi = ea[2 * k + 1];
                        sr += H[2 * mi] * wr - H[2 * mi + 1] * wi;
                        si += H[2 * mi] * wi + H[2 * mi + 1] * wr;
                    }
                    size_t oi = (((size_t)s * ng + g) * nb + b) * na + a;
                    out[2 * oi] = sr; out[2 * oi + 1] = si;
                }
            }
        }
        free(d); free(G); free(H);
    }
    free(ea); free(eg);
    return err;
}

/* Wavelet analysis on a separable grid (Eq. 20 with Eq. 24):
 *   W^s(rho) = sum f_{lm} conj(Psi^s_{ln}) e^{i m alpha} d^l_{mn}(beta) e^{i n gamma}. */
int orc_analysis(int L, int nn, const int *nlist, int S, const double *flm, const double *psi,
                 int nb, const double *betas, int na, int ng, int mg, double *out, int nthreads)
{
    coef_src c = {L, nn, S, flm, psi, NULL};
    return inverse_core(&c, nlist, nb, betas, na, ng, mg, out, nthreads);
}

/* Inverse Wigner transform of arbitrary coefficients c[s][l][m+L-1][ni] (Eq. 22 with the
 * normalisation (2l+1)/(8 pi^2) already folded into c). */
int orc_inverse_wigner(int L, int nn, const int *nlist, int S, const double *cgen,
                       int nb, const double *betas, int na, int ng, int mg, double *out, int nthreads)
{
    coef_src c = {L, nn, S, NULL, NULL, cgen};
    return inverse_core(&c, nlist, nb, betas, na, ng, mg, out, nthreads);
}

/*
 * Step shared by both forward transforms: the alpha and gamma integrals by the
 * uniform quadratures (Eq. 19 and its gamma analogue), giving for every scale,
 * n and sampled beta the function
 *   Gt[s][ni][b][m+L-1] = wa * wg * sum_g sum_a W[s][g][b][a] e^{-i m alpha_a} e^{-i n gamma_g}
 * with alpha_a = 2 pi a / na, gamma_g = 2 pi g / mg, wa = 2 pi / na, and wg
 * supplied per n (gw[ni]).
 */
static int alpha_gamma_rules(int L, int nn, const int *nlist, int S, const double *W,
                             int nb, int na, int ng, int mg, const double *gw,
                             double *Gt, int nthreads)
{
    int M = 2 * L - 1;
    double *ea = (double *)malloc(sizeof(double) * 2 * (size_t)na);
    double *eg = (double *)malloc(sizeof(double) * 2 * (size_t)mg);
    if (!ea || !eg) { free(ea); free(eg); return -1; }
    for (int k = 0; k < na; ++k) {
        ld t = 2.0L * PI_L * (ld)k / (ld)na;
        ea[2 * k] = (double)cosl(t); ea[2 * k + 1] = (double)sinl(t);
    }
    for (int k = 0; k < mg; ++k) {
        ld t = 2.0L * PI_L * (ld)k / (ld)mg;
        eg[2 * k] = (double)cosl(t); eg[2 * k + 1] = (double)sinl(t);
    }
    double wa = (double)(2.0L * PI_L / (ld)na);
    int err = 0;
#pragma omp parallel for collapse(2) schedule(dynamic, 1) num_threads(nthreads)
    for (int s = 0; s < S; ++s) {
        for (int b = 0; b < nb; ++b) {
            double *Hg = (double *)malloc(sizeof(double) * 2 * (size_t)ng * M);
            if (!Hg) {
#pragma omp atomic write
                err = -1;
                continue;
            }
            /* Hg[g][m] = sum_a W e^{-i m alpha_a} */
            for (int g = 0; g < ng; ++g) {
                const double *row = W + 2 * ((((size_t)s * ng + g) * nb + b) * (size_t)na);
                for (int mi = 0; mi < M; ++mi) {
                    int m = mi - (L - 1);
                    double sr = 0.0, si = 0.0;
                    for (int a = 0; a < na; ++a) {
                        int k = pmod_(-(long long)m * a, na);
                        double wr = ea[2 * k], wi = ea[2 * k + 1];
                        sr += row[2 * a] * wr - row[2 * a + 1] * wi;
                        si += row[2 * a] * wi + row[2 * a + 1] * wr;
                    }
                    Hg[2 * ((size_t)g * M + mi)] = sr;
                    Hg[2 * ((size_t)g * M + mi) + 1] = si;
                }
            }
            for (int ni = 0; ni < nn; ++ni) {
                for (int mi = 0; mi < M; ++mi) {
                    double sr = 0.0, si = 0.0;
                    for (int g = 0; g < ng; ++g) {
                        int k = pmod_(-(long long)nlist[ni] * g, mg);
                        double wr = eg[2 * k], wi = eg[2 * k + 1];
                        double hr = Hg[2 * ((size_t)g * M + mi)], hi = Hg[2 * ((size_t)g * M + mi) + 1];
                        sr += hr * wr - hi * wi;
                        si += hr * wi + hi * wr;
                    }
                    size_t o = (((size_t)s * nn + ni) * nb + b) * M + mi;
                    Gt[2 * o] = wa * gw[ni] * sr;
                    Gt[2 * o + 1] = wa * gw[ni] * si;
                }
            }
            free(Hg);
        }
    }
    free(ea); free(eg);
    return err;
}

/*
 * Forward Wigner transform of samples on the equiangular grid with L samples in
 * beta (beta_b = pi(2b+1)/(2L-1)), na = 2L-1 in alpha and ng = mg = 2N-1 in gamma:
 *   out[s][l][m+L-1][ni] = int W^s(rho) D^l_{mn}(rho) d rho     (Eq. 23)
 * W complex [S][ng][L][na]; xgl, wgl: quadrature colatitudes in [0, pi] and weights
 * (including the sin(beta) of the measure).
 * Only the columns m in [m_lo, m_hi] are produced (the rest of out is left as is).
 */
/* First step of the forward transform on the equiangular grid: the alpha and gamma
 * rules for nb rows of samples, Gt complex [S][nn][nb][2L-1] (see alpha_gamma_rules). */
int orc_alpha_gamma_rules_mw(int L, int nn, const int *nlist, int S, const double *W, int nb,
                             int na, int ng, int mg, double *Gt, int nthreads)
{
    double *gw = (double *)malloc(sizeof(double) * (size_t)nn);
    if (!gw) return -1;
    for (int ni = 0; ni < nn; ++ni) gw[ni] = (double)(2.0L * PI_L / (ld)ng);
    int err = alpha_gamma_rules(L, nn, nlist, S, W, nb, na, ng, mg, gw, Gt, nthreads);
    free(gw);
    return err;
}

/* Second step: the beta integral of the interpolant of Gt (all L rows) against
 * sin(beta) d^l_mn(beta), for the columns m in [m_lo, m_hi], or, when cols is not NULL,
 * for the ncols columns listed in cols (each column is independent of the others). */
static int beta_wigner_cols(int L, int nn, const int *nlist, int S, const double *Gt,
                            int ngl, const double *xgl, const double *wgl,
                            int m_lo, int m_hi, int ncols_list, const int *cols, double *out, int nthreads)
{
    int M = 2 * L - 1;
    int T = 2 * L - 1; /* samples on the full circle after the extension */
    int err = 0;
    /* e^{i pi k/(2L-1)} for the extended beta grid beta_t = pi(2t+1)/(2L-1) */
    int P2 = 2 * T;
    double *eb = (double *)malloc(sizeof(double) * 2 * (size_t)P2);
    /* e^{i p theta_k} at the quadrature colatitudes, p in [-(L-1), L-1] */
    double *ek = (double *)malloc(sizeof(double) * 2 * (size_t)ngl * M);
    if (!eb || !ek) { free(eb); free(ek); return -1; }
    for (int k = 0; k < P2; ++k) {
        ld t = PI_L * (ld)k / (ld)T;
        eb[2 * k] = (double)cosl(t); eb[2 * k + 1] = (double)sinl(t);
    }
    for (int k = 0; k < ngl; ++k) {
        ld th = (ld)xgl[k];
        for (int p = -(L - 1); p <= L - 1; ++p) {
            size_t o = (size_t)k * M + (size_t)(p + L - 1);
            ek[2 * o] = (double)cosl((ld)p * th);
            ek[2 * o + 1] = (double)sinl((ld)p * th);
        }
    }
    if (m_lo < -(L - 1)) m_lo = -(L - 1);
    if (m_hi > L - 1) m_hi = L - 1;
    int ncols = cols ? ncols_list : m_hi - m_lo + 1;
    if (cols)
        for (int ci = 0; ci < ncols; ++ci)
            if (cols[ci] < -(L - 1) || cols[ci] > L - 1) { free(eb); free(ek); return -2; }
#pragma omp parallel for collapse(2) schedule(dynamic, 1) num_threads(nthreads)
    for (int ni = 0; ni < nn; ++ni) {
        for (int ci = 0; ci < ncols; ++ci) {
            int m = cols ? cols[ci] : m_lo + ci;
            int n = nlist[ni];
            int mi = m + L - 1;
            int par = ((m + n) % 2 == 0) ? 1 : -1;
            double *ext = (double *)malloc(sizeof(double) * 2 * (size_t)T);
            double *gh = (double *)malloc(sizeof(double) * 2 * (size_t)M);
            double *gk = (double *)malloc(sizeof(double) * 2 * (size_t)ngl * S);
            ld *d = (ld *)malloc(sizeof(ld) * (size_t)L);
            if (!ext || !gh || !gk || !d) {
#pragma omp atomic write
                err = -1;
                free(ext); free(gh); free(gk); free(d);
                continue;
            }
            for (int s = 0; s < S; ++s) {
                /* samples extended to the full circle: G(2 pi - beta) = (-1)^{m+n} G(beta) */
                for (int t = 0; t < T; ++t) {
                    int src = t < L ? t : (2 * L - 2 - t);
                    double sg = t < L ? 1.0 : (double)par;
                    size_t o = (((size_t)s * nn + ni) * L + src) * M + mi;
                    ext[2 * t] = sg * Gt[2 * o];
                    ext[2 * t + 1] = sg * Gt[2 * o + 1];
                }
                /* trigonometric interpolation: Ghat(p) = (1/T) sum_t ext_t e^{-i p beta_t} */
                for (int p = -(L - 1); p <= L - 1; ++p) {
                    double sr = 0.0, si = 0.0;
                    for (int t = 0; t < T; ++t) {
                        int k = pmod_(-(long long)p * (2 * t + 1), P2);
                        double wr = eb[2 * k], wi = eb[2 * k + 1];
                        sr += ext[2 * t] * wr - ext[2 * t + 1] * wi;
                        si += ext[2 * t] * wi + ext[2 * t + 1] * wr;
                    }
                    gh[2 * (p + L - 1)] = sr / (double)T;
                    gh[2 * (p + L - 1) + 1] = si / (double)T;
                }
                /* the interpolant at the quadrature colatitudes */
                for (int k = 0; k < ngl; ++k) {
                    const double *e = ek + 2 * (size_t)k * M;
                    double sr = 0.0, si = 0.0;
                    for (int pi = 0; pi < M; ++pi) {
                        double gr = gh[2 * pi], gi = gh[2 * pi + 1];
                        sr += gr * e[2 * pi] - gi * e[2 * pi + 1];
                        si += gr * e[2 * pi + 1] + gi * e[2 * pi];
                    }
                    gk[2 * ((size_t)s * ngl + k)] = sr;
                    gk[2 * ((size_t)s * ngl + k) + 1] = si;
                }
            }
            /* out^l = sum_k w_k G(beta_k) d^l_{mn}(beta_k) */
            for (int s = 0; s < S; ++s)
                for (int l = 0; l < L; ++l) {
                    size_t o = (((size_t)s * L + l) * M + mi) * nn + ni;
                    out[2 * o] = 0.0; out[2 * o + 1] = 0.0;
                }
            ld *acc = (ld *)calloc((size_t)S * L * 2, sizeof(ld));
            if (!acc) {
#pragma omp atomic write
                err = -1;
                free(ext); free(gh); free(gk); free(d);
                continue;
            }
            for (int k = 0; k < ngl; ++k) {
                ld th = (ld)xgl[k];
                wigner_run(L, m, n, cosl(th), cosl(th / 2.0L), sinl(th / 2.0L), d);
                for (int s = 0; s < S; ++s) {
                    ld gr = gk[2 * ((size_t)s * ngl + k)] * (ld)wgl[k];
                    ld gi = gk[2 * ((size_t)s * ngl + k) + 1] * (ld)wgl[k];
                    for (int l = 0; l < L; ++l) {
                        acc[2 * ((size_t)s * L + l)] += gr * d[l];
                        acc[2 * ((size_t)s * L + l) + 1] += gi * d[l];
                    }
                }
            }
            for (int s = 0; s < S; ++s)
                for (int l = 0; l < L; ++l) {
                    size_t o = (((size_t)s * L + l) * M + mi) * nn + ni;
                    out[2 * o] = (double)acc[2 * ((size_t)s * L + l)];
                    out[2 * o + 1] = (double)acc[2 * ((size_t)s * L + l) + 1];
                }
            free(acc); free(ext); free(gh); free(gk); free(d);
        }
    }
    free(eb); free(ek);
    return err;
}

int orc_beta_wigner_mw(int L, int nn, const int *nlist, int S, const double *Gt,
                       int ngl, const double *xgl, const double *wgl,
                       int m_lo, int m_hi, double *out, int nthreads)
{
    return beta_wigner_cols(L, nn, nlist, S, Gt, ngl, xgl, wgl, m_lo, m_hi, 0, NULL, out, nthreads);
}

int orc_beta_wigner_mw_cols(int L, int nn, const int *nlist, int S, const double *Gt,
                            int ngl, const double *xgl, const double *wgl,
                            int ncols, const int *cols, double *out, int nthreads)
{
    return beta_wigner_cols(L, nn, nlist, S, Gt, ngl, xgl, wgl, -(L - 1), L - 1, ncols, cols, out, nthreads);
}

int orc_forward_wigner_mw(int L, int nn, const int *nlist, int S, const double *W,
                          int na, int ng, int mg, int ngl, const double *xgl, const double *wgl,
                          int m_lo, int m_hi, double *out, int nthreads)
{
    int M = 2 * L - 1;
    double *Gt = (double *)malloc(sizeof(double) * 2 * (size_t)S * nn * L * M);
    if (!Gt) return -1;
    int err = orc_alpha_gamma_rules_mw(L, nn, nlist, S, W, L, na, ng, mg, Gt, nthreads);
    if (!err) err = orc_beta_wigner_mw(L, nn, nlist, S, Gt, ngl, xgl, wgl, m_lo, m_hi, out, nthreads);
    free(Gt);
    return err;
}

/*
 * Forward Wigner transform on the paper's Driscoll-Healy discretisation
 * (Sec. 3.1): beta_t = pi(2t+1)/(4L), t < 2L, weighted by q(beta_t) (Eq. 18);
 * alpha_a = 2 pi a/(2L-1); gamma_g = pi g/N, g < N, weighted by 2 pi z_n
 * (Eq. 39).  qw: the 2L quadrature weights; zw[ni]: z_n per n.
 *   out[s][l][m+L-1][ni] = sum_t q_t Gt(beta_t) d^l_{mn}(beta_t)       (Eq. 34 + 40)
 */
int orc_forward_wigner_dh(int L, int nn, const int *nlist, int S, const double *W,
                          int na, int ng, int mg, const double *zw, const double *qw,
                          double *out, int nthreads)
{
    int M = 2 * L - 1;
    int nb = 2 * L;
    double *gw = (double *)malloc(sizeof(double) * (size_t)nn);
    double *Gt = (double *)malloc(sizeof(double) * 2 * (size_t)S * nn * nb * M);
    if (!gw || !Gt) { free(gw); free(Gt); return -1; }
    /* the gamma rule of Eq. 39 is 2 pi z_n times a plain sum; alpha_gamma_rules
       multiplies by 2 pi/na itself */
    for (int ni = 0; ni < nn; ++ni) gw[ni] = (double)(2.0L * PI_L) * zw[ni];
    int err = alpha_gamma_rules(L, nn, nlist, S, W, nb, na, ng, mg, gw, Gt, nthreads);
    if (err) { free(gw); free(Gt); return err; }
#pragma omp parallel for collapse(2) schedule(dynamic, 1) num_threads(nthreads)
    for (int ni = 0; ni < nn; ++ni) {
        for (int mi = 0; mi < M; ++mi) {
            int m = mi - (L - 1), n = nlist[ni];
            ld *d = (ld *)malloc(sizeof(ld) * (size_t)L);
            ld *acc = (ld *)calloc((size_t)S * L * 2, sizeof(ld));
            if (!d || !acc) {
#pragma omp atomic write
                err = -1;
                free(d); free(acc);
                continue;
            }
            for (int t = 0; t < nb; ++t) {
                ld th = PI_L * (ld)(2 * t + 1) / (ld)(4 * L);
                wigner_run(L, m, n, cosl(th), cosl(th / 2.0L), sinl(th / 2.0L), d);
                for (int s = 0; s < S; ++s) {
                    size_t o = (((size_t)s * nn + ni) * nb + t) * M + mi;
                    ld gr = (ld)Gt[2 * o] * (ld)qw[t], gi = (ld)Gt[2 * o + 1] * (ld)qw[t];
                    for (int l = 0; l < L; ++l) {
                        acc[2 * ((size_t)s * L + l)] += gr * d[l];
                        acc[2 * ((size_t)s * L + l) + 1] += gi * d[l];
                    }
                }
            }
            for (int s = 0; s < S; ++s)
                for (int l = 0; l < L; ++l) {
                    size_t o = (((size_t)s * L + l) * M + mi) * nn + ni;
                    out[2 * o] = (double)acc[2 * ((size_t)s * L + l)];
                    out[2 * o + 1] = (double)acc[2 * ((size_t)s * L + l) + 1];
                }
            free(d); free(acc);
        }
    }
    free(gw); free(Gt);
    return err;
}
