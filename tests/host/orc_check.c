/* Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the oracle (orc.c):
 * calls every exported routine on small inputs and checks two closed-form facts on the way,
 * the round trip of random Wigner coefficients through the inverse transform and the exact
 * forward transforms on the equiangular and Driscoll-Healy grids.  Exit status 0 and no
 * sanitizer report is a pass. */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int orc_inverse_wigner(int L, int nn, const int *nlist, int S, const double *cgen, int nb, const double *betas,
                       int na, int ng, int mg, double *out, int nthreads);
int orc_analysis(int L, int nn, const int *nlist, int S, const double *flm, const double *psi, int nb,
                 const double *betas, int na, int ng, int mg, double *out, int nthreads);
int orc_forward_wigner_mw(int L, int nn, const int *nlist, int S, const double *W, int na, int ng, int mg, int ngl,
                          const double *xgl, const double *wgl, int m_lo, int m_hi, double *out, int nthreads);
int orc_alpha_gamma_rules_mw(int L, int nn, const int *nlist, int S, const double *W, int nb, int na, int ng, int mg,
                             double *Gt, int nthreads);
int orc_beta_wigner_mw_cols(int L, int nn, const int *nlist, int S, const double *Gt, int ngl, const double *xgl,
                            const double *wgl, int ncols, const int *cols, double *out, int nthreads);
int orc_forward_wigner_dh(int L, int nn, const int *nlist, int S, const double *W, int na, int ng, int mg,
                          const double *zw, const double *qw, double *out, int nthreads);
void orc_wigner_d(int L, int m, int n, double beta, double *out);
void orc_wigner_d_ext(int L, int m, int n, double beta, double *hi, double *lo);

static unsigned long long rs = 12345;
static double urand(void) {
    rs = rs * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(rs >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

/* Gauss-Legendre nodes on [-1, 1] by Newton's method on P_n */
static void leggauss(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            pp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

int main(void) {
    const int L = 8, N = 3, S = 2, nn = 2, M = 2 * L - 1;
    const int nlist[2] = {-2, 0};  /* any orders with |n| < N */
    int fails = 0;
    /* coefficients c[s][l][m+L-1][ni], zero where |m| > l or |n| > l */
    size_t nc = (size_t)S * L * M * nn;
    double *c = calloc(2 * nc, sizeof(double));
    for (int s = 0; s < S; ++s)
        for (int l = 0; l < L; ++l)
            for (int m = -l; m <= l; ++m)
                for (int ni = 0; ni < nn; ++ni)
                    if (abs(nlist[ni]) <= l) {
                        size_t o = (((size_t)s * L + l) * M + m + L - 1) * nn + ni;
                        c[2 * o] = urand();
                        c[2 * o + 1] = urand();
                    }
    /* equiangular grid: inverse, then the exact forward transform */
    double *bmw = malloc(sizeof(double) * L);
    for (int b = 0; b < L; ++b) bmw[b] = M_PI * (2.0 * b + 1.0) / (2.0 * L - 1.0);
    const int G = 2 * N - 1;
    double *W = calloc(2 * (size_t)S * G * L * M, sizeof(double));
    if (orc_inverse_wigner(L, nn, nlist, S, c, L, bmw, M, G, G, W, 2) != 0) ++fails;
    const int ngl = 4 * L + 16;
    double *xg = malloc(sizeof(double) * ngl), *wg = malloc(sizeof(double) * ngl);
    leggauss(ngl, xg, wg);
    for (int k = 0; k < ngl; ++k) {
        double b = 0.5 * M_PI * (xg[k] + 1.0);
        wg[k] = 0.5 * M_PI * wg[k] * sin(b);
        xg[k] = b;
    }
    double *f = calloc(2 * nc, sizeof(double));
    if (orc_forward_wigner_mw(L, nn, nlist, S, W, M, G, G, ngl, xg, wg, -(L - 1), L - 1, f, 2) != 0) ++fails;
    double err = 0.0;
    for (int s = 0; s < S; ++s)
        for (int l = 0; l < L; ++l)
            for (int mi = 0; mi < M; ++mi)
                for (int ni = 0; ni < nn; ++ni) {
                    size_t o = (((size_t)s * L + l) * M + mi) * nn + ni;
                    double sc = (2.0 * l + 1.0) / (8.0 * M_PI * M_PI);
                    err = fmax(err, fabs(f[2 * o] * sc - c[2 * o]) + fabs(f[2 * o + 1] * sc - c[2 * o + 1]));
                }
    if (!(err < 1e-10)) {
        printf("equiangular round trip error %g\n", err);
        ++fails;
    }
    /* the two steps separately on a few columns */
    double *Gt = calloc(2 * (size_t)S * nn * L * M, sizeof(double));
    if (orc_alpha_gamma_rules_mw(L, nn, nlist, S, W, L, M, G, G, Gt, 2) != 0) ++fails;
    const int cols[3] = {-3, 0, L - 1};
    double *f2 = calloc(2 * nc, sizeof(double));
    if (orc_beta_wigner_mw_cols(L, nn, nlist, S, Gt, ngl, xg, wg, 3, cols, f2, 2) != 0) ++fails;
    /* Driscoll-Healy grid: 2L colatitudes, N orientations on [0, pi) */
    double *bdh = malloc(sizeof(double) * 2 * L), *q = malloc(sizeof(double) * 2 * L), zw[2];
    for (int t = 0; t < 2 * L; ++t) {
        bdh[t] = M_PI * (2.0 * t + 1.0) / (4.0 * L);
        double acc = 0.0;
        for (int k = 0; k < L; ++k) acc += sin((2 * k + 1) * bdh[t]) / (2 * k + 1);
        q[t] = (2.0 / L) * sin(bdh[t]) * acc;
    }
    zw[0] = zw[1] = 1.0 / N;
    /* orders of the Driscoll-Healy grid must match N - 1 mod 2 */
    const int ndh[2] = {-2, 2};
    for (size_t o = 0; o < nc; ++o)
        if (abs(ndh[o % nn]) > (int)((o / nn / M) % L)) c[2 * o] = c[2 * o + 1] = 0.0;
    double *Wd = calloc(2 * (size_t)S * N * 2 * L * M, sizeof(double));
    if (orc_inverse_wigner(L, nn, ndh, S, c, 2 * L, bdh, M, N, 2 * N, Wd, 2) != 0) ++fails;
    double *fd = calloc(2 * nc, sizeof(double));
    if (orc_forward_wigner_dh(L, nn, ndh, S, Wd, M, N, 2 * N, zw, q, fd, 2) != 0) ++fails;
    err = 0.0;
    for (size_t o = 0; o < nc; ++o) {
        int l = (int)((o / nn / M) % L);
        double sc = (2.0 * l + 1.0) / (8.0 * M_PI * M_PI);
        err = fmax(err, fabs(fd[2 * o] * sc - c[2 * o]) + fabs(fd[2 * o + 1] * sc - c[2 * o + 1]));
    }
    if (!(err < 1e-10)) {
        printf("Driscoll-Healy round trip error %g\n", err);
        ++fails;
    }
    /* separable analysis and the Wigner d routines */
    double *flm = calloc(2 * (size_t)L * L, sizeof(double)), *psi = calloc(2 * (size_t)S * L * nn, sizeof(double));
    for (int i = 0; i < 2 * L * L; ++i) flm[i] = urand();
    for (int i = 0; i < 2 * S * L * nn; ++i) psi[i] = urand();
    double *Wa = calloc(2 * (size_t)S * G * L * M, sizeof(double));
    if (orc_analysis(L, nn, nlist, S, flm, psi, L, bmw, M, G, G, Wa, 2) != 0) ++fails;
    double d[8], hi[8], lo[8];
    orc_wigner_d(L, 3, -2, 1.1, d);
    orc_wigner_d_ext(L, -7, 7, 3.0, hi, lo);
    for (int l = 0; l < L; ++l)
        if (!isfinite(d[l]) || !isfinite(hi[l]) || !isfinite(lo[l])) ++fails;
    free(c); free(bmw); free(W); free(xg); free(wg); free(f); free(Gt); free(f2); free(bdh); free(q);
    free(Wd); free(fd); free(flm); free(psi); free(Wa);
    printf("orc_check: %d failures\n", fails);
    return fails == 0 ? 0 : 1;
}
