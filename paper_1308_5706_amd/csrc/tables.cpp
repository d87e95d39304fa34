// Host-side tables of the scale-discretized wavelets (Sec. 2.2, Eq. 7-16) and of
// Delta = d(pi/2), the Wigner small-d matrix at pi/2 (Sec. 3.2, Eq. 25).
#include <cmath>
#include <cstdlib>
#include <map>

#include "s2dw_internal.h"

namespace s2dw {

namespace {

typedef long double ld;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<ld> &x, std::vector<ld> &w) {
    x.assign(n, 0.0L);
    w.assign(n, 0.0L);
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        ld z = cosl(pi * (i + 0.75L) / (n + 0.5L));
        ld dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            ld dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-21L) break;
        }
        {
            ld p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}

// The integral of Eq. 13, written in the variable x of the bump s (Eq. 12):
// u = 1/lambda + (lambda - 1)/(2 lambda) (x + 1), so that s_lambda(u) = s(x) and
//   I(t) = int_t^1 s_lambda(u)^2 / u du = int_{x(t)}^1 exp(-2/(1-x^2)) / u(x) du/dx dx.
// Evaluated by composite Gauss-Legendre quadrature (64 panels on [-1, 1], 24 nodes
// each) in long double: the integrand is smooth and vanishes with all derivatives at
// the ends.
class KIntegral {
  public:
    explicit KIntegral(double lambda) : lam_(lambda) {
        gauss_legendre(kNodes, gx_, gw_);
        // cumulative integral from each panel edge to 1
        cum_.assign(kPanels + 1, 0.0L);
        for (int p = kPanels - 1; p >= 0; --p) cum_[p] = cum_[p + 1] + panel(edge(p), edge(p + 1));
    }
    // k_lambda(a) - k_lambda(b) for a <= b: the integral of Eq. 13 over [a, b], clipped to
    // [1/lambda, 1], by composite Gauss-Legendre quadrature over that interval alone (so
    // that tiny differences keep their relative precision).
    ld dk(ld a, ld b) const {
        if (a < 1.0L / lam_) a = 1.0L / lam_;
        if (b > 1.0L) b = 1.0L;
        if (!(b > a)) return 0.0L;
        ld xa = x_of(a), xb = x_of(b), acc = 0.0L;
        const int np = 32;
        for (int i = 0; i < np; ++i) acc += panel(xa + (xb - xa) * i / np, xa + (xb - xa) * (i + 1) / np);
        return acc / cum_[0];
    }
    // k_lambda(t) of Eq. 13.
    ld k(ld t) const {
        if (t <= 1.0L / lam_) return 1.0L;
        if (t >= 1.0L) return 0.0L;
        ld x = x_of(t);
        int p = (int)floorl((x + 1.0L) * 0.5L * kPanels);
        if (p < 0) p = 0;
        if (p > kPanels - 1) p = kPanels - 1;
        ld v = panel(x, edge(p + 1)) + cum_[p + 1];
        return v / cum_[0];
    }

  private:
    static constexpr int kPanels = 64;
    static constexpr int kNodes = 24;
    ld edge(int p) const { return -1.0L + 2.0L * (ld)p / kPanels; }
    ld x_of(ld t) const { return (t - 1.0L / lam_) * 2.0L * lam_ / (lam_ - 1.0L) - 1.0L; }
    ld f(ld x) const {
        if (x <= -1.0L || x >= 1.0L) return 0.0L;
        ld u = 1.0L / lam_ + (lam_ - 1.0L) / (2.0L * lam_) * (x + 1.0L);
        ld s = expl(-1.0L / (1.0L - x * x));
        return s * s / u * (lam_ - 1.0L) / (2.0L * lam_);
    }
    ld panel(ld a, ld b) const {
        ld h = 0.5L * (b - a), c = 0.5L * (b + a), acc = 0.0L;
        for (int i = 0; i < kNodes; ++i) acc += gw_[i] * f(c + h * gx_[i]);
        return acc * h;
    }
    ld lam_;
    std::vector<ld> gx_, gw_, cum_;
};

}  // namespace

int jmax_of(int L, double lambda) {
    // the lowest J with lambda^-J L <= 1
    int J = 0;
    long double p = 1.0L;
    while (p < (long double)L) {
        p *= (long double)lambda;
        ++J;
    }
    return J;
}

bool build_wavelet_tables(int L, int N, double lambda, int J_min, HostTables &t) {
    if (L < 2 || N < 1 || N > 2 * kMaxK || N > L || !(lambda > 1.0) || !std::isfinite(lambda)) return false;
    int JL = jmax_of(L, lambda);
    if (J_min < 0 || J_min > JL) return false;
    int J = JL - J_min;
    if (J + 1 > kMaxScales) return false;
    t.L = L;
    t.N = N;
    t.S = J + 1;
    t.eta_imag = (N - 1) % 2 != 0;
    t.nk.clear();
    for (int n = 0; n < N; ++n)
        if ((N + n) % 2 == 1) t.nk.push_back(n);
    t.K = (int)t.nk.size();
    KIntegral ki(lambda);
    const ld lam = lambda;
    t.kappa.assign((size_t)t.S * L, 0.0);
    t.lo.assign(t.S, L);
    t.hi.assign(t.S, -1);
    for (int j = 0; j < t.S; ++j) {
        ld lj = powl(lam, (ld)j);
        for (int l = 0; l < L; ++l) {
            // kappa^j(l) = kappa_lambda(lambda^j l / L),  kappa_lambda(x) = sqrt(k(x/lambda) - k(x)),
            // the difference taken as the integral over [x/lambda, x]
            ld x = lj * (ld)l / (ld)L;
            ld v = ki.dk(x / lam, x);
            double kv = v > 0.0L ? (double)sqrtl(v) : 0.0;
            t.kappa[(size_t)j * L + l] = kv;
            if (kv > 0.0) {
                if (l < t.lo[j]) t.lo[j] = l;
                t.hi[j] = l;
            }
        }
    }
    t.phi.assign(L, 0.0);
    ld lJ = powl(lam, (ld)J);
    for (int l = 0; l < L; ++l) {
        ld v = ki.k(lJ * (ld)l / (ld)L);
        t.phi[l] = v > 0.0L ? (double)sqrtl(v) : 0.0;
    }
    // |s_ln| of Eq. 11 for the nonnegative carried n
    t.sig.assign((size_t)L * t.K, 0.0);
    for (int l = 0; l < L; ++l) {
        int gam = l - ((((N + l) % 2) == 0) ? 1 : 0);
        if (gam > N - 1) gam = N - 1;
        for (int k = 0; k < t.K; ++k) {
            int n = t.nk[k];
            if (gam < 0 || n > gam || ((gam - n) % 2) != 0) continue;
            int c = (gam - n) / 2;
            // binomial(gam, c) / 2^gam
            ld b = 1.0L;
            for (int i = 1; i <= c; ++i) b = b * (ld)(gam - c + i) / (ld)i;
            t.sig[(size_t)l * t.K + k] = (double)sqrtl(b / powl(2.0L, (ld)gam));
        }
    }
    return true;
}

// Delta^l_{m'm} = d^l_{m'm}(pi/2) for m', m >= 0 obeys, from l to l+1 (the three-term
// recurrence of d^l at cos(beta) = 0), with S(l, x) = sqrt(l^2 - x^2):
//   Delta^{l+1} = -[(2l+1) m' m Delta^l + (l+1) S(l,m') S(l,m) Delta^{l-1}]
//                  / [l S(l+1,m') S(l+1,m)]
//              = -(u_l(m') p_l(m)) Delta^l - (v_l(m') q_l(m)) Delta^{l-1}
// with p_l(x) = x / S(l+1,x), q_l(x) = S(l,x) / S(l+1,x), u_l = (2l+1)/l p_l,
// v_l = (l+1)/l q_l (all zero where l+1 <= x, and u_0 = v_0 = 0).  The start value at
// l0 = max(m', m) is the corner of Wigner's explicit sum at pi/2:
//   Delta^{l0}_{l0, m} = (-1)^{l0-m} sqrt(C(2 l0, l0+m)) 2^-l0,
//   Delta^{l0}_{m', l0} = sqrt(C(2 l0, l0+m')) 2^-l0.
void build_delta_tables(int L, DeltaTables &d) {
    d.L = L;
    d.Lp = (L + 63) / 64 * 64;
    const int Lp = d.Lp;
    d.pq.assign((size_t)L * Lp * 2, 0.0);
    d.uv.assign((size_t)Lp * L * 2, 0.0);
    for (int l = 0; l < L; ++l) {
        ld l1 = (ld)(l + 1);
        for (int x = 0; x < L && x < l + 1; ++x) {
            ld s1 = sqrtl((l1 - x) * (l1 + x));
            ld s0 = (x <= l) ? sqrtl(((ld)l - x) * ((ld)l + x)) : 0.0L;
            ld p = (ld)x / s1, q = s0 / s1;
            d.pq[((size_t)l * Lp + x) * 2 + 0] = (double)p;
            d.pq[((size_t)l * Lp + x) * 2 + 1] = (double)q;
            if (l > 0) {
                d.uv[((size_t)x * L + l) * 2 + 0] = (double)((2.0L * l + 1.0L) / (ld)l * p);
                d.uv[((size_t)x * L + l) * 2 + 1] = (double)((l1) / (ld)l * q);
            }
        }
    }
    // rescaling factors g_l(x) (the q side) and h_l(x) (the v side), l = x .. L, in long
    // double; they stay within a few powers of L of 1
    std::vector<ld> gq((size_t)(L + 1) * L, 0.0L), hv((size_t)L * (L + 1), 0.0L);
    auto Sf = [](ld l, int x) { return sqrtl((l - x) * (l + x)); };
    for (int x = 0; x < L; ++x) {
        ld *gx = &gq[(size_t)x * (L + 1)], *hx = &hv[(size_t)x * (L + 1)];
        gx[x] = 1.0L;
        hx[x] = 1.0L;
        if (x + 1 <= L) gx[x + 1] = hx[x + 1] = 1.0L;
        for (int l = x + 1; l + 1 <= L; ++l) {
            const ld q = Sf((ld)l, x) / Sf((ld)l + 1, x);         // q_l(x), l > x
            const ld v = ((ld)l + 1) / (ld)l * q;                  // v_l(x), l >= 1
            gx[l + 1] = q * gx[l - 1];
            hx[l + 1] = v * hx[l - 1];
        }
    }
    d.pt.assign((size_t)L * Lp, 0.0);
    d.ut.assign((size_t)Lp * L, 0.0);
    d.g.assign((size_t)L * Lp, 0.0);
    d.h.assign((size_t)Lp * L, 0.0);
    for (int x = 0; x < L; ++x) {
        const ld *gx = &gq[(size_t)x * (L + 1)], *hx = &hv[(size_t)x * (L + 1)];
        for (int l = x; l < L; ++l) {
            const ld s1 = Sf((ld)l + 1, x);
            const ld p = (ld)x / s1;                                // p_l(x)
            d.pt[(size_t)l * Lp + x] = (double)(p * gx[l] / gx[l + 1]);
            if (l > 0) d.ut[(size_t)x * L + l] = (double)((2.0L * l + 1.0L) / (ld)l * p * hx[l] / hx[l + 1]);
            d.g[(size_t)l * Lp + x] = (double)gx[l];
            d.h[(size_t)x * L + l] = (double)hx[l];
        }
    }
    // corner values T(a, b) = sqrt(C(2a, a+b)) 2^-a for 0 <= b <= a < L, built from
    // T(a, a) = 2^-a downwards with T(a, b-1) = T(a, b) sqrt((a+b)/(a-b+1))
    d.seed.assign((size_t)Lp * Lp, 0.0);
    d.seedt.assign((size_t)Lp * Lp, 0.0);
    d.seedtm.assign((size_t)Lp * Lp, 0.0);
    d.seedte.assign((size_t)Lp * Lp, 0);
    std::vector<ld> T(L);
    for (int a = 0; a < L; ++a) {
        T[a] = ldexpl(1.0L, -a);
        for (int b = a; b > 0; --b) T[b - 1] = T[b] * sqrtl((ld)(a + b) / (ld)(a - b + 1));
        for (int b = 0; b <= a; ++b) {
            // row m' = a, column m = b <= a: (-1)^{a-b} T(a, b);  row m' = b, column m = a: T(a, b)
            const ld v1 = ((a - b) & 1) ? -T[b] : T[b];
            const ld v2 = T[b];
            const size_t i1 = (size_t)a * Lp + b, i2 = (size_t)b * Lp + a;
            d.seed[i1] = (double)v1;
            d.seed[i2] = (double)v2;
            // rescaled: c_{l0} = g_{l0}(m) h_{l0}(m') with l0 = a
            const ld t1 = v1 / (gq[(size_t)b * (L + 1) + a] * hv[(size_t)a * (L + 1) + a]);  // m' = a, m = b
            const ld t2 = v2 / (gq[(size_t)a * (L + 1) + a] * hv[(size_t)b * (L + 1) + a]);  // m' = b, m = a
            int e;
            d.seedtm[i1] = (double)frexpl(t1, &e);
            d.seedte[i1] = e;
            d.seedt[i1] = (double)t1;
            d.seedtm[i2] = (double)frexpl(t2, &e);
            d.seedte[i2] = e;
            d.seedt[i2] = (double)t2;
        }
    }
}

void build_delta_ncols(const DeltaTables &d, const std::vector<int> &nk, std::vector<double> &out) {
    const int L = d.L, Lp = d.Lp, K = (int)nk.size();
    out.assign((size_t)Lp * L * K, 0.0);
    for (int mp = 0; mp < L; ++mp) {
        for (int k = 0; k < K; ++k) {
            int n = nk[k];
            if (n >= L) continue;
            int l0 = mp > n ? mp : n;
            // these corners never underflow: |n| < 16, so C(2 l0, l0 + n) 4^-l0 ~ (pi l0)^-1/2
            double dm1 = 0.0, d0 = d.seed[(size_t)mp * Lp + n];
            for (int l = l0; l < L; ++l) {
                out[((size_t)mp * L + l) * K + k] = d0;
                if (l + 1 >= L) break;
                const double *uv = &d.uv[((size_t)mp * L + l) * 2];
                const double *pq = &d.pq[((size_t)l * Lp + n) * 2];
                double dn = -(uv[0] * pq[0]) * d0 - (uv[1] * pq[1]) * dm1;
                dm1 = d0;
                d0 = dn;
            }
        }
    }
}

}  // namespace s2dw
