// Host check of the Wigner-stage recurrence tables (tables.cpp): the rescaled recurrence
//   D_{l+1} = -(ut_l(m') pt_l(m)) D_l - D_{l-1},  Delta^l_{m'm} = g_l(m) h_l(m') D_l,
// reproduces Delta^l_{m'm} = d^l_{m'm}(pi/2) as the three-term recurrence in l defines it.
// Reference: the recurrence evaluated in long double with its coefficients computed in long
// double from their definitions (sqrt((l+1)^2 - x^2) etc.) and the exact start values.
// Prints one line "plain <err> orig_plain <err> xn <err> orig_xn <err>": the max relative
// errors where |Delta| > 1e-4 of the rescaled recurrence and of the unscaled one on the same
// double tables, for pairs with a normal start value (plain, run in double) and for the
// extended-exponent ones (xn, run in long double from the mantissa / exponent start).
#include "s2dw_internal.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>

using namespace s2dw;
typedef long double ld;

int main(int argc, char **argv) {
    const int L = argc > 1 ? atoi(argv[1]) : 64;
    const int step = argc > 2 ? atoi(argv[2]) : 1;
    DeltaTables d;
    build_delta_tables(L, d);
    const int Lp = d.Lp;
    auto S = [](ld l, int x) { return sqrtl((l - x) * (l + x)); };
    ld worst_plain = 0, worst_xn = 0, worst_orig_xn = 0, worst_orig_plain = 0;
    for (int mp = 0; mp < L; mp += step)
        for (int m = 0; m < L; m += step) {
            const size_t i = (size_t)mp * Lp + m;
            const int l0 = mp > m ? mp : m, lo = mp < m ? mp : m;
            ld T = ldexpl(1.0L, -l0);  // |Delta^{l0}| = sqrt(C(2 l0, l0 + lo)) 2^-l0
            for (int b = l0; b > lo; --b) T = T * sqrtl((ld)(l0 + b) / (ld)(l0 - b + 1));
            const ld start = (mp == l0 && ((l0 - lo) & 1)) ? -T : T;
            const bool xn = d.seedte[i] < -1000;
            // reference t; rescaled r (long double, XN) and q (double, plain); unscaled o (long
            // double, XN) and z (double, plain)
            ld t0 = 0, t1 = start, o0 = 0, o1 = start;
            ld r0 = 0, r1 = xn ? ldexpl((ld)d.seedtm[i], d.seedte[i]) : (ld)d.seedt[i];
            double q0 = 0, q1 = d.seedt[i], z0 = 0, z1 = d.seed[i];
            for (int l = l0; l < L; ++l) {
                const ld c = (ld)d.g[(size_t)l * Lp + m] * (ld)d.h[(size_t)mp * L + l];
                if (fabsl(t1) > 1e-4L) {
                    if (xn) {
                        const ld er = fabsl(c * r1 - t1) / fabsl(t1), eo = fabsl(o1 - t1) / fabsl(t1);
                        if (er > worst_xn) worst_xn = er;
                        if (eo > worst_orig_xn) worst_orig_xn = eo;
                    } else {
                        const ld e = fabsl(c * (ld)q1 - t1) / fabsl(t1);
                        if (e > worst_plain) worst_plain = e;
                        const ld ez = fabsl((ld)z1 - t1) / fabsl(t1);
                        if (ez > worst_orig_plain) worst_orig_plain = ez;
                    }
                }
                if (l + 1 >= L) break;
                const ld p = (ld)m / S(l + 1, m), q = S(l, m) / S(l + 1, m);
                const ld pu = (ld)mp / S(l + 1, mp), qv = S(l, mp) / S(l + 1, mp);
                const ld u = (2.0L * l + 1) / l * pu, v = (ld)(l + 1) / l * qv;
                const ld tn = l == 0 ? 0.0L : -(u * p) * t1 - (v * q) * t0;
                const double *uv = &d.uv[((size_t)mp * L + l) * 2];
                const double *pq = &d.pq[((size_t)l * Lp + m) * 2];
                const ld on = -((ld)uv[0] * pq[0]) * o1 - ((ld)uv[1] * pq[1]) * o0;
                const double a = d.ut[(size_t)mp * L + l] * d.pt[(size_t)l * Lp + m];
                const ld rn = -(ld)a * r1 - r0;
                const double qn = -a * q1 - q0;
                const double zn = -(uv[0] * pq[0]) * z1 - (uv[1] * pq[1]) * z0;
                t0 = t1, t1 = tn, o0 = o1, o1 = on, r0 = r1, r1 = rn, q0 = q1, q1 = qn, z0 = z1, z1 = zn;
            }
        }
    printf("plain %.3Le orig_plain %.3Le xn %.3Le orig_xn %.3Le\n", worst_plain, worst_orig_plain, worst_xn, worst_orig_xn);
    return 0;
}
