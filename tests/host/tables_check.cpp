// Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the library's host
// tables (tables.cpp): builds the wavelet and Delta tables over a spread of parameters,
// including the edges of the argument ranges and parameter sets that are refused, and checks
// a few invariants on the way.  Exit status 0 and no sanitizer report is a pass.
#include "s2dw_internal.h"

#include <cmath>
#include <cstdio>

using namespace s2dw;

int main() {
    int fails = 0;
    const int Ls[] = {2, 3, 7, 16, 33, 64, 130};
    const int Ns[] = {1, 2, 3, 4, 8, 15, 16};
    const double lams[] = {1.5, 2.0, 3.0};
    for (int L : Ls)
        for (int N : Ns)
            for (double lam : lams) {
                const int JL = jmax_of(L, lam);
                for (int J_min = -1; J_min <= JL + 1; ++J_min) {
                    HostTables t;
                    const bool ok = build_wavelet_tables(L, N, lam, J_min, t);
                    const bool valid = N <= L && J_min >= 0 && J_min <= JL;
                    if (ok != valid) {
                        std::printf("accepted/refused wrongly: L=%d N=%d lam=%g J_min=%d\n", L, N, lam, J_min);
                        ++fails;
                    }
                    if (!ok) continue;
                    if ((int)t.kappa.size() != t.S * L || (int)t.phi.size() != L || (int)t.sig.size() != L * t.K) {
                        std::printf("table sizes: L=%d N=%d\n", L, N);
                        ++fails;
                    }
                    for (double v : t.kappa)
                        if (!std::isfinite(v) || v < 0.0) ++fails;
                }
            }
    // refused parameters
    HostTables t;
    if (build_wavelet_tables(1, 1, 2.0, 0, t) || build_wavelet_tables(8, 0, 2.0, 0, t) ||
        build_wavelet_tables(8, 2, 1.0, 0, t) || build_wavelet_tables(8, 2, NAN, 0, t) ||
        build_wavelet_tables(8, 2, INFINITY, 0, t) || build_wavelet_tables(64, 17, 2.0, 0, t))
        ++fails;
    for (int L : {2, 5, 64, 65, 300}) {
        DeltaTables d;
        build_delta_tables(L, d);
        std::vector<double> cols;
        build_delta_ncols(d, {0, 1, 3}, cols);
        if ((int)cols.size() != d.Lp * L * 3) ++fails;
        for (double v : cols)
            if (!std::isfinite(v)) ++fails;
    }
    std::printf("tables_check: %d failures\n", fails);
    return fails == 0 ? 0 : 1;
}
