"""Host checks of the roofline accounting in bench.py (no device work): the algorithmic work
per stage follows the stated formulas, and each stage is priced under its fixed roof (HBM
bytes for the separation-of-variables stages, FP64 FLOP for the Wigner stages)."""
import importlib.util
import math
import os

import numpy as np
import pytest

from oracle import tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_wigner_terms_brute_force(bench):
    # count (l, m, m', n) terms of the quarter m, m' >= 0 directly on a tiny case
    L, N, lam, J_min = 12, 3, 2.0, 0
    kappa = tables.kappa_table(L, lam, J_min)
    nl = [n for n in range(-(N - 1), N) if (N + n) % 2 == 1]
    brute = 0
    for j in range(kappa.shape[0]):
        for el in range(L):
            if kappa[j, el] > 0:
                for m in range(el + 1):
                    for mp in range(el + 1):
                        brute += sum(1 for n in nl if abs(n) <= el)
    assert bench.wigner_terms(kappa, N) == brute


def test_stage_units_formulas(bench):
    L, N, lam, J_min = 64, 4, 2.0, 1
    kappa = tables.kappa_table(L, lam, J_min)
    T = bench.wigner_terms(kappa, N)
    u = bench.stage_units(kappa, L, N, T)
    Ljs = [max(np.nonzero(kappa[j] > 0)[0]) + 1 for j in range(kappa.shape[0]) if np.any(kappa[j] > 0)]
    Tg, Nh = 2 * L - 1, N - N // 2
    dft = 5.0 * Tg * math.log2(Tg)
    by = dict(u["beta_adj"])
    assert by["hbm"] == sum(16 * N * Lj * L + 32 * Nh * Lj * Lj for Lj in Ljs)
    conv = [10.0 * (Tg + 2 * Lj - 2) * math.log2(Tg + 2 * Lj - 2) + 6.0 * (Tg + 2 * Lj - 2) for Lj in Ljs]
    assert by["alu"] == pytest.approx(sum(N * Lj * (dft + c) for Lj, c in zip(Ljs, conv)))
    two = [Lj for Lj in Ljs if Nh * (2 * Lj - 1) > 9 * (2 * N - 1)]
    one = [Lj for Lj in Ljs if Nh * (2 * Lj - 1) <= 9 * (2 * N - 1)]
    assert two and one
    assert dict(u["gamma_fwd"]) == {"hbm": float(len(two) * (16 * Nh * L * Tg + 8 * (2 * N - 1) * L * Tg))}
    assert dict(u["alpha_fwd"])["alu"] == pytest.approx(len(two) * Nh * L * dft)
    assert dict(u["alpha_gamma_fwd"]) == {"hbm": float(sum(16 * N * Lj * L + 8 * (2 * N - 1) * L * Tg
                                                             for Lj in one))}
    assert dict(u["gamma_alpha_adj"]) == {"hbm": float(sum(8 * (2 * N - 1) * L * Tg + 16 * N * Lj * L
                                                             for Lj in one))}
    assert dict(u["alpha_adj"])["alu"] == pytest.approx(len(two) * Nh * L * dft)
    # without the fused passes every scale has an alpha and a gamma pass
    u2 = bench.stage_units(kappa, L, N, T, fused=False, fused_adj=False)
    assert "alpha_gamma_fwd" not in u2 and "gamma_alpha_adj" not in u2
    u3 = bench.stage_units(kappa, L, N, T, fused_adj=False)  # mixed precision: the analysis pass only
    assert u3["alpha_gamma_fwd"] == u["alpha_gamma_fwd"] and "gamma_alpha_adj" not in u3
    assert dict(u3["gamma_adj"]) == dict(u2["gamma_adj"])
    assert dict(u2["gamma_fwd"]) == {"hbm": float(len(Ljs) * (16 * Nh * L * Tg + 8 * (2 * N - 1) * L * Tg))}
    assert u["wigner_fwd"] == [("alu", 5.0 * T)]


def test_stage_units_prime_factor_lengths(bench):
    # T = 2047, N = 8: the analysis scales with the blocked alpha transforms keep the two-pass
    # form, the others take the fused kernel; the FP64 synthesis (four orders) keeps the
    # two-pass form, the mixed one is fused.  T = 4095, N = 4: every scale fused both ways
    L, N, lam, J_min = 1024, 8, 2.0, 1
    assert bench.pfa_fused(L, N) and bench.pfa_fused(2048, 4)
    assert not bench.pfa_fused(1024, 10) and not bench.pfa_fused(2048, 8) and not bench.pfa_fused(512, 4)
    kappa = tables.kappa_table(L, lam, J_min)
    T = bench.wigner_terms(kappa, N)
    Ljs = [max(np.nonzero(kappa[j] > 0)[0]) + 1 for j in range(kappa.shape[0]) if np.any(kappa[j] > 0)]
    Tg, G, Nh = 2 * L - 1, 2 * N - 1, N - N // 2
    blk = [Lj for Lj in Ljs if bench.blocked_alpha(L, Lj)]
    assert blk and all(Lj < 256 for Lj in blk) and not bench.blocked_alpha(L, 1024)
    direct = [Lj for Lj in Ljs if bench.direct_alpha_gamma(N, Lj)]
    u = bench.stage_units(kappa, L, N, T)
    fw = [Lj for Lj in Ljs if Lj not in blk or Lj in direct]
    assert dict(u["alpha_gamma_fwd"])["hbm"] == float(sum(16 * N * Lj * L + 8 * G * L * Tg for Lj in fw))
    two = [Lj for Lj in Ljs if Lj not in fw]
    assert two and dict(u["gamma_fwd"])["hbm"] == float(len(two) * (16 * Nh * L * Tg + 8 * G * L * Tg))
    npf = sum(1 for Lj in fw if Lj not in direct)
    assert dict(u["alpha_gamma_fwd"])["alu"] == pytest.approx(npf * Nh * L * 5.0 * Tg * math.log2(Tg))
    assert dict(u["gamma_alpha_adj"])["hbm"] == float(sum(8 * G * L * Tg + 16 * N * Lj * L for Lj in direct))
    u3 = bench.stage_units(kappa, L, N, T, fused_adj=False, mixed=True)
    assert dict(u3["gamma_alpha_adj"])["hbm"] == float(sum(8 * G * L * Tg + 16 * N * Lj * L for Lj in Ljs))
    assert "gamma_adj" not in u3 and "alpha_adj" not in u3
    L2, N2 = 2048, 4
    kappa2 = tables.kappa_table(L2, lam, 4)
    u4 = bench.stage_units(kappa2, L2, N2, bench.wigner_terms(kappa2, N2))
    for st in ("alpha_fwd", "gamma_fwd", "alpha_adj", "gamma_adj"):
        assert st not in u4


def test_roofline_roof_is_fixed_per_stage(bench):
    # separation-of-variables stages are priced by HBM bytes whatever their FLOP count, with the
    # FFT-FLOP figure as a secondary field; the Wigner stages by their algorithmic FLOP
    ps = {"ms_per_launch": 1.0, "launches_per_step": 2.0}
    for units in ({"beta_adj": [("hbm", 8e9), ("alu", 1e10)]}, {"beta_adj": [("hbm", 8e8), ("alu", 1e11)]}):
        r = bench.roofline("beta_adj", ps, units)
        by, fl = dict(units["beta_adj"])["hbm"] / 2, dict(units["beta_adj"])["alu"] / 2
        assert r["bound"] == "hbm" and r["unit"] == "GB/s"
        assert r["achieved"] == pytest.approx(by / 1e-3 / 1e9) and r["frac"] == pytest.approx(by / 1e-3 / 1e9 / 8000.0)
        assert r["algorithmic_per_launch"] == pytest.approx(by)
        assert r["flop_model"]["frac"] == pytest.approx(fl / 1e-3 / 1e12 / bench.PEAK_FP64_TFLOPS)
    r = bench.roofline("gamma_fwd", ps, {"gamma_fwd": [("hbm", 4e9)]})
    assert r["bound"] == "hbm" and "flop_model" not in r and r["achieved"] == pytest.approx(2000.0)
    r = bench.roofline("wigner_adj", ps, {"wigner_adj": [("alu", 1e11)]})
    assert r["bound"] == "alu" and r["frac"] == pytest.approx(50.0 / bench.PEAK_FP64_TFLOPS)


def test_step_stats(bench):
    s = bench.step_stats([1.0, 3.0, 2.0, 10.0])
    assert s["median_ms"] == 2.5 and s["mean_ms"] == 4.0 and s["min_ms"] == 1.0 and s["max_ms"] == 10.0
    assert s["std_ms"] == pytest.approx(np.std([1.0, 3.0, 2.0, 10.0])) and s["steps"] == 4


def test_profile_kernel_names_map_to_stages():
    from paper_1308_5706_amd import profiling
    cases = {
        "void s2dw::gamma_fwd_kernel<HIP_vector_type<double, 2u>, 2>(s2dw::GammaArgs)": "gamma_fwd",
        "void s2dw::alpha_gamma_fwd_kernel<true, 4>(s2dw::AlphaGammaArgs)": "alpha_gamma_fwd",
        "void s2dw::gamma_alpha_adj_kernel<4>(s2dw::GammaAlphaArgs)": "gamma_alpha_adj",
        "void s2dw::gamma_adj_kernel<HIP_vector_type<double, 2u>, 2>(s2dw::GammaArgs)": "gamma_adj",
        "void s2dw::alpha_adj_blk_kernel<HIP_vector_type<double, 2u>, 512>(s2dw::StageArgs)": "alpha_adj",
        "void s2dw::beta_adj_multi_kernel<HIP_vector_type<double, 2u>, 4096>(s2dw::StageArgs, s2dw::": "beta_adj",
        "void s2dw::wig_adj_kernel<2, 2, double>(s2dw::WigAdjArgs)": "wigner_adj",
        "__amd_rocclr_copyBuffer": None,
    }
    for name, stage in cases.items():
        assert profiling.stage_of(name) == stage, name
