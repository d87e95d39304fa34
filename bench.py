"""Benchmark: SO(3) wavelet coefficients per second, analysis + synthesis, on one MI355X.

A step is one round trip of one map through the whole hot path: wavelet analysis
(Wigner stage + beta/gamma/alpha stages) with the scaling coefficients, then the exact
synthesis back to f_lm.  Workload (the metric's configuration): L = 1024, N = 8,
lambda = 2, J_min = 1 (10 scales, full-resolution grid 15 x 1024 x 2047 per scale),
f_lm synthetic (seeded complex Gaussian, C_l = 1/(l+1)^2, real-signal symmetry),
resident in HBM before the timed region.

Prints one JSON line.  The roofline entry covers the kernel that takes the most time,
timed live with HIP events on the stream the library launches on; cpu_baseline times
the CPU reference on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector peak: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E


def n_list(N):
    return [n for n in range(-(N - 1), N) if (N + n) % 2 == 1]


def wigner_terms(kappa, N):
    """Terms of the l-sum (or the m'-contraction) over the m >= 0, m' >= 0 quarter:
    sum_j sum_{l: kappa^j(l) > 0} (l+1)^2 #{n carried with |n| <= l}."""
    nl = n_list(N)
    T = 0
    S, L = kappa.shape
    for j in range(S):
        for el in range(L):
            if kappa[j, el] > 0.0:
                T += (el + 1) ** 2 * sum(1 for n in nl if abs(n) <= el)
    return T


def cpu_baseline(L, N, lam, J_min, budget_rows=None, budget_cols=None):
    """The CPU reference timed on a bounded sample of the workload, scaled to coefficients/s.
    Sample: analysis of `budget_rows` of the L beta rows (all scales, alpha, gamma);
    synthesis alpha/gamma rules on `budget_rows` rows and the beta/Wigner step on
    `budget_cols` of the 2L-1 m columns.  Each part's cost is linear in its rows/columns."""
    import numpy as np
    import oracle
    from oracle import tables
    from paper_1308_5706_amd.inputs import random_flm, random_wavelet_samples
    threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    budget_rows = budget_rows or threads
    budget_cols = budget_cols or max(2, threads // 4)
    f = random_flm(L, 0)
    psi = tables.wavelets(L, N, lam, J_min)
    S = psi.shape[0]
    betas = oracle.mw_betas(L)
    t0 = time.perf_counter()
    oracle.analysis(f, L, N, lam, J_min, betas=betas[:budget_rows], psi=psi)
    t_an = (time.perf_counter() - t0) * L / budget_rows
    Ws = random_wavelet_samples(S, 2 * N - 1, budget_rows, 2 * L - 1, 1)
    t0 = time.perf_counter()
    oracle.alpha_gamma_rules_mw(Ws, L, N)
    t_rules = (time.perf_counter() - t0) * L / budget_rows
    Gt = np.zeros((S, len(n_list(N)), L, 2 * L - 1), dtype=np.complex128)
    t0 = time.perf_counter()
    oracle.beta_wigner_mw(Gt, L, N, (0, budget_cols - 1))
    t_beta = (time.perf_counter() - t0) * (2 * L - 1) / budget_cols
    coeffs = S * (2 * N - 1) * L * (2 * L - 1)
    total = t_an + t_rules + t_beta
    return {"value": coeffs / total, "unit": "SO(3) coeffs/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"analysis of {budget_rows}/{L} beta rows; synthesis alpha/gamma rules on {budget_rows}/{L} "
                       f"rows and beta/Wigner step on {budget_cols}/{2 * L - 1} m columns; each scaled linearly "
                       f"to the full map (estimated round trip {total:.1f} s)")}


def direct_alpha_gamma(N, Lj):
    """Whether a scale takes the fused alpha and gamma passes (real signals on the
    equiangular grid; the library's rule: Nh (2Lj - 1) complex multiply-adds per sample at
    most 9 G and 256, G = 2N - 1 the W values written or read per sample)."""
    Nh = N - N // 2
    return Nh * (2 * Lj - 1) <= min(9 * (2 * N - 1), 256) and 2 * Nh * Lj <= 1024


def pfa_fused(L, N):
    """Whether the fused prime-factor alpha and gamma kernels serve a real-signal transform
    at band-limit L (T = 2L - 1 of 2047 or 4095, at most 16 complex values per thread waiting
    in registers: the library's rule)."""
    Nh, T = N - N // 2, 2 * L - 1
    return (T == 2047 and Nh <= 4) or (T == 4095 and Nh <= 2)


def blocked_alpha(L, Lj):
    """Whether the library takes the blocked alpha transforms for a scale of band-limit Lj
    (its cost model: nblk convolutions of size Q in {512, 1024, 2048} against one of size
    PB >= T + 2Lj - 2, taken when they cost under 0.7 of it)."""
    T = 2 * L - 1
    cost = lambda q: q * math.log2(q)
    PB = 1 << math.ceil(math.log2(2 * Lj + T - 2))
    best, blk = 0.7 * cost(PB), False
    for Q in (512, 1024, 2048):
        B = Q - 2 * Lj + 2
        if B < 64:
            continue
        nbk = -(-T // B)
        if nbk >= 2 and nbk * cost(Q) < best:
            best, blk = nbk * cost(Q), True
    return blk


def fused_scales(L, N, Ljs, mixed=False):
    """The scales (by band-limit) that take the fused prime-factor kernels by the library's
    default rule: (analysis, synthesis)."""
    if not pfa_fused(L, N):
        return [], []
    T, Nh = 2 * L - 1, N - N // 2
    fwd = [Lj for Lj in Ljs if T == 4095 or not blocked_alpha(L, Lj)]
    adj = list(Ljs) if (T == 4095 or mixed or Nh <= 2) else []
    return fwd, adj


def stage_units(kappa, L, N, T, fused=True, fused_adj=True, pfa=None, mixed=False):
    """Algorithmic work of each stage per step (one map), summed over the scales.

    Wigner stages (one launch per direction): 5 FLOP per term of the l-sum / m'-contraction
    over the m >= 0, m' >= 0 quarter (1 multiply for Delta Delta, 2 FMA for the complex
    product).  Bluestein and gamma stages (one launch per scale j, the coarse scales of the
    synthesis beta stage in one shared launch): bytes of the arrays the stage must read and
    write per scale, T = 2L - 1, G = 2N - 1, Nh = ceil(N/2), Lj = band-limit:
      beta_fwd  U quarter 16 N Lj^2 in,      Ub 16 N Lj L out
      alpha_fwd Ub 16 N Lj L in,             Y 16 Nh L T out
      gamma_fwd Y 16 Nh L T in,              W 8 G L T out
      gamma_adj W 8 G L T in,                X 16 Nh L T out
      alpha_adj X 16 Nh L T in,              G 16 N Lj L out
      beta_adj  G 16 N Lj L in,              V 32 Nh Lj^2 out
      alpha_gamma_fwd (coarse scales of the analysis, fused = True; they leave
                alpha_fwd and gamma_fwd)  Ub 16 N Lj L in,  W 8 G L T out
      gamma_alpha_adj (the same scales of an FP64 synthesis, fused_adj = True; they leave
                gamma_adj and alpha_adj)  W 8 G L T in,  G 16 N Lj L out
    With pfa (default: pfa_fused(L, N)) the scales that fused_scales names take the fused
    prime-factor kernels, also counted as alpha_gamma_fwd and gamma_alpha_adj, with the same
    bytes and, as FLOP, the alpha DFTs of its rings.
    and, for the four Fourier stages, FLOP with a length-n complex DFT counted as an FFT,
    5 n log2 n, whatever way it is computed:
      beta_fwd  N Lj columns, one length-T DFT each
      alpha_fwd Nh L rings, one length-T DFT each
      alpha_adj Nh L rings, one length-T DFT each
      beta_adj  N Lj columns, one length-T DFT and the quadrature-weight convolution (2Lj - 1
                outputs from T inputs: a linear convolution of length M = T + 2Lj - 2 by two
                FFTs and a pointwise product, 10 M log2 M + 6 M)
    Each entry is a list of (bound, work) pairs.
    """
    S = kappa.shape[0]
    Tg, G, Nh = 2 * L - 1, 2 * N - 1, N - N // 2
    Ljs = []
    for j in range(S):
        nz = [l for l in range(L) if kappa[j, l] > 0.0]
        if nz:
            Ljs.append(max(nz) + 1)
    if pfa is None:
        pfa = pfa_fused(L, N)
    fw, ad = fused_scales(L, N, Ljs, mixed) if pfa else ([], [])
    direct = [Lj for Lj in Ljs if fused and direct_alpha_gamma(N, Lj)]
    direct_adj = [Lj for Lj in Ljs if fused_adj and direct_alpha_gamma(N, Lj)]
    pf = [Lj for Lj in Ljs if Lj in fw and Lj not in direct]
    pf_adj = [Lj for Lj in Ljs if Lj in ad and Lj not in direct_adj]
    one, one_adj = direct + pf, direct_adj + pf_adj
    two = [Lj for Lj in Ljs if Lj not in one]
    two_adj = [Lj for Lj in Ljs if Lj not in one_adj]
    per = {
        "beta_fwd": [16 * N * Lj * Lj + 16 * N * Lj * L for Lj in Ljs],
        "alpha_fwd": [16 * N * Lj * L + 16 * Nh * L * Tg for Lj in two],
        "gamma_fwd": [16 * Nh * L * Tg + 8 * G * L * Tg for Lj in two],
        "alpha_gamma_fwd": [16 * N * Lj * L + 8 * G * L * Tg for Lj in one],
        "gamma_adj": [8 * G * L * Tg + 16 * Nh * L * Tg for Lj in two_adj],
        "alpha_adj": [16 * Nh * L * Tg + 16 * N * Lj * L for Lj in two_adj],
        "gamma_alpha_adj": [8 * G * L * Tg + 16 * N * Lj * L for Lj in one_adj],
        "beta_adj": [16 * N * Lj * L + 32 * Nh * Lj * Lj for Lj in Ljs],
    }
    dft = 5.0 * Tg * math.log2(Tg)

    def conv(Lj):
        M = Tg + 2 * Lj - 2
        return 10.0 * M * math.log2(M) + 6.0 * M

    flops = {
        "beta_fwd": sum(N * Lj * dft for Lj in Ljs),
        "alpha_fwd": len(two) * Nh * L * dft,
        "alpha_adj": len(two_adj) * Nh * L * dft,
        "alpha_gamma_fwd": len(pf) * Nh * L * dft,
        "gamma_alpha_adj": len(pf_adj) * Nh * L * dft,
        "beta_adj": sum(N * Lj * (dft + conv(Lj)) for Lj in Ljs),
    }
    units = {k: [("hbm", float(sum(v)))] for k, v in per.items() if v}
    for k, v in flops.items():
        if k in units and v > 0:
            units[k].append(("alu", float(v)))
    units["wigner_fwd"] = [("alu", 5.0 * T)]
    units["wigner_adj"] = [("alu", 5.0 * T)]
    return units


def roofline(stage, ps, units):
    """Achieved rate of a stage: its algorithmic work per step (all scales; several scales
    may share a launch) over its device time per step, i.e. the work of an average launch
    over the average launch duration.  The roof is fixed per stage: the Wigner stages
    (Delta recursion + l-sum or m'-contraction) are FP64 vector arithmetic, priced by the
    algorithmic FLOP of their terms; every separation-of-variables stage (the beta, alpha
    and gamma sums of both directions) is priced by the HBM bytes it must move.  For the
    four Fourier stages the FFT-FLOP count (5 n log2 n per length-n DFT) is added as a
    secondary figure, ``flop_model``."""
    per_launch_s = ps["ms_per_launch"] * 1e-3
    entries = dict(units.get(stage, [("hbm", 0.0)]))
    primary = "alu" if stage.startswith("wigner") else "hbm"
    work = entries.get(primary, 0.0) / ps["launches_per_step"]
    if primary == "alu":
        r = {"bound": "alu", "achieved": work / per_launch_s / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
    else:
        r = {"bound": "hbm", "achieved": work / per_launch_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["algorithmic_per_launch"] = work
    r["traffic"] = None
    r["kernel"] = stage
    r["launch_ms"] = ps["ms_per_launch"]
    r["launches_per_step"] = ps["launches_per_step"]
    if primary == "hbm" and "alu" in entries:
        fl = entries["alu"] / ps["launches_per_step"]
        r["flop_model"] = {"what": "FFT-FLOP, 5 n log2 n per length-n DFT", "achieved": fl / per_launch_s / 1e12,
                           "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                           "frac": fl / per_launch_s / 1e12 / PEAK_FP64_TFLOPS}
    return r


def step_stats(ms):
    """Median, mean, standard deviation, minimum and maximum of per-step device times."""
    import numpy as np
    a = np.asarray(ms, dtype=np.float64)
    return {"median_ms": float(np.median(a)), "mean_ms": float(a.mean()), "std_ms": float(a.std()),
            "min_ms": float(a.min()), "max_ms": float(a.max()), "steps": int(a.size)}


def batched_leg(maps=256, replays=5, oracle_maps=4):
    """The batched mixed-precision form (many maps of mixed (L, N) in one HIP graph, and the
    same maps through the persistent executor): throughput against the plain FP64 path, each
    map's error against the FP64 GPU result, and the checker: sampled maps (L <= 128) of both
    forms against the FP64 CPU oracle."""
    import numpy as np
    import oracle
    from paper_1308_5706_amd import batch
    out, data = batch.run(maps, replays)
    errs, perrs = [], []
    for (L, N), (idx, F, W, fr, PW) in sorted(data.items()):
        if L > 128:
            continue
        for k in range(min(F.shape[0], oracle_maps - len(errs))):
            ref = oracle.analysis(F[k].cpu().numpy(), L, N, 2.0, 1)
            for got, lst in ((W[k], errs), (PW[k], perrs)):
                g = got.double().cpu().numpy()
                lst.append(max(float(np.max(np.abs(g[j] - ref[j])) / np.max(np.abs(ref[j])))
                               for j in range(ref.shape[0])))
        if len(errs) >= oracle_maps:
            break
    out["oracle_maps"] = len(errs)
    out["max_rel_err_W_vs_oracle"] = max(errs) if errs else None
    out["persistent"]["max_rel_err_W_vs_oracle"] = max(perrs) if perrs else None
    del data
    return out


def oracle_config1():
    """The CPU oracle timed end to end (analysis with scaling, then synthesis) on the
    medium configuration L = 256, N = 8, lambda = 2, J_min = 2, on every host core it uses."""
    import numpy as np
    import oracle
    from oracle import tables
    from paper_1308_5706_amd.inputs import random_flm
    L, N, lam, J_min = 256, 8, 2.0, 2
    f = random_flm(L, 0)
    psi = tables.wavelets(L, N, lam, J_min)
    phi = tables.phi_table(L, lam, J_min)
    t0 = time.perf_counter()
    W = oracle.analysis(f, L, N, lam, J_min, psi=psi)
    wp = oracle.scaling(f, L, lam, J_min, phi=phi)
    t1 = time.perf_counter()
    fr = oracle.synthesis(W, wp, L, N, lam, J_min, psi=psi, phi=phi)
    t2 = time.perf_counter()
    coeffs = W.size
    return {"workload": f"L={L}, N={N}, lambda={lam}, J_min={J_min}, one map, round trip", "seconds": t2 - t0,
            "analysis_s": t1 - t0, "synthesis_s": t2 - t1, "coeffs_per_s": coeffs / (t2 - t0),
            "cores": int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1)),
            "round_trip_rel_err": float(np.max(np.abs(fr - f)) / np.max(np.abs(f)))}


def gpu_config1(s2dw, torch, steps=20):
    """The GPU round trip on the same medium configuration, for comparison with the oracle."""
    from paper_1308_5706_amd.inputs import random_flm
    L, N, lam, J_min = 256, 8, 2.0, 2
    f = torch.as_tensor(random_flm(L, 0)).to("cuda")
    for _ in range(3):
        W, Wp = s2dw.analysis(f, L, N, lam, J_min)
        fr = s2dw.synthesis(W, Wp, L, N, lam, J_min)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        W, Wp = s2dw.analysis(f, L, N, lam, J_min, out=W)
        s2dw.synthesis(W, Wp, L, N, lam, J_min, out=fr)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"ms_per_round_trip": ms, "coeffs_per_s": W.numel() / (ms * 1e-3),
            "round_trip_rel_err": float((fr - f).abs().max().item() / f.abs().max().item())}


def extra_legs(args, s2dw, torch, dev, f, W, fr, L, N, lam, J_min, S, prec):
    """Features measured beside the headline round trip (outside its timed region): steering,
    the multiresolution layout, the Driscoll-Healy grid and a complex signal."""
    # steering (Eq. 10) of the step's W to Q off-grid angles: a post-step outside the timed
    # round trip, one launch per call; bytes = W read (S G L T) + steered planes written (S Q L T)
    Q, reps = 8, 10
    gam = torch.linspace(0.1, 6.0, Q, dtype=torch.float64, device=dev)
    Wq = torch.empty((S, Q, L, 2 * L - 1), dtype=W.dtype, device=dev)
    s2dw.steer(W, gam, L, N, lam, J_min, out=Wq)
    torch.cuda.synchronize()
    s2dw.profile(True)
    for _ in range(reps):
        s2dw.steer(W, gam, L, N, lam, J_min, out=Wq)
    sq = s2dw.profile_read()["steer"]
    s2dw.profile(False)
    del Wq
    steer_ms = sq[0] / sq[1]
    steer_bytes = S * (2 * N - 1 + Q) * L * (2 * L - 1) * W.element_size()
    steer = {"angles": Q, "ms_per_launch": steer_ms,
             "roofline": {"bound": "hbm", "achieved": steer_bytes / (steer_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                          "unit": "GB/s", "algorithmic_per_launch": steer_bytes}}
    steer["roofline"]["frac"] = steer["roofline"]["achieved"] / PEAK_HBM_GBS

    # the same round trip in the multiresolution layout (each scale on the grid of its own
    # band-limit): exact as well, with fewer samples; reported beside the full-grid figure
    Wm = torch.empty(s2dw._w_shape(L, N, lam, J_min, "multires"), dtype=W.dtype, device=dev)
    frm = torch.empty_like(fr)

    def step_mr():
        _, Wp = s2dw.analysis(f, L, N, lam, J_min, out=Wm, precision=prec, grid="multires")
        s2dw.synthesis(Wm, Wp, L, N, lam, J_min, out=frm, precision=prec, grid="multires")

    for _ in range(max(1, args.warmup)):
        step_mr()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_mr()
    torch.cuda.synchronize()
    ms_mr = (time.perf_counter() - t0) * 1e3 / args.steps
    multires = {"ms_per_step": ms_mr, "samples_per_map": Wm.numel(),
                "round_trip_rel_err": float((frm - f).abs().max().item() / f.abs().max().item())}
    del Wm
    print(f"# multires round trip {ms_mr:.3f} ms/step", file=sys.stderr, flush=True)

    # and on the paper's own Driscoll-Healy grid (2L colatitudes, N base orientations)
    W = None
    torch.cuda.empty_cache()
    Wd = torch.empty(s2dw._w_shape(L, N, lam, J_min, "dh"), dtype=torch.float64 if prec == "fp64" else torch.float32,
                     device=dev)

    def step_dh():
        _, Wp = s2dw.analysis(f, L, N, lam, J_min, out=Wd, precision=prec, grid="dh")
        s2dw.synthesis(Wd, Wp, L, N, lam, J_min, out=frm, precision=prec, grid="dh")

    for _ in range(max(1, args.warmup)):
        step_dh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_dh()
    torch.cuda.synchronize()
    ms_dh = (time.perf_counter() - t0) * 1e3 / args.steps
    dh_grid = {"ms_per_step": ms_dh, "samples_per_map": Wd.numel(),
               "coeffs_per_s": Wd.numel() / (ms_dh * 1e-3),
               "round_trip_rel_err": float((frm - f).abs().max().item() / f.abs().max().item())}
    del Wd
    print(f"# Driscoll-Healy round trip {ms_dh:.3f} ms/step", file=sys.stderr, flush=True)

    # a complex (non-real) signal on the equiangular grid: complex W, two real maps' work
    from paper_1308_5706_amd.inputs import random_flm_complex
    fc = torch.as_tensor(random_flm_complex(L, 0)).to(dev)
    Wc = torch.empty((S, 2 * N - 1, L, 2 * L - 1), dtype=torch.complex128 if prec == "fp64" else torch.complex64,
                     device=dev)

    def step_cx():
        _, Wp = s2dw.analysis(fc, L, N, lam, J_min, out=Wc, precision=prec, reality=False)
        s2dw.synthesis(Wc, Wp, L, N, lam, J_min, out=frm, precision=prec, reality=False)

    for _ in range(max(1, args.warmup)):
        step_cx()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_cx()
    torch.cuda.synchronize()
    ms_cx = (time.perf_counter() - t0) * 1e3 / args.steps
    complex_signal = {"ms_per_step": ms_cx, "complex_coeffs_per_s": Wc.numel() / (ms_cx * 1e-3),
                      "round_trip_rel_err": float((frm - fc).abs().max().item() / fc.abs().max().item())}
    del Wc
    print(f"# complex-signal round trip {ms_cx:.3f} ms/step", file=sys.stderr, flush=True)
    return {"steer": steer, "multires": multires, "driscoll_healy": dh_grid, "complex_signal": complex_signal}


def paper_sweep(args):
    """Analogue of the paper's numerical experiment (Sec. 3.4, Fig. 3): round trips of random
    band-limited signals whose f_lm have real and imaginary parts uniform in [-1, 1], N = 3,
    lambda = 2, all scales (J_min = 0), ten signals per band-limit L, on the equiangular grid
    and on the paper's Driscoll-Healy grid.  The error is the largest absolute difference
    between the reconstructed and the original f_lm (mean and worst over the ten signals);
    the time is the median device round trip (analysis with scaling, then synthesis) of one
    signal.  The slope of log time against log L over the three largest L is reported next to
    the paper's O(L^3)."""
    import numpy as np
    import torch
    from paper_1308_5706_amd import s2dw
    from paper_1308_5706_amd.inputs import random_flm_uniform

    N, lam, J_min, runs = 3, 2.0, 0, 10
    Ls = [int(x) for x in args.sweep_L.split(",")]
    out = {}
    for grid in ("mw", "dh"):
        rows = []
        for L in Ls:
            errs, times = [], []
            for r in range(runs):
                f = torch.as_tensor(random_flm_uniform(L, 100 + r)).to("cuda")
                if r == 0:  # plan and workspaces
                    W, Wp = s2dw.analysis(f, L, N, lam, J_min, grid=grid)
                    s2dw.synthesis(W, Wp, L, N, lam, J_min, grid=grid)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                W, Wp = s2dw.analysis(f, L, N, lam, J_min, grid=grid)
                fr = s2dw.synthesis(W, Wp, L, N, lam, J_min, grid=grid)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                errs.append(float((fr - f).abs().max().item()))
                W = Wp = fr = None
            rows.append({"L": L, "err_mean": float(np.mean(errs)), "err_max": float(np.max(errs)),
                         "ms": 1e3 * float(np.median(times))})
            print(f"# sweep {grid} L={L}: error {rows[-1]['err_mean']:.2e}, {rows[-1]['ms']:.3f} ms", file=sys.stderr,
                  flush=True)
        big = rows[-3:]
        slope = float(np.polyfit(np.log([q["L"] for q in big]), np.log([q["ms"] for q in big]), 1)[0])
        out[grid] = {"rows": rows, "time_slope_vs_L": slope}
    print(json.dumps({"paper_sweep": out, "N": N, "lambda": lam, "J_min": J_min, "signals_per_L": runs,
                      "signal": "f_lm real and imaginary parts uniform in [-1, 1] (real signal)",
                      "data": "synthetic"}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=1024)
    ap.add_argument("--N", type=int, default=8)
    ap.add_argument("--lam", type=float, default=2.0)
    ap.add_argument("--jmin", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="mixed: W in FP32 and the FFT stages / m'-sum in FP32 (Delta recursion and l-sum FP64)")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner pick the Wigner tile shape before timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline round trip (no steering / multiresolution / Driscoll-Healy / "
                         "complex-signal legs), e.g. under a profiler")
    ap.add_argument("--paper-sweep", action="store_true",
                    help="only run the analogue of the paper's accuracy and timing experiment (Fig. 3): "
                         "N = 3, all scales, ten uniform random signals per band-limit, both grids")
    ap.add_argument("--sweep-L", default="64,128,256,512,1024,2048", help="band-limits of --paper-sweep")
    ap.add_argument("--batch-maps", type=int, default=256, help="maps of the batched leg")
    ap.add_argument("--requests", type=int, default=10000, help="requests of the served leg")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device-to-device copy of this many GiB (to scale HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the library runs a "
              "transform on one GPU; maps and requests are independent, so several GPUs would each take "
              "their own)", file=sys.stderr)
        sys.exit(2)

    if args.paper_sweep:
        paper_sweep(args)
        return

    import numpy as np
    import torch
    from paper_1308_5706_amd import s2dw
    from paper_1308_5706_amd.inputs import random_flm

    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 30)) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "copies": 3}), flush=True)
        return

    L, N, lam, J_min = args.L, args.N, args.lam, args.jmin
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S = s2dw.num_scales(L, lam, J_min)
    f_host = random_flm(L, 0)
    f = torch.as_tensor(f_host).to(dev)
    prec = args.precision
    W = torch.empty((S, 2 * N - 1, L, 2 * L - 1), dtype=torch.float64 if prec == "fp64" else torch.float32,
                    device=dev)
    fr = torch.empty(L * L, dtype=torch.complex128, device=dev)
    print(f"# workload L={L} N={N} lambda={lam} J_min={J_min} scales={S}", file=sys.stderr, flush=True)

    tuned = None
    if args.autotune:
        tuned = s2dw.autotune(L, N, lam, J_min, count=1, precision=prec)
        print(f"# autotune: {tuned[0]} m' slots per wave, {tuned[1]} maps per chunk", file=sys.stderr, flush=True)

    def step():
        _, Wp = s2dw.analysis(f, L, N, lam, J_min, out=W, precision=prec)
        s2dw.synthesis(W, Wp, L, N, lam, J_min, out=fr, precision=prec)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"# warmup step {i} done", file=sys.stderr, flush=True)
    rt_err = float((fr - f).abs().max().item() / f.abs().max().item())

    def per_launch(stages):
        return {k: {"ms_per_launch": v[0] / v[1], "launches_per_step": v[1] / args.steps,
                    "ms_per_step": v[0] / args.steps} for k, v in stages.items()}

    # Per-stage breakdown from an untimed pass with every stage timed; it picks the kernel
    # with the largest device time per step (one stage = one kernel launch per scale, or per
    # direction for the Wigner stages).  Each timed launch adds two event records to the
    # stream, so the timed steps below record events around that stage only.
    s2dw.profile_stages(None)
    s2dw.profile(True)
    for _ in range(args.steps):
        step()
    per_stage = per_launch(s2dw.profile_read())
    s2dw.profile(False)
    dom = max(per_stage, key=lambda k: per_stage[k]["ms_per_step"])

    s2dw.profile_stages([dom])
    s2dw.profile(True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    spread = step_stats([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    live = per_launch(s2dw.profile_read())
    s2dw.profile(False)
    s2dw.profile_stages(None)
    print(f"# timed {args.steps} steps in {t1 - t0:.3f} s", file=sys.stderr, flush=True)

    ms_step = (t1 - t0) * 1e3 / args.steps
    coeffs = S * (2 * N - 1) * L * (2 * L - 1)
    value = coeffs / (ms_step * 1e-3)

    # roofline of that kernel, timed with HIP events during the timed steps
    kappa, _, _ = s2dw.wavelet_tables(L, N, lam, J_min)
    T = wigner_terms(kappa, N)
    units = stage_units(kappa, L, N, T, fused_adj=prec == "fp64", mixed=prec != "fp64")
    roof = roofline(dom, live[dom], units)
    traffic = None
    try:
        from paper_1308_5706_amd import profiling
        st = profiling.read_stage_traffic(f"round_trip_L{L}_N{N}")
        if st and dom in st:
            traffic = st[dom]["bytes_per_dispatch"]
    except Exception as e:  # a missing or unreadable summary leaves traffic unknown
        print(f"# traffic summary not used: {e}", file=sys.stderr)
    roof["traffic"] = traffic
    stage_roofs = {k: roofline(k, v, units) for k, v in per_stage.items() if k in units}

    extras = {} if args.no_extras else extra_legs(args, s2dw, torch, dev, f, W, fr, L, N, lam, J_min, S, prec)
    W = None
    torch.cuda.empty_cache()
    if not args.no_extras:
        print("# batched leg: 256 maps of mixed (L, N), mixed precision, one graph; then the persistent executor",
              file=sys.stderr, flush=True)
        extras["batched"] = batched_leg(args.batch_maps)
        s2dw.release_caches()
        torch.cuda.empty_cache()
        print(f"# served leg: {args.requests} Poisson requests, mixed L", file=sys.stderr, flush=True)
        from paper_1308_5706_amd import serve
        served = serve.benchmark(args.requests, 0.7, ("fp64", "mixed"))
        extras["served"] = {r["precision"]: r for r in served}
        s2dw.release_caches()
        torch.cuda.empty_cache()
        extras["gpu_config1"] = gpu_config1(s2dw, torch)

    out = {"metric": "SO(3) wavelet coeffs/s (analysis+synthesis) at L=1024,N=8; p50/p99 mixed-L",
           "value": value, "unit": "SO(3) coeffs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == "fp64" else "f32/f64", "data": "synthetic",
           "config": {"workload": f"SD wavelet round trip, one map, L={L}, N={N}, lambda={lam}, J_min={J_min}, "
                                  f"{S} scales, grid {2 * N - 1}x{L}x{2 * L - 1}",
                      "L": L, "N": N, "lambda": lam, "J_min": J_min, "scales": S, "coeffs_per_map": coeffs,
                      "precision": prec, "round_trip_rel_err": rt_err,
                      "wigner_slots": tuned[0] if tuned else None},
           "roofline": roof,
           "step_time": spread,
           "stages_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in per_stage.items()},
           "stages_roofline": {k: {"bound": v["bound"], "frac": round(v["frac"], 4),
                                   "achieved": round(v["achieved"], 2), "unit": v["unit"]}
                               for k, v in stage_roofs.items()},
           "wigner_terms_per_direction": T}
    out.update(extras)
    if "served" in extras:
        for prec_s, r in extras["served"].items():
            sfx = "" if prec_s == "fp64" else "_mixed"
            out["p50_ms" + sfx] = r["p50_ms"]
            out["p99_ms" + sfx] = r["p99_ms"]
    if "batched" in extras:
        out["batched_coeffs_per_s"] = extras["batched"]["value"]
        out["persistent_coeffs_per_s"] = extras["batched"]["persistent"]["value"]
    if not args.no_cpu_baseline:
        print("# cpu baseline sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(L, N, lam, J_min)
        if not args.no_extras:
            print("# oracle round trip at L=256, N=8, J_min=2", file=sys.stderr, flush=True)
            out["oracle_config1"] = oracle_config1()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
