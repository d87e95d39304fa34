"""Batched + precision form: many maps of mixed (L, N) through the batched kernels, all
groups captured in one HIP graph and replayed; FP32 stages (mixed precision) with each
map's error against the FP64 result stated.

    python -m paper_1308_5706_amd.batch --maps 256

draws the maps' (L, N) from seeded generators (L uniform in {64, 128, 256, 512}, N uniform
in {2, 4, 8}, lambda = 2, J_min = 1, f_lm complex Gaussian with C_l = 1/(l+1)^2 and the
real-signal symmetry), lets the autotuner pick the Wigner tile shape and the batch chunk
per (L, N) group, captures the round trip (analysis with scaling + synthesis) of every
group in one graph, and reports the throughput of the replays next to the plain path (the
same maps one by one in FP64), plus per-map relative max-errors of the mixed-precision W
and round trip against the FP64 GPU path.  The same maps then go through the persistent
executor (every group in two launches per direction, the four captured in one graph), with
their throughput and errors reported beside.  The comparison of batched maps with the CPU
oracle belongs to the tests and to the benchmark's checker leg, not to this driver.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import s2dw
from .inputs import random_flm


def draw_maps(maps: int, seed: int = 3):
    """The (L, N) of each map: L uniform in {64, 128, 256, 512}, N uniform in {2, 4, 8}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = [int(x) for x in rng.choice([64, 128, 256, 512], size=maps)]
    Ns = [int(x) for x in rng.choice([2, 4, 8], size=maps)]
    return Ls, Ns


def run(maps: int = 256, replays: int = 5, lam: float = 2.0, J_min: int = 1):
    """Runs the batched leg; returns (result dict, per-map data) where per-map data maps
    (L, N) -> (map indices, f_lm [B][L*L], mixed W [B][...], round trip f [B][L*L], the
    persistent executor's mixed W [B][...]) on the device, for callers that check sampled
    maps against a reference."""
    Ls, Ns = draw_maps(maps)
    groups = {}
    for i, key in enumerate(zip(Ls, Ns)):
        groups.setdefault(key, []).append(i)
    F = {key: torch.stack([torch.as_tensor(random_flm(key[0], 3_000_000 + i)) for i in idx]).to("cuda")
         for key, idx in groups.items()}
    coeffs = sum(s2dw.num_scales(L, lam, J_min) * (2 * N - 1) * L * (2 * L - 1) for L, N in zip(Ls, Ns))

    # FP64 plain path (one map at a time) and its results, the reference for the errors
    ref = {}
    for key, f in F.items():  # warm the plans
        s2dw.analysis(f[0], key[0], key[1], lam, J_min)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for key, f in F.items():
        L, N = key
        Wl, fl = [], []
        for k in range(f.shape[0]):
            W, Wp = s2dw.analysis(f[k], L, N, lam, J_min)
            fl.append(s2dw.synthesis(W, Wp, L, N, lam, J_min))
            Wl.append(W)
        ref[key] = (Wl, fl)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    print(f"# plain FP64 path: {t_plain * 1e3:.1f} ms for {maps} maps", file=sys.stderr, flush=True)

    # mixed precision, batched per group with tuned shapes, all groups in one graph
    tuned = {}
    for key, f in F.items():
        tuned[key] = s2dw.autotune(key[0], key[1], lam, J_min, count=f.shape[0], precision="mixed")
    # The groups are independent: they go to `branches` streams forked from the capture stream
    # (heaviest first, each to the least loaded branch), so that the graph runs the small-L
    # groups' latency-bound kernels side by side.  The library keeps a workspace per stream.
    s = torch.cuda.Stream()
    branches = [torch.cuda.Stream() for _ in range(4)]
    load = [0.0] * len(branches)
    where = {}
    for key in sorted(F, key=lambda k: -F[k].shape[0] * k[0] ** 3 * k[1]):
        b = min(range(len(branches)), key=lambda i: load[i])
        where[key] = b
        load[b] += F[key].shape[0] * key[0] ** 3 * key[1]
    bufs = {}
    for key, f in F.items():  # warm-up on each group's stream: allocates its workspace
        L, N = key
        with torch.cuda.stream(branches[where[key]]):
            W, Wp = s2dw.analysis_batched(f, L, N, lam, J_min, precision="mixed")
            fr = s2dw.synthesis_batched(W, Wp, L, N, lam, J_min, precision="mixed")
            bufs[key] = (W, Wp, fr)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for b in branches:
            b.wait_stream(s)
        for key, f in F.items():
            L, N = key
            W, Wp, fr = bufs[key]
            with torch.cuda.stream(branches[where[key]]):
                s2dw.analysis_batched(f, L, N, lam, J_min, out=W, precision="mixed")
                s2dw.synthesis_batched(W, Wp, L, N, lam, J_min, out=fr, precision="mixed")
        for b in branches:
            s.wait_stream(b)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / replays

    errs_w, errs_rt = [], []
    for key, f in F.items():
        W, Wp, fr = bufs[key]
        Wl, fl = ref[key]
        for k in range(f.shape[0]):
            a = W[k].double()
            errs_w.append(float((a - Wl[k]).abs().max() / Wl[k].abs().max()))
            errs_rt.append(float((fr[k] - f[k]).abs().max() / f[k].abs().max()))
    del g

    # the persistent executor: every group's maps through two launches per direction, the
    # four launches captured in one graph
    keys = list(F.keys())
    ins = [(L, N, lam, J_min, F[(L, N)]) for L, N in keys]
    with torch.cuda.stream(s):  # first calls on the capture stream record and upload the work lists
        pouts = s2dw.analysis_persistent(ins, precision="mixed", stream=s)
        pfr = s2dw.synthesis_persistent([(L, N, lam, J_min, W, Wp) for (L, N, _, _, _), (W, Wp) in zip(ins, pouts)],
                                        precision="mixed", stream=s)
    torch.cuda.synchronize()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    gp = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gp, stream=s):
        s2dw.analysis_persistent(ins, precision="mixed", stream=s, status=status)
        s2dw.synthesis_persistent([(L, N, lam, J_min, W, Wp) for (L, N, _, _, _), (W, Wp) in zip(ins, pouts)],
                                  precision="mixed", stream=s, status=status)
    gp.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        gp.replay()
    torch.cuda.synchronize()
    t_pers = (time.perf_counter() - t0) / replays
    if int(status.item()) != 0:
        raise RuntimeError("persistent executor: a dependency wait ran out")
    perr_w, perr_rt = [], []
    for (L, N), (W, _), fr in zip(keys, pouts, pfr):
        Wl, _ = ref[(L, N)]
        f = F[(L, N)]
        for k in range(f.shape[0]):
            perr_w.append(float((W[k].double() - Wl[k]).abs().max() / Wl[k].abs().max()))
            perr_rt.append(float((fr[k] - f[k]).abs().max() / f[k].abs().max()))
    del gp
    persistent = {"value": coeffs / t_pers, "ms_per_batch": t_pers * 1e3, "launches_per_direction": 2,
                  "speedup_vs_plain": t_plain / t_pers, "speedup_vs_per_group_graph": t_graph / t_pers,
                  "max_rel_err_W_vs_fp64": max(perr_w), "max_rel_err_round_trip": max(perr_rt)}
    out = {"metric": "SO(3) wavelet coeffs/s (analysis+synthesis), batched mixed-(L, N) maps, mixed precision",
           "value": coeffs / t_graph, "unit": "SO(3) coeffs/s", "maps": maps, "ms_per_batch": t_graph * 1e3,
           "plain_fp64_ms": t_plain * 1e3, "plain_fp64_coeffs_per_s": coeffs / t_plain,
           "speedup_vs_plain": t_plain / t_graph, "groups": len(groups),
           "tuned": {f"{k[0]},{k[1]}": v for k, v in tuned.items()},
           "max_rel_err_W_vs_fp64": max(errs_w), "max_rel_err_round_trip": max(errs_rt),
           "median_rel_err_W_vs_fp64": float(np.median(errs_w)), "persistent": persistent, "data": "synthetic"}
    pW = {key: W for key, (W, _) in zip(keys, pouts)}
    data = {key: (groups[key], F[key], bufs[key][0], bufs[key][2], pW[key]) for key in F}
    return out, data


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--maps", type=int, default=256)
    ap.add_argument("--replays", type=int, default=5)
    args = ap.parse_args()
    out, _ = run(args.maps, args.replays)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
