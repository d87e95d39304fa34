"""Batched form: a batch of maps through the same launches equals the single-map calls
bitwise; the autotuner keeps parity with the oracle; batched calls captured in a HIP graph
replay to the eager result."""
import numpy as np
import pytest
import torch

import oracle
from paper_1308_5706_amd import s2dw
from paper_1308_5706_amd.inputs import random_flm

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(x).to("cuda")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("L,N,J_min,precision", [(48, 4, 0, "fp64"), (64, 8, 1, "mixed"), (33, 3, 1, "fp64")])
def test_batched_equals_single_calls(L, N, J_min, precision):
    print(f"batched L={L} N={N} J_min={J_min} {precision}", flush=True)
    B = 5
    F = torch.stack([dev(random_flm(L, 100 + i)) for i in range(B)])
    W, Wp = s2dw.analysis_batched(F, L, N, 2.0, J_min, precision=precision)
    fr = s2dw.synthesis_batched(W, Wp, L, N, 2.0, J_min, precision=precision)
    for i in range(B):
        Wi, Wpi = s2dw.analysis(F[i], L, N, 2.0, J_min, precision=precision)
        assert torch.equal(W[i], Wi), i
        assert torch.equal(Wp[i], Wpi), i
        fi = s2dw.synthesis(Wi, Wpi, L, N, 2.0, J_min, precision=precision)
        assert torch.equal(fr[i], fi), i


def test_autotune_keeps_parity():
    L, N, J_min = 64, 8, 1
    print("autotune", flush=True)
    slots, chunk = s2dw.autotune(L, N, 2.0, J_min, count=8)
    print(f"  picked {slots} m' slots per wave, {chunk} maps per chunk", flush=True)
    assert slots in (1, 2, 4) and 1 <= chunk <= 8
    F = torch.stack([dev(random_flm(L, 200 + i)) for i in range(3)])
    W, Wp = s2dw.analysis_batched(F, L, N, 2.0, J_min)
    fr = s2dw.synthesis_batched(W, Wp, L, N, 2.0, J_min)
    torch.cuda.synchronize()
    ref = oracle.analysis(F[1].cpu().numpy(), L, N, 2.0, J_min)
    Wh = W[1].cpu().numpy()
    for j in range(ref.shape[0]):
        assert rel(Wh[j], ref[j]) < 1e-11
    assert float((fr - F).abs().max() / F.abs().max()) < 1e-12


def test_graph_capture_replays_match_eager():
    L, N, J_min, B = 40, 4, 1, 3
    print("graph capture", flush=True)
    F = torch.stack([dev(random_flm(L, 300 + i)) for i in range(B)])
    s = torch.cuda.Stream()
    S = s2dw.num_scales(L, 2.0, J_min)
    W = torch.empty((B, S, 2 * N - 1, L, 2 * L - 1), dtype=torch.float64, device="cuda")
    Wp = torch.empty((B, L * L), dtype=torch.complex128, device="cuda")
    fr = torch.empty((B, L * L), dtype=torch.complex128, device="cuda")
    with torch.cuda.stream(s):  # warm-up on the capture stream: builds the plan and its workspace
        s2dw.analysis_batched(F, L, N, 2.0, J_min, out=W)
        s2dw.synthesis_batched(W, None, L, N, 2.0, J_min, out=fr)
    torch.cuda.synchronize()
    W_ref = W.clone()
    f_ref = fr.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        s2dw.analysis_batched(F, L, N, 2.0, J_min, out=W)
        s2dw.synthesis_batched(W, None, L, N, 2.0, J_min, out=fr)
    for r in range(3):
        W.zero_()
        fr.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(W, W_ref), r
        assert torch.equal(fr, f_ref), r
        # eager work between replays
        s2dw.analysis(F[0], L, N, 2.0, J_min)
        torch.cuda.synchronize()


def test_graph_branches_replay_match_eager():
    # two (L, N) groups on two streams forked from the capture stream and joined back (as the
    # batched leg captures its groups): every replay equals the eager results bitwise, with
    # eager work between the replays
    print("graph capture on two branches", flush=True)
    groups = [(40, 4, 1, 3), (33, 3, 0, 2)]
    s = torch.cuda.Stream()
    branches = [torch.cuda.Stream(), torch.cuda.Stream()]
    F, bufs, refs = {}, {}, {}
    for k, (L, N, J_min, B) in enumerate(groups):
        F[k] = torch.stack([dev(random_flm(L, 500 + 10 * k + i)) for i in range(B)])
        S = s2dw.num_scales(L, 2.0, J_min)
        W = torch.empty((B, S, 2 * N - 1, L, 2 * L - 1), dtype=torch.float64, device="cuda")
        fr = torch.empty((B, L * L), dtype=torch.complex128, device="cuda")
        with torch.cuda.stream(branches[k]):  # warm-up on the branch: its workspace
            s2dw.analysis_batched(F[k], L, N, 2.0, J_min, out=W)
            s2dw.synthesis_batched(W, None, L, N, 2.0, J_min, out=fr)
        torch.cuda.synchronize()
        bufs[k] = (W, fr)
        refs[k] = (W.clone(), fr.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for b in branches:
            b.wait_stream(s)
        for k, (L, N, J_min, B) in enumerate(groups):
            W, fr = bufs[k]
            with torch.cuda.stream(branches[k]):
                s2dw.analysis_batched(F[k], L, N, 2.0, J_min, out=W)
                s2dw.synthesis_batched(W, None, L, N, 2.0, J_min, out=fr)
        for b in branches:
            s.wait_stream(b)
    for r in range(3):
        for W, fr in bufs.values():
            W.zero_()
            fr.zero_()
        g.replay()
        torch.cuda.synchronize()
        for k in bufs:
            assert torch.equal(bufs[k][0], refs[k][0]), (r, k)
            assert torch.equal(bufs[k][1], refs[k][1]), (r, k)
        L, N, J_min, _ = groups[0]
        s2dw.analysis(F[0][0], L, N, 2.0, J_min)  # eager work between replays
        torch.cuda.synchronize()


def test_batched_mixed_maps_against_oracle():
    # the batched mixed-precision form of the many-maps configuration (L from {64, 128}, N from
    # {2, 4, 8}, J_min = 1), every map of each batch against the FP64 oracle at the mixed bar
    print("batched mixed-precision maps vs oracle", flush=True)
    lam, J_min = 2.0, 1
    for (L, N) in [(64, 8), (128, 2), (128, 4)]:
        F = torch.stack([dev(random_flm(L, 3_000_000 + 10 * L + N + i)) for i in range(3)])
        W, Wp = s2dw.analysis_batched(F, L, N, lam, J_min, precision="mixed")
        fr = s2dw.synthesis_batched(W, Wp, L, N, lam, J_min, precision="mixed")
        torch.cuda.synchronize()
        for k in range(F.shape[0]):
            fk = F[k].cpu().numpy()
            ref = oracle.analysis(fk, L, N, lam, J_min)
            Wk = W[k].double().cpu().numpy()
            e = max(rel(Wk[j], ref[j]) for j in range(ref.shape[0]))
            print(f"  L={L} N={N} map {k}: W rel. error {e:.1e}", flush=True)
            assert e < 1e-5, (L, N, k, e)
            assert rel(fr[k].cpu().numpy(), fk) < 1e-5
