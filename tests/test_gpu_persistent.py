"""The persistent executor (many maps of several parameter sets, all scales, two launches per
direction): results against the per-group batched path and the oracle, mixed precision at its
bar, bitwise repeatability and graph replays, the bounded dependency wait forced from the host,
and the refusals of what it does not run.  FP64 bar: relative max-error <= 1e-11 against the
oracle, <= 1e-12 against the batched path (the same arithmetic in other tile shapes) and for
the round trip; mixed: <= 1e-5 against the FP64 results."""
import numpy as np
import pytest
import torch

import oracle
from paper_1308_5706_amd import s2dw
from paper_1308_5706_amd.inputs import random_flm

pytestmark = pytest.mark.gpu

# (L, N, lambda, J_min, maps): odd and even N (with and without the order n = 0), the
# direct fused alpha/gamma passes of the coarse scales and the transforms of the others
GROUPS = [(32, 2, 2.0, 1, 3), (64, 4, 2.0, 1, 2), (48, 8, 2.0, 1, 2), (40, 3, 2.0, 0, 1), (33, 1, 3.0, 0, 2)]


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def inputs(seed0=700):
    return [(L, N, lam, J, torch.stack([torch.as_tensor(random_flm(L, seed0 + 10 * g + i)) for i in range(B)]).to("cuda"))
            for g, (L, N, lam, J, B) in enumerate(GROUPS)]


def status_tensor():
    return torch.full((1,), -7, dtype=torch.int32, device="cuda")


def test_persistent_fp64_matches_batched_and_oracle():
    print("persistent FP64 analysis + synthesis, 5 groups", flush=True)
    ins = inputs()
    st = status_tensor()
    outs = s2dw.analysis_persistent(ins, status=st)
    torch.cuda.synchronize()
    assert st.item() == 0
    for (L, N, lam, J, f), (W, Wp) in zip(ins, outs):
        Wb, Wpb = s2dw.analysis_batched(f, L, N, lam, J)
        torch.cuda.synchronize()
        assert torch.equal(Wp, Wpb)
        Wh, Wbh = W.cpu().numpy(), Wb.cpu().numpy()
        for k in range(f.shape[0]):
            for j in range(Wh.shape[1]):
                assert rel(Wh[k, j], Wbh[k, j]) < 1e-12, (L, N, k, j)
        ref = oracle.analysis(f[0].cpu().numpy(), L, N, lam, J)
        e = max(rel(Wh[0, j], ref[j]) for j in range(ref.shape[0]))
        print(f"  L={L} N={N}: map 0 vs oracle {e:.2e}", flush=True)
        assert e < 1e-11
    st2 = status_tensor()
    fr = s2dw.synthesis_persistent([(L, N, lam, J, W, Wp) for (L, N, lam, J, _), (W, Wp) in zip(ins, outs)],
                                   status=st2)
    torch.cuda.synchronize()
    assert st2.item() == 0
    for (L, N, lam, J, f), (W, Wp), g in zip(ins, outs, fr):
        assert rel(g.cpu().numpy(), f.cpu().numpy()) < 1e-12, (L, N)
        gb = s2dw.synthesis_batched(W, Wp, L, N, lam, J)
        torch.cuda.synchronize()
        assert rel(g.cpu().numpy(), gb.cpu().numpy()) < 1e-12, (L, N)
    s2dw.release_caches()


def test_persistent_synthesis_of_arbitrary_samples():
    # W that is not the analysis of any f_lm (random samples): the persistent synthesis against
    # the batched one, which the synthesis parity tests hold to the oracle
    print("persistent synthesis of arbitrary samples", flush=True)
    rng = np.random.default_rng(5)
    items = []
    for L, N, lam, J, B in GROUPS[:3]:
        S = s2dw.num_scales(L, lam, J)
        W = torch.as_tensor(rng.standard_normal((B, S, 2 * N - 1, L, 2 * L - 1))).to("cuda")
        Wp = torch.as_tensor(rng.standard_normal((B, L * L)) + 1j * rng.standard_normal((B, L * L))).to("cuda")
        items.append((L, N, lam, J, W, Wp))
    fr = s2dw.synthesis_persistent(items)
    torch.cuda.synchronize()
    for (L, N, lam, J, W, Wp), g in zip(items, fr):
        gb = s2dw.synthesis_batched(W, Wp, L, N, lam, J)
        torch.cuda.synchronize()
        assert rel(g.cpu().numpy(), gb.cpu().numpy()) < 1e-12, (L, N)
    s2dw.release_caches()


def test_persistent_mixed_precision():
    print("persistent mixed precision", flush=True)
    ins = inputs(900)
    st = status_tensor()
    outs = s2dw.analysis_persistent(ins, precision="mixed", status=st)
    fr = s2dw.synthesis_persistent([(L, N, lam, J, W, Wp) for (L, N, lam, J, _), (W, Wp) in zip(ins, outs)],
                                   precision="mixed", status=st)
    torch.cuda.synchronize()
    assert st.item() == 0
    for (L, N, lam, J, f), (W, _), g in zip(ins, outs, fr):
        assert W.dtype == torch.float32
        Wd, _ = s2dw.analysis_batched(f, L, N, lam, J)
        torch.cuda.synchronize()
        Wh, Wdh = W.double().cpu().numpy(), Wd.cpu().numpy()
        e = max(rel(Wh[k, j], Wdh[k, j]) for k in range(f.shape[0]) for j in range(Wh.shape[1]))
        r = rel(g.cpu().numpy(), f.cpu().numpy())
        print(f"  L={L} N={N}: W {e:.1e}, round trip {r:.1e}", flush=True)
        assert e < 1e-5 and r < 1e-5
    s2dw.release_caches()


def test_persistent_repeats_and_graph_replays_bitwise():
    print("persistent repeat + graph capture", flush=True)
    ins = inputs(1100)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):  # first calls on the capture stream: record and upload the work lists
        outs = s2dw.analysis_persistent(ins, stream=s)
        fr = s2dw.synthesis_persistent([(L, N, lam, J, W, Wp) for (L, N, lam, J, _), (W, Wp) in zip(ins, outs)],
                                       stream=s)
    torch.cuda.synchronize()
    W_ref = [W.clone() for W, _ in outs]
    f_ref = [g.clone() for g in fr]
    with torch.cuda.stream(s):  # a second eager call: same results, bit for bit
        outs2 = s2dw.analysis_persistent(ins, stream=s)
    torch.cuda.synchronize()
    assert all(torch.equal(a[0], b) for a, b in zip(outs2, W_ref))
    st = status_tensor()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        outs3 = s2dw.analysis_persistent(ins, stream=s, status=st)
        fr3 = s2dw.synthesis_persistent([(L, N, lam, J, W, Wp) for (L, N, lam, J, _), (W, Wp) in zip(ins, outs3)],
                                        stream=s, status=st)
    for r in range(3):
        for W, _ in outs3:
            W.zero_()
        for x in fr3:
            x.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert st.item() == 0, r
        assert all(torch.equal(a[0], b) for a, b in zip(outs3, W_ref)), r
        assert all(torch.equal(a, b) for a, b in zip(fr3, f_ref)), r
        s2dw.analysis(ins[0][4][0], ins[0][0], ins[0][1], ins[0][2], ins[0][3])  # eager work between replays
        torch.cuda.synchronize()
    s2dw.release_caches()


def test_persistent_bounded_wait_forced_from_host():
    # every dependency wait made unsatisfiable (a host setting): each runs out after its bound,
    # the launches still finish, status reports it, and the next call runs clean
    print("persistent bounded wait", flush=True)
    ins = inputs(1300)[:2]
    good = s2dw.analysis_persistent(ins)
    torch.cuda.synchronize()
    W_ref = [W.clone() for W, _ in good]
    st = status_tensor()
    try:
        s2dw.persistent_wait_bound(200, never_satisfied=True)
        s2dw.analysis_persistent(ins, status=st)
        torch.cuda.synchronize()
        assert st.item() == 1
    finally:
        s2dw.persistent_wait_bound(0, never_satisfied=False)
    st2 = status_tensor()
    outs = s2dw.analysis_persistent(ins, status=st2)
    torch.cuda.synchronize()
    assert st2.item() == 0
    assert all(torch.equal(a[0], b) for a, b in zip(outs, W_ref))
    s2dw.release_caches()


def test_persistent_refusals():
    f = torch.as_tensor(random_flm(32, 1)).reshape(1, -1).to("cuda")
    with pytest.raises(s2dw.S2DWError) as e:
        s2dw.analysis_persistent([(32, 10, 2.0, 1, f)])  # N > 8
    assert e.value.code == -4
    big = torch.zeros((1, 1024 * 1024), dtype=torch.complex128, device="cuda")
    with pytest.raises(s2dw.S2DWError) as e:
        s2dw.analysis_persistent([(1024, 2, 2.0, 6, big)])  # transforms above 2048
    assert e.value.code == -4
    s2dw.release_caches()
