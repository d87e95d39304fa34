"""Multiresolution layout (each scale on the equiangular grid of its own band-limit L_j,
Sec. 3.2 closing remarks): analysis, synthesis, round trip, batched, mixed-precision and
steered forms against the oracle.  FP64 bar: relative max-error <= 1e-11 per scale (relative
to the largest magnitude of the oracle's array of that scale); round trip <= 1e-12; mixed
precision <= 1e-5."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import tables
from paper_1308_5706_amd import s2dw
from paper_1308_5706_amd.inputs import random_flm, random_wavelet_samples

pytestmark = pytest.mark.gpu

TOL = 1e-11


def rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / (den if den > 0 else 1.0))


def dev(x):
    return torch.as_tensor(x).to("cuda")


def flat(Ws):
    return np.concatenate([np.asarray(w).reshape(-1) for w in Ws])


CASES = [  # (L, N, J_min, lambda)
    (32, 4, 0, 2.0),
    (33, 3, 1, 2.0),   # odd L: odd plane sizes
    (64, 8, 1, 2.0),   # coarse scales with L_j < N
    (27, 3, 0, 3.0),
    (30, 2, 1, 1.7),   # non-dyadic band-limits
    (130, 5, 2, 2.0),
]


def test_band_limits_match_the_oracle():
    for L, N, J_min, lam in CASES:
        bl = oracle.scale_bandlimits(L, lam, J_min)
        for j, Lj in enumerate(bl):
            sh, _ = s2dw.scale_grid(L, N, lam, J_min, j, grid="multires")
            assert sh == (2 * N - 1, Lj, 2 * Lj - 1 if Lj else 0)


@pytest.mark.parametrize("L,N,J_min,lam", CASES)
def test_multires_analysis_matches_oracle(L, N, J_min, lam):
    print(f"multires analysis L={L} N={N} J_min={J_min} lambda={lam}", flush=True)
    f = random_flm(L, 600 + L)
    ref = oracle.analysis_multires(f, L, N, lam, J_min)
    W, Wp = s2dw.analysis(dev(f), L, N, lam, J_min, grid="multires")
    got = [w.cpu().numpy() for w in s2dw.split_scales(W, L, N, lam, J_min)]
    for j in range(len(ref)):
        assert got[j].shape == ref[j].shape
        if ref[j].size:
            assert rel(got[j], ref[j]) < TOL, (j, rel(got[j], ref[j]))
    assert rel(Wp.cpu().numpy(), oracle.scaling(f, L, lam, J_min)) < TOL


@pytest.mark.parametrize("L,N,J_min,lam", CASES)
def test_multires_synthesis_matches_oracle_on_arbitrary_samples(L, N, J_min, lam):
    print(f"multires synthesis L={L} N={N} J_min={J_min} lambda={lam}", flush=True)
    bl = oracle.scale_bandlimits(L, lam, J_min)
    Ws = [random_wavelet_samples(1, 2 * N - 1, Lj, max(2 * Lj - 1, 0), 700 + j)[0] for j, Lj in enumerate(bl)]
    Wphi = oracle.scaling(random_flm(L, 701), L, lam, J_min)
    ref = oracle.synthesis_multires(Ws, Wphi, L, N, lam, J_min)
    got = s2dw.synthesis(dev(flat(Ws)), dev(Wphi), L, N, lam, J_min, grid="multires").cpu().numpy()
    assert rel(got, ref) < TOL, rel(got, ref)


@pytest.mark.parametrize("L,N,J_min,lam", CASES)
def test_multires_round_trip(L, N, J_min, lam):
    f = random_flm(L, 800 + L)
    W, Wp = s2dw.analysis(dev(f), L, N, lam, J_min, grid="multires")
    fr = s2dw.synthesis(W, Wp, L, N, lam, J_min, grid="multires").cpu().numpy()
    assert rel(fr, f) < 1e-12


def test_multires_medium_configuration_and_size():
    L, N, J_min = 256, 8, 2
    print("multires medium configuration", flush=True)
    f = random_flm(L, 0)
    ref = oracle.analysis_multires(f, L, N, 2.0, J_min)
    W, Wp = s2dw.analysis(dev(f), L, N, 2.0, J_min, grid="multires")
    assert W.numel() == sum(r.size for r in ref)
    full = s2dw.num_scales(L, 2.0, J_min) * (2 * N - 1) * L * (2 * L - 1)
    assert W.numel() < 0.4 * full
    got = [w.cpu().numpy() for w in s2dw.split_scales(W, L, N, 2.0, J_min)]
    for j in range(len(ref)):
        assert rel(got[j], ref[j]) < TOL, j
    refs = oracle.synthesis_multires(ref, oracle.scaling(f, L, 2.0, J_min), L, N, 2.0, J_min)
    assert rel(s2dw.synthesis(W, Wp, L, N, 2.0, J_min, grid="multires").cpu().numpy(), refs) < TOL


def test_multires_mixed_precision():
    L, N, J_min = 64, 4, 1
    f = random_flm(L, 9)
    ref = oracle.analysis_multires(f, L, N, 2.0, J_min)
    W, Wp = s2dw.analysis(dev(f), L, N, 2.0, J_min, grid="multires", precision="mixed")
    assert W.dtype == torch.float32
    got = [w.cpu().numpy().astype(np.float64) for w in s2dw.split_scales(W, L, N, 2.0, J_min)]
    for j in range(len(ref)):
        assert rel(got[j], ref[j]) < 1e-5, j
    fr = s2dw.synthesis(W, Wp, L, N, 2.0, J_min, grid="multires", precision="mixed").cpu().numpy()
    assert rel(fr, f) < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_multires_batched_equals_single(precision):
    L, N, J_min, B = 40, 4, 1, 3
    F = torch.stack([dev(random_flm(L, 50 + i)) for i in range(B)])
    W, Wp = s2dw.analysis_batched(F, L, N, 2.0, J_min, precision=precision, grid="multires")
    fr = s2dw.synthesis_batched(W, Wp, L, N, 2.0, J_min, precision=precision, grid="multires")
    for i in range(B):
        Wi, Wpi = s2dw.analysis(F[i], L, N, 2.0, J_min, precision=precision, grid="multires")
        assert torch.equal(W[i], Wi), i
        fi = s2dw.synthesis(Wi, Wpi, L, N, 2.0, J_min, precision=precision, grid="multires")
        assert torch.equal(fr[i], fi), i


def test_multires_steer_matches_oracle():
    L, N, J_min = 48, 5, 1
    f = random_flm(L, 11)
    g = np.array([0.3, -1.9, 7.5, 0.0])
    W, _ = s2dw.analysis(dev(f), L, N, 2.0, J_min, scaling=False, grid="multires")
    Ws = s2dw.steer(W, g, L, N, 2.0, J_min, grid="multires").cpu().numpy()
    psi = tables.wavelets(L, N, 2.0, J_min)
    off = 0
    for j, Lj in enumerate(oracle.scale_bandlimits(L, 2.0, J_min)):
        n = len(g) * Lj * (2 * Lj - 1)
        got = Ws[off:off + n].reshape(len(g), Lj, 2 * Lj - 1)
        off += n
        ref = oracle.analysis_at(f, L, N, 2.0, J_min, g, betas=oracle.mw_betas(Lj), psi=psi[j:j + 1],
                                 nalpha=2 * Lj - 1)[0]
        assert rel(got, ref) < TOL, j
    assert off == Ws.size
