"""Parity at the full sizes of the large configurations, on outputs the oracle can compute
one at a time: whole beta rows of W (every scale, gamma and alpha sample), in the same
launch configuration the benchmark times; plus the exact round trip, which holds at any
size.  FP64 bar: relative max-error <= 1e-11 per scale, relative to the largest magnitude
of the oracle's sampled rows of that scale."""
import numpy as np
import pytest
import torch

import oracle
from oracle import tables
from paper_1308_5706_amd import s2dw
from paper_1308_5706_amd.inputs import random_flm

pytestmark = pytest.mark.gpu

TOL = 1e-11

FULL = [  # (L, N, J_min): the large configuration and the benchmark workload
    (2048, 4, 4),
    (1024, 8, 1),
]


@pytest.mark.parametrize("L,N,J_min", FULL)
def test_full_size_rows_and_round_trip(L, N, J_min):
    lam = 2.0
    print(f"full size L={L} N={N} J_min={J_min}: analysis on the GPU", flush=True)
    f = random_flm(L, 0)
    fd = torch.as_tensor(f).to("cuda")
    W, Wp = s2dw.analysis(fd, L, N, lam, J_min)
    torch.cuda.synchronize()
    rows = [0, L // 3, L - 2, L - 1]  # includes beta = pi (b = L - 1)
    got = W[:, :, rows, :].cpu().numpy()
    print("  oracle on the sampled beta rows", flush=True)
    psi = tables.wavelets(L, N, lam, J_min)
    ref = oracle.analysis(f, L, N, lam, J_min, betas=oracle.mw_betas(L)[rows], psi=psi)
    assert got.shape == ref.shape
    for j in range(ref.shape[0]):
        den = np.max(np.abs(ref[j]))
        err = float(np.max(np.abs(got[j] - ref[j])) / den)
        assert err < TOL, (j, err)
    print("  steering (Eq. 10) to off-grid angles, two sampled beta rows", flush=True)
    g = np.array([0.7, -2.1])
    Ws = s2dw.steer(W, g, L, N, lam, J_min)
    got = Ws[:, :, rows[:2], :].cpu().numpy()
    del Ws
    ref = oracle.analysis_at(f, L, N, lam, J_min, g, betas=oracle.mw_betas(L)[rows[:2]], psi=psi)
    for j in range(ref.shape[0]):
        err = float(np.max(np.abs(got[j] - ref[j])) / np.max(np.abs(ref[j])))
        assert err < TOL, (j, err)
    print("  synthesis on the GPU (round trip)", flush=True)
    fr = s2dw.synthesis(W, Wp, L, N, lam, J_min)
    torch.cuda.synchronize()
    rt = float((fr - fd).abs().max().item() / fd.abs().max().item())
    assert rt < 1e-12, rt
    del W, Wp, fr
    s2dw.release_caches()
    torch.cuda.empty_cache()


def test_full_size_multires_rows_and_round_trip():
    # the benchmark workload in the multiresolution layout: sampled beta rows of the finest and
    # of a coarse scale against the oracle, and the exact round trip
    L, N, J_min, lam = 1024, 8, 1, 2.0
    print(f"full size multires L={L} N={N} J_min={J_min}", flush=True)
    f = random_flm(L, 0)
    fd = torch.as_tensor(f).to("cuda")
    W, Wp = s2dw.analysis(fd, L, N, lam, J_min, grid="multires")
    scales = s2dw.split_scales(W, L, N, lam, J_min)
    psi = tables.wavelets(L, N, lam, J_min)
    for j in [0, 5]:
        Lj = scales[j].shape[1]
        rows = [0, Lj - 1]
        got = scales[j][:, rows, :].cpu().numpy()
        print(f"  oracle on scale {j} (L_j = {Lj}), rows {rows}", flush=True)
        ref = oracle.analysis_at(f, L, N, lam, J_min, 2 * np.pi * np.arange(2 * N - 1) / (2 * N - 1),
                                 betas=oracle.mw_betas(Lj)[rows], psi=psi[j:j + 1], nalpha=2 * Lj - 1)[0]
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        assert err < TOL, (j, err)
    fr = s2dw.synthesis(W, Wp, L, N, lam, J_min, grid="multires")
    torch.cuda.synchronize()
    rt = float((fr - fd).abs().max().item() / fd.abs().max().item())
    assert rt < 1e-12, rt
    del W, Wp, fr, scales
    s2dw.release_caches()
    torch.cuda.empty_cache()


def test_full_size_driscoll_healy_rows_and_round_trip():
    # the benchmark workload on the paper's own grid (Sec. 3.1): 2L colatitudes, N base
    # orientations; sampled beta rows against the oracle and the exact round trip
    L, N, J_min, lam = 1024, 8, 1, 2.0
    print(f"full size Driscoll-Healy L={L} N={N} J_min={J_min}", flush=True)
    f = random_flm(L, 0)
    fd = torch.as_tensor(f).to("cuda")
    W, Wp = s2dw.analysis(fd, L, N, lam, J_min, grid="dh")
    rows = [0, L, 2 * L - 1]
    got = W[:, :, rows, :].cpu().numpy()
    print("  oracle on the sampled beta rows", flush=True)
    ref = oracle.analysis_at(f, L, N, lam, J_min, np.pi * np.arange(N) / N, betas=oracle.dh_betas(L)[rows])
    for j in range(ref.shape[0]):
        err = float(np.max(np.abs(got[j] - ref[j])) / np.max(np.abs(ref[j])))
        assert err < TOL, (j, err)
    fr = s2dw.synthesis(W, Wp, L, N, lam, J_min, grid="dh")
    torch.cuda.synchronize()
    rt = float((fr - fd).abs().max().item() / fd.abs().max().item())
    assert rt < 1e-12, rt
    del W, Wp, fr
    s2dw.release_caches()
    torch.cuda.empty_cache()


def test_full_size_complex_signal_rows_and_round_trip():
    # a complex signal at the benchmark workload: complex coefficients on sampled beta rows
    # against the oracle, and the exact round trip
    from paper_1308_5706_amd.inputs import random_flm_complex
    L, N, J_min, lam = 1024, 8, 1, 2.0
    print(f"full size complex signal L={L} N={N} J_min={J_min}", flush=True)
    f = random_flm_complex(L, 0)
    fd = torch.as_tensor(f).to("cuda")
    W, Wp = s2dw.analysis(fd, L, N, lam, J_min, reality=False)
    rows = [0, L - 1]
    got = W[:, :, rows, :].cpu().numpy()
    print("  oracle on the sampled beta rows", flush=True)
    ref = oracle.analysis_complex(f, L, N, lam, J_min, betas=oracle.mw_betas(L)[rows])
    for j in range(ref.shape[0]):
        err = float(np.max(np.abs(got[j] - ref[j])) / np.max(np.abs(ref[j])))
        assert err < TOL, (j, err)
    fr = s2dw.synthesis(W, Wp, L, N, lam, J_min, reality=False)
    torch.cuda.synchronize()
    rt = float((fr - fd).abs().max().item() / fd.abs().max().item())
    assert rt < 1e-12, rt
    del W, Wp, fr
    s2dw.release_caches()
    torch.cuda.empty_cache()
