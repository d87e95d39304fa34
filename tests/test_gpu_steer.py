"""Steering (Eq. 9-10): wavelet coefficients at arbitrary gamma from the 2N-1 grid samples,
against the oracle's Eq. 20 evaluated at those angles.  FP64 bar: relative max-error
<= 1e-11 per scale (relative to the largest magnitude of the oracle's values of that
scale); mixed precision (float W): <= 1e-5."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1308_5706_amd import s2dw
from paper_1308_5706_amd.inputs import random_flm

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(x).to("cuda")


def worst_per_scale(got, ref):
    return max(float(np.max(np.abs(got[j] - ref[j])) / np.max(np.abs(ref[j]))) for j in range(ref.shape[0]))


def angles(N, seed, q):
    # off-grid angles of both signs and beyond one turn, plus two grid angles
    rng = np.random.default_rng(seed)
    G = 2 * N - 1
    g = rng.uniform(-3 * math.pi, 5 * math.pi, q)
    return np.concatenate([g, [0.0, 2 * math.pi * (G - 1) / G]])


# (L, N, J_min): even and odd plane sizes (vector widths 2 and 1), N = 1 (gamma-independent),
# several angle chunks of the kernel
CASES = [(32, 4, 0), (33, 3, 1), (24, 1, 0), (48, 8, 1), (17, 16, 0)]


@pytest.mark.parametrize("L,N,J_min", CASES)
def test_steer_matches_oracle(L, N, J_min):
    print(f"steer L={L} N={N} J_min={J_min}", flush=True)
    f = random_flm(L, 500 + L)
    g = angles(N, L, 17)
    ref = oracle.analysis_at(f, L, N, 2.0, J_min, g)
    # the GPU analysis steered on the GPU (the whole path)
    W, _ = s2dw.analysis(dev(f), L, N, 2.0, J_min, scaling=False)
    Ws = s2dw.steer(W, g, L, N, 2.0, J_min)
    torch.cuda.synchronize()
    assert tuple(Ws.shape) == ref.shape
    assert worst_per_scale(Ws.cpu().numpy(), ref) < 1e-11
    # the oracle's grid coefficients steered on the GPU (the steering kernel alone)
    Wo = dev(np.ascontiguousarray(oracle.analysis(f, L, N, 2.0, J_min)))
    Wso = s2dw.steer(Wo, g, L, N, 2.0, J_min)
    torch.cuda.synchronize()
    assert worst_per_scale(Wso.cpu().numpy(), ref) < 1e-11


def test_steer_grid_angles_and_half_turn():
    L, N, J_min = 40, 5, 1
    f = random_flm(L, 7)
    G = 2 * N - 1
    W, _ = s2dw.analysis(dev(f), L, N, 2.0, J_min, scaling=False)
    Wg = s2dw.steer(W, 2 * np.pi * np.arange(G) / G, L, N, 2.0, J_min)
    g = np.array([0.4, 2.5])
    W0 = s2dw.steer(W, g, L, N, 2.0, J_min)
    W1 = s2dw.steer(W, g + np.pi, L, N, 2.0, J_min)
    torch.cuda.synchronize()
    scale = float(W.abs().max())
    assert float((Wg - W).abs().max()) < 1e-13 * scale
    assert float((W1 - (-1) ** (N - 1) * W0).abs().max()) < 1e-13 * scale


def test_steer_mixed_precision():
    L, N, J_min = 64, 8, 1
    f = random_flm(L, 9)
    g = angles(N, 3, 5)
    W, _ = s2dw.analysis(dev(f), L, N, 2.0, J_min, scaling=False, precision="mixed")
    assert W.dtype == torch.float32
    Ws = s2dw.steer(W, g, L, N, 2.0, J_min)
    torch.cuda.synchronize()
    assert Ws.dtype == torch.float32
    ref = oracle.analysis_at(f, L, N, 2.0, J_min, g)
    assert worst_per_scale(Ws.cpu().numpy().astype(np.float64), ref) < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_steer_batched_equals_single(precision):
    L, N, J_min, B = 30, 4, 0, 3
    F = torch.stack([dev(random_flm(L, 40 + i)) for i in range(B)])
    W, _ = s2dw.analysis_batched(F, L, N, 2.0, J_min, scaling=False, precision=precision)
    g = angles(N, 5, 10)
    Wb = s2dw.steer(W, g, L, N, 2.0, J_min)
    for i in range(B):
        assert torch.equal(Wb[i], s2dw.steer(W[i], g, L, N, 2.0, J_min)), i


def test_steer_empty_angle_list_and_errors():
    L, N = 16, 3
    W, _ = s2dw.analysis(dev(random_flm(L, 1)), L, N, 2.0, 0, scaling=False)
    out = s2dw.steer(W, [], L, N, 2.0, 0)
    assert out.shape[1] == 0
    with pytest.raises(ValueError):
        s2dw.steer(W[:, :2], [0.1], L, N, 2.0, 0)
