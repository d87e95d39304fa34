"""Pins of the oracle's wavelet tables (Sec. 2.2, Eq. 6-16) against facts the
paper fixes: admissibility, peak and support of the kernels, the normalisation
and parity of the directionality coefficients, J_L, and hand-evaluated values."""
import json
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import tables

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("L,lam,J_min", [(32, 2.0, 0), (128, 2.0, 2), (256, 2.0, 2), (100, 1.5, 1),
                                         (81, 3.0, 0), (1024, 2.0, 1)])
def test_admissibility_resolution_of_identity(L, lam, J_min):
    # Eq. 6: |Phi_l0|^2 + sum_j sum_m |Psi^j_lm|^2 = 1 for every l
    psi = tables.wavelets(L, 4, lam, J_min)
    phi = tables.phi_table(L, lam, J_min)
    total = phi ** 2 + (np.abs(psi) ** 2).sum(axis=(0, 2))
    # for l = 0 the wavelets vanish (kappa^j(0) = 0) and Phi_00 = 1
    assert np.max(np.abs(total - 1.0)) < 5e-15


def test_admissibility_catches_a_dropped_scale():
    # the pin is sensitive: dropping any one scale breaks it somewhere
    L, lam, J_min = 128, 2.0, 1
    kap = tables.kappa_table(L, lam, J_min)
    phi = tables.phi_table(L, lam, J_min)
    for j in range(kap.shape[0]):
        total = phi ** 2 + np.delete(kap, j, axis=0).__pow__(2).sum(axis=0)
        assert np.max(np.abs(total - 1.0)) > 1e-3


@pytest.mark.parametrize("lam", [2.0, 1.5, 3.0])
def test_kernel_peak_and_support(lam):
    # kappa_lambda reaches a peak of unity at t = 1, support [1/lambda, lambda] (Sec. 2.2)
    assert abs(tables.kappa_lambda(1.0, lam) - 1.0) < 1e-15
    for t in np.linspace(1.0 / lam, lam, 41)[1:-1]:
        assert tables.kappa_lambda(t, lam) <= 1.0 + 1e-15
        assert tables.kappa_lambda(t, lam) > 0.0
    for t in [0.0, 0.5 / lam, 1.0 / lam, lam, 1.5 * lam]:
        assert tables.kappa_lambda(t, lam) == 0.0
    # k_lambda is 1 below 1/lambda, 0 above 1, decreasing in between (Eq. 13)
    ts = np.linspace(1.0 / lam, 1.0, 30)
    ks = [tables.k_lambda(t, lam) for t in ts]
    assert ks[0] == 1.0 and ks[-1] == 0.0
    assert all(a >= b for a, b in zip(ks, ks[1:]))


def test_k_lambda_against_independent_quadrature():
    # Eq. 13 evaluated with mpmath's tanh-sinh quadrature at 30 digits
    mpmath.mp.dps = 30
    lam = 2.0

    def s2(u):
        x = 2 * lam / (lam - 1) * (u - 1 / lam) - 1
        return mpmath.exp(-2 / (1 - x * x)) / u if -1 < x < 1 else mpmath.mpf(0)

    den = mpmath.quad(s2, [1 / lam, 0.75, 1])
    for t in [0.55, 0.6, 0.75, 0.9, 0.97]:
        ref = mpmath.quad(s2, [t, 1]) / den
        assert abs(tables.k_lambda(t, lam) - float(ref)) < 2e-14


def test_fig1_tiling_fixture():
    g = json.load(open(os.path.join(GOLDEN, "fig1_tiling.json")))
    L, lam, J = g["L"], g["lambda"], g["J"]
    assert tables.j_max(L, lam) == g["J_L"]
    J_min = g["J_L"] - J
    kap = tables.kappa_table(L, lam, J_min)
    assert kap.shape == (J + 1, L)
    els = np.arange(L)
    for j, ((lo, hi), peak) in enumerate(zip(g["supports"], g["peaks"])):
        # zero outside the printed support and at its ends; positive inside it, except
        # in the tails next to the ends where the value underflows double precision
        assert np.all(kap[j][(els <= lo) | (els >= hi)] == 0.0)
        inside = (els > lo * 1.06) & (els < hi / 1.06)
        assert np.all(kap[j][inside] > 0.0)
        # rising up to the peak, falling after it
        up = kap[j][(els > lo) & (els <= min(peak, L - 1))]
        down = kap[j][(els >= peak) & (els < hi)]
        assert np.all(np.diff(up) >= 0) and np.all(np.diff(down) <= 0)
        if peak < L:
            assert abs(kap[j][peak] - 1.0) < 1e-15
    phi = tables.phi_table(L, lam, J_min)
    assert np.all(phi[: g["scaling_one_below"] + 1] == 1.0)
    assert np.all(phi[g["scaling_zero_from"]:] == 0.0)


@pytest.mark.parametrize("L,lam,J", [(1024, 2.0, 10), (1000, 2.0, 10), (1025, 2.0, 11), (81, 3.0, 4),
                                     (82, 3.0, 5), (2, 2.0, 1), (2048, 2.0, 11)])
def test_j_max(L, lam, J):
    assert tables.j_max(L, lam) == J
    assert lam ** (-J) * L <= 1.0 < lam ** (-(J - 1)) * L


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 8])
def test_directionality_normalisation_and_parity(N):
    L = 40
    s = tables.directionality(L, N)
    # Eq. 8: sum_m |s_lm|^2 = 1 wherever s_l is non-zero; s_lm = 0 for |m| >= N (by storage)
    norms = (np.abs(s) ** 2).sum(axis=1)
    for el in range(L):
        assert norms[el] == pytest.approx(1.0, abs=1e-15) or norms[el] == 0.0
    assert np.all(norms[1:] > 0.5)
    for n in range(-(N - 1), N):
        col = s[:, n + N - 1]
        if (N + n) % 2 == 0:  # beta_(N,n) = 0
            assert np.all(col == 0)
    # a real wavelet: s_{l,-n} = (-1)^n conj(s_ln); odd (even) azimuthal symmetry for N even (odd)
    for n in range(-(N - 1), N):
        assert np.allclose(s[:, -n + N - 1], (-1) ** n * np.conj(s[:, n + N - 1]), atol=0, rtol=0)
        if np.any(s[:, n + N - 1] != 0):
            assert (-1) ** n == (-1 if N % 2 == 0 else 1)


def test_directionality_hand_values():
    # Eq. 11 evaluated by hand for l >= N (gamma_(N,l) = N - 1)
    s2 = tables.directionality(10, 2)
    assert s2[5, 0] == pytest.approx(1j / math.sqrt(2), abs=3e-16)
    assert s2[5, 2] == pytest.approx(1j / math.sqrt(2), abs=3e-16)
    s3 = tables.directionality(10, 3)
    assert s3[5, 2] == pytest.approx(math.sqrt(0.5), abs=3e-16)    # n = 0: sqrt(C(2,1)/4)
    assert s3[5, 0] == pytest.approx(0.5, abs=3e-16)               # n = -2: sqrt(C(2,0)/4)
    s4 = tables.directionality(10, 4)
    assert s4[5, 3 + 3] == pytest.approx(1j * math.sqrt(1 / 8), abs=3e-16)  # n = 3
    assert s4[5, 1 + 3] == pytest.approx(1j * math.sqrt(3 / 8), abs=3e-16)  # n = 1
    # small l: gamma_(N,l) < N - 1.  N = 4, l = 2: gamma = min(3, 2 - 1) = 1 -> n = +-1 only
    assert s4[2, 1 + 3] == pytest.approx(1j * math.sqrt(0.5), abs=3e-16)
    assert s4[2, 3 + 3] == 0
    # zero-mean: for N even, s_00 = 0 (N = 4: gamma = -1)
    assert np.all(s4[0] == 0)


def test_wavelet_zero_mean_even_for_odd_N():
    # for odd N, Eq. 11 gives s_00 = 1, but kappa^j(0) = 0 keeps Psi^j_00 = 0
    psi = tables.wavelets(64, 3, 2.0, 0)
    assert np.all(psi[:, 0, :] == 0)
