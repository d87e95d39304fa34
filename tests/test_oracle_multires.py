"""Pins of the oracle's multiresolution transforms (each scale on the equiangular grid of its
own band-limit, Sec. 3.2 closing remarks): the band-limits follow from the support of the
kernel of Eq. 14-15, the samples of a single harmonic match the closed form of Eq. 20 with
Wigner's explicit d, the per-scale Wigner coefficients match Eq. 21, and the round trip is
exact (Sec. 3.4)."""
import math

import numpy as np
import pytest

import oracle
from oracle import tables
from paper_1308_5706_amd.inputs import random_flm
from test_oracle_wigner import explicit_d


@pytest.mark.parametrize("L,lam,J_min", [(64, 2.0, 0), (1024, 2.0, 1), (27, 3.0, 0), (100, 1.7, 1), (48, 2.0, 2)])
def test_band_limits_follow_the_kernel_support(L, lam, J_min):
    # kappa^j(l) = kappa_lambda(lambda^j l / L) vanishes unless lambda^j l / L < lambda (Eq. 14-15):
    # the band-limit of scale j is min(L, ceil(L lambda^(1-j)))
    bl = oracle.scale_bandlimits(L, lam, J_min)
    J = tables.j_max(L, lam) - J_min
    assert len(bl) == J + 1
    for j, Lj in enumerate(bl):
        x = L * lam ** (1 - j)
        assert Lj == min(L, math.ceil(x - 1e-9)), (j, Lj, x)


def test_single_harmonic_on_the_scale_grids():
    # f = delta_{l0 m0}: W^j(a, b, g) = sum_n conj(Psi^j_{l0 n}) e^{i m0 a} d^{l0}_{m0 n}(b) e^{i n g}
    L, N, lam = 16, 3, 2.0
    l0, m0 = 6, 3
    f = np.zeros(L * L, dtype=complex)
    f[l0 * l0 + l0 + m0] = 1.0
    f[l0 * l0 + l0 - m0] = (-1) ** m0  # real signal
    psi = tables.wavelets(L, N, lam, 0)
    Ws = oracle.analysis_multires(f, L, N, lam, 0, psi=psi)
    for j, Lj in enumerate(oracle.scale_bandlimits(L, lam, 0)):
        assert Ws[j].shape == (2 * N - 1, Lj, 2 * Lj - 1)
        for b in sorted({0, Lj // 2, Lj - 1}):
            for a in sorted({0, 2 * Lj - 2}):
                for g in range(2 * N - 1):
                    be = math.pi * (2 * b + 1) / (2 * Lj - 1)
                    al, ga = 2 * math.pi * a / (2 * Lj - 1), 2 * math.pi * g / (2 * N - 1)
                    ref = 0.0
                    for mm, c in [(m0, 1.0), (-m0, (-1) ** m0)]:
                        ref += sum(c * np.conj(psi[j, l0, n + N - 1]) * np.exp(1j * mm * al)
                                   * float(explicit_d(l0, mm, n, be)) * np.exp(1j * n * ga)
                                   for n in range(-(N - 1), N))
                    assert abs(Ws[j][g, b, a] - ref.real) < 1e-14


@pytest.mark.parametrize("L,N,J_min", [(16, 3, 0), (24, 4, 1), (20, 8, 0)])
def test_scale_wigner_coefficients_closed_form_eq21(L, N, J_min):
    lam = 2.0
    f = random_flm(L, 31)
    psi = tables.wavelets(L, N, lam, J_min)
    Ws = oracle.analysis_multires(f, L, N, lam, J_min, psi=psi)
    nl = tables.n_list(N)
    for j, Lj in enumerate(oracle.scale_bandlimits(L, lam, J_min)):
        wig = oracle.forward_wigner_mw(Ws[j][None], Lj, N)[0]
        for el in range(Lj):
            for m in range(-el, el + 1):
                ref = 8 * math.pi ** 2 / (2 * el + 1) * f[el * el + el + m] * np.conj(psi[j, el, [n + N - 1 for n in nl]])
                assert np.max(np.abs(wig[el, m + Lj - 1] - ref)) < 1e-12


@pytest.mark.parametrize("L,N,J_min,lam", [(32, 4, 0, 2.0), (40, 8, 1, 2.0), (27, 3, 0, 3.0), (30, 2, 1, 1.7)])
def test_multires_exact_reconstruction(L, N, J_min, lam):
    f = random_flm(L, 33)
    Ws = oracle.analysis_multires(f, L, N, lam, J_min)
    fr = oracle.synthesis_multires(Ws, oracle.scaling(f, L, lam, J_min), L, N, lam, J_min)
    assert np.max(np.abs(fr - f)) / np.max(np.abs(f)) < 1e-13
