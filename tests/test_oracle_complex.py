"""Pins of the oracle for complex (non-real) signals, where no symmetry between f_lm and
f_{l,-m} holds and the wavelet coefficients are complex: the defining integral of Eq. 1 by
brute-force quadrature, the closed-form Wigner coefficients of Eq. 21, exact reconstruction
(Sec. 3.4) on the equiangular and Driscoll-Healy grids, and linearity over the real and
imaginary parts of the signal."""
import math

import numpy as np
import pytest

import oracle
from oracle import tables
from paper_1308_5706_amd.inputs import random_flm, random_flm_complex
from test_oracle_transform import expand, rot, to_angles, to_xyz


@pytest.mark.parametrize("N", [2, 3])
def test_complex_signal_against_brute_force_eq1(N):
    L, lam, J_min = 6, 2.0, 0
    f = random_flm_complex(L, 41)
    psi = tables.wavelets(L, N, lam, J_min)
    fc = {el: {m: f[el * el + el + m] for m in range(-el, el + 1)} for el in range(L)}
    nth, nph = 2 * L, 4 * L
    x, w = np.polynomial.legendre.leggauss(nth)
    TH = np.repeat(np.arccos(x), nph).reshape(nth, nph)
    PH = np.tile(2 * math.pi * np.arange(nph) / nph, nth).reshape(nth, nph)
    W8 = np.repeat(w, nph).reshape(nth, nph) * (2 * math.pi / nph)
    fvals = expand(fc, L, TH, PH)
    beta = 2.2
    Wor = oracle.analysis_complex(f, L, N, lam, J_min, betas=[beta], psi=psi)
    assert np.max(np.abs(Wor.imag)) > 1e-3  # genuinely complex
    for a in [0, 5]:
        for gi in [0, 2 * N - 2]:
            alpha = 2 * math.pi * a / (2 * L - 1)
            gamma = 2 * math.pi * gi / (2 * N - 1)
            th2, ph2 = to_angles(to_xyz(TH, PH) @ rot(alpha, beta, gamma))
            for j in range(psi.shape[0]):
                pc = {el: {n: psi[j, el, n + N - 1] for n in range(-(N - 1), N) if abs(n) <= el}
                      for el in range(L)}
                ref = np.sum(W8 * fvals * np.conj(expand(pc, L, th2, ph2)))
                assert abs(Wor[j, gi, 0, a] - ref) < 1e-13


def test_complex_wigner_coefficients_closed_form_eq21():
    L, N, J_min = 10, 3, 0
    f = random_flm_complex(L, 43)
    psi = tables.wavelets(L, N, 2.0, J_min)
    W = oracle.analysis_complex(f, L, N, 2.0, J_min, psi=psi)
    wig = oracle.forward_wigner_mw(W, L, N)
    nl = tables.n_list(N)
    for el in range(L):
        for m in range(-el, el + 1):
            ref = 8 * math.pi ** 2 / (2 * el + 1) * f[el * el + el + m] * np.conj(psi[:, el, [n + N - 1 for n in nl]])
            assert np.max(np.abs(wig[:, el, m + L - 1] - ref)) < 1e-12


@pytest.mark.parametrize("L,N,J_min", [(16, 3, 0), (24, 4, 1), (20, 1, 0)])
def test_complex_exact_reconstruction(L, N, J_min):
    f = random_flm_complex(L, 45)
    W = oracle.analysis_complex(f, L, N, 2.0, J_min)
    fr = oracle.synthesis(W, oracle.scaling(f, L, 2.0, J_min), L, N, 2.0, J_min)
    assert np.max(np.abs(fr - f)) / np.max(np.abs(f)) < 1e-13
    Wd = oracle.analysis_dh(f, L, N, 2.0, J_min)
    frd = oracle.synthesis_dh(Wd, oracle.scaling(f, L, 2.0, J_min), L, N, 2.0, J_min)
    assert np.max(np.abs(frd - f)) / np.max(np.abs(f)) < 1e-13


def test_linearity_over_real_and_imaginary_parts():
    # f = a + i b with a, b real signals gives W(f) = W(a) + i W(b) (Eq. 1 is linear in f)
    L, N = 12, 4
    a, b = random_flm(L, 47), random_flm(L, 48)
    W = oracle.analysis_complex(a + 1j * b, L, N, 2.0, 0)
    Wa = oracle.analysis(a, L, N, 2.0, 0)
    Wb = oracle.analysis(b, L, N, 2.0, 0)
    assert np.max(np.abs(W - (Wa + 1j * Wb))) < 1e-14 * np.max(np.abs(W)) * 10
