"""Pins of the oracle's Wigner small-d functions (Eq. 24, 25) against Wigner's
explicit sum in 40-digit arithmetic, scipy's spherical harmonics, unitarity at
large l, the closed forms of Delta = d(pi/2) and the Fourier factorisation
of Eq. 25 that the fast algorithms rest on."""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle


def explicit_d(el, m, n, beta, dps=40):
    """Wigner's explicit sum for d^l_{mn}(beta) = <l m|exp(-i beta J_y)|l n>."""
    mpmath.mp.dps = dps
    b = mpmath.mpf(beta)
    c, s = mpmath.cos(b / 2), mpmath.sin(b / 2)
    f = mpmath.factorial
    pre = mpmath.sqrt(f(el + m) * f(el - m) * f(el + n) * f(el - n))
    tot = mpmath.mpf(0)
    for k in range(0, 2 * el + 1):
        a1, a2, a3, a4 = el + n - k, k, m - n + k, el - m - k
        if min(a1, a2, a3, a4) < 0:
            continue
        term = pre / (f(a1) * f(a2) * f(a3) * f(a4))
        term *= c ** (2 * el + n - m - 2 * k) * s ** (m - n + 2 * k)
        tot += (-1) ** (m - n + k) * term
    return tot


BETAS = [0.0371, 0.7, math.pi / 2, 2.2, math.pi - 0.013, math.pi * 31 / 63]


@pytest.mark.parametrize("beta", BETAS)
def test_small_l_against_explicit_sum(beta):
    L = 13
    worst = 0.0
    for m in range(-(L - 1), L):
        for n in range(-(L - 1), L):
            d = oracle.wigner_d(L, m, n, beta)
            for el in range(L):
                ref = float(explicit_d(el, m, n, beta)) if el >= max(abs(m), abs(n)) else 0.0
                worst = max(worst, abs(d[el] - ref))
    assert worst < 1e-15


def test_first_order_values():
    # d^1_{10}(beta) = -sin(beta)/sqrt(2), d^1_{00} = cos(beta), d^1_{11} = (1+cos beta)/2
    b = 0.83
    assert oracle.wigner_d(2, 1, 0, b)[1] == pytest.approx(-math.sin(b) / math.sqrt(2), abs=1e-16)
    assert oracle.wigner_d(2, 0, 0, b)[1] == pytest.approx(math.cos(b), abs=1e-16)
    assert oracle.wigner_d(2, 1, 1, b)[1] == pytest.approx((1 + math.cos(b)) / 2, abs=1e-16)
    assert oracle.wigner_d(2, 0, 1, b)[1] == pytest.approx(math.sin(b) / math.sqrt(2), abs=1e-16)


@pytest.mark.parametrize("el,m,n,beta", [(40, 17, -5, 1.1), (64, 63, 2, 0.4), (64, -30, 30, 2.9),
                                         (100, 3, 7, math.pi / 2)])
def test_moderate_l_against_explicit_sum(el, m, n, beta):
    # high working precision makes the alternating explicit sum usable here
    ref = float(explicit_d(el, m, n, beta, dps=120))
    d = oracle.wigner_d(el + 1, m, n, beta)[el]
    assert abs(d - ref) < 2e-15


@pytest.mark.parametrize("el", [1, 5, 17, 60, 150])
def test_m0_column_against_scipy_harmonics(el):
    # Y_lm(theta, phi) = sqrt((2l+1)/(4 pi)) e^{i m phi} d^l_{m0}(theta) (Condon-Shortley)
    th = 1.234
    norm = math.sqrt((2 * el + 1) / (4 * math.pi))
    for m in range(-el, el + 1, max(1, el // 7)):
        y = sph_harm_y(el, m, th, 0.0).real
        d = oracle.wigner_d(el + 1, m, 0, th)[el]
        assert abs(norm * d - y) < 1e-13 * max(1.0, norm)


@pytest.mark.parametrize("L", [1024, 2048])
@pytest.mark.parametrize("beta", [0.3, math.pi / 2, math.pi * (2 * 700 + 1) / (2 * 2048 - 1)])
def test_unitarity_at_large_l(L, beta):
    # the columns of d^l(beta) are orthonormal: sum_m d_mn d_mn' = delta_nn'
    el = L - 1
    cols = {}
    for n in (0, 3, 1100 if L > 1100 else 700):
        cols[n] = np.array([oracle.wigner_d(L, m, n, beta)[el] for m in range(-el, el + 1)])
    for n, c in cols.items():
        assert abs(np.dot(c, c) - 1.0) < 1e-12
    assert abs(np.dot(cols[0], cols[3])) < 1e-12


def test_delta_closed_forms():
    # Delta^l_{ll} = 2^-l ; Delta^l_{l0} = (-1)^l sqrt((2l)!)/(2^l l!)
    mpmath.mp.dps = 30
    for el in [1, 7, 100, 500, 1000]:
        hi, lo = oracle.wigner_d_ext(el + 1, el, el, math.pi / 2)
        assert (hi[el] + lo[el]) == pytest.approx(2.0 ** (-el), rel=1e-15)
        ref = (-1) ** el * mpmath.sqrt(mpmath.factorial(2 * el)) / (2 ** el * mpmath.factorial(el))
        d0 = oracle.wigner_d(el + 1, el, 0, math.pi / 2)[el]
        assert d0 == pytest.approx(float(ref), rel=1e-14)


def test_delta_underflow_regime_keeps_digits():
    # edge values 2^-l0 with l0 > 1022 are below double range; the extended exponent keeps them,
    # and unitarity of the whole column at l = 2047 proves the recurrence recovered them
    L = 2048
    el = L - 1
    n = 1300
    col = np.array([oracle.wigner_d(L, m, n, math.pi / 2)[el] for m in range(-el, el + 1)])
    assert abs(np.dot(col, col) - 1.0) < 1e-12
    assert abs(oracle.wigner_d(L, 1300, 1300, math.pi / 2)[el]) > 1e-6


def test_symmetries():
    L, b = 30, 0.91
    for m in range(-5, 6):
        for n in range(-4, 5):
            d = oracle.wigner_d(L, m, n, b)
            assert np.allclose(d, (-1) ** (m - n) * oracle.wigner_d(L, n, m, b), atol=1e-15)
            assert np.allclose(d, oracle.wigner_d(L, -n, -m, b), atol=1e-15)
    # Delta_{-m',m} = (-1)^{l+m} Delta_{m'm} (used to fold m' in the fast algorithms)
    el = np.arange(L)
    for mp in range(0, 8):
        for m in range(-6, 7):
            a = oracle.wigner_d(L, -mp, m, math.pi / 2)
            bb = oracle.wigner_d(L, mp, m, math.pi / 2)
            assert np.allclose(a, (-1.0) ** (el + m) * bb, atol=1e-15)


@pytest.mark.parametrize("el", [6, 25])
def test_fourier_factorisation_eq25(el):
    # d^l_mn(beta) = e^{-i(n-m) pi/2} sum_{m'} Delta_{m'm} Delta_{m'n} e^{-i m' beta}   (Eq. 25)
    beta = 1.37
    L = el + 1
    delta = np.zeros((2 * el + 1, 2 * el + 1))
    for mp in range(-el, el + 1):
        for m in range(-el, el + 1):
            delta[mp + el, m + el] = oracle.wigner_d(L, mp, m, math.pi / 2)[el]
    mps = np.arange(-el, el + 1)
    for m in range(-el, el + 1, 3):
        for n in range(-el, el + 1, 4):
            val = np.exp(-1j * (n - m) * math.pi / 2) * np.sum(
                delta[:, m + el] * delta[:, n + el] * np.exp(-1j * mps * beta))
            assert abs(val.imag) < 1e-14
            assert abs(val.real - oracle.wigner_d(L, m, n, beta)[el]) < 1e-14
