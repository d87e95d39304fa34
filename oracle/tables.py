"""Harmonic-space tables of the scale-discretized wavelets (Sec. 2.2, Eq. 7-16).

TEST INFRASTRUCTURE ONLY: part of the CPU reference ("oracle") that the GPU
library is checked against.  It shares no code with the GPU library.

Everything here follows the printed definitions one to one:
  s(t), s_lambda(t)            Eq. 12
  k_lambda(t)                  Eq. 13, both integrals by adaptive Gauss-Kronrod
  kappa_lambda(t)              Eq. 14 (the difference of Eq. 13 taken as one integral)
  kappa^j(l)                   Eq. 15
  J_L(lambda)                  the smallest integer J with lambda^{-J} L <= 1
  Phi_{l0}                     Eq. 16
  s_{ln} (directionality)      Eq. 11
  Psi^j_{ln} = kappa^j(l) s_ln Eq. 7
Scale j = 0 is the highest-frequency wavelet (footnote to Eq. 15); the number
of wavelet scales kept is J + 1 with J = J_L(lambda) - J_min.
"""
from __future__ import annotations

import functools
import math
import warnings

import numpy as np
from scipy import integrate


def schwartz(t: float) -> float:
    """s(t) = exp(-(1 - t^2)^-1) on (-1, 1), zero elsewhere (Eq. 12)."""
    if -1.0 < t < 1.0:
        return math.exp(-1.0 / (1.0 - t * t))
    return 0.0


def s_lambda(t: float, lam: float) -> float:
    """s_lambda(t) = s(2 lambda/(lambda - 1) (t - 1/lambda) - 1) (Eq. 12)."""
    return schwartz(2.0 * lam / (lam - 1.0) * (t - 1.0 / lam) - 1.0)


def _integrand(u: float, lam: float) -> float:
    return s_lambda(u, lam) ** 2 / u


def _quad(a: float, b: float, lam: float) -> float:
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        val, _err = integrate.quad(_integrand, a, b, args=(lam,), epsabs=0.0,
                                   epsrel=1e-13, limit=400)
    return val


@functools.lru_cache(maxsize=None)
def _k_denominator(lam: float) -> float:
    return _quad(1.0 / lam, 1.0, lam)


def k_lambda(t: float, lam: float) -> float:
    """k_lambda(t) (Eq. 13): 1 for t <= 1/lambda, 0 for t >= 1, else the ratio of integrals."""
    if t <= 1.0 / lam:
        return 1.0
    if t >= 1.0:
        return 0.0
    return _quad(t, 1.0, lam) / _k_denominator(lam)


def kappa_lambda(t: float, lam: float) -> float:
    """kappa_lambda(t) = sqrt(k_lambda(t/lambda) - k_lambda(t)) (Eq. 14).

    Both terms of the difference are the same integral of Eq. 13 with the same upper
    limit, so the difference is that integral over [t/lambda, t], clipped to the
    support [1/lambda, 1] of s_lambda.  It is evaluated as one integral: subtracting
    two values close to 1 would leave kappa with an absolute error of ~1e-8 (the square
    root of the rounding error) near the ends of its support."""
    a = max(t / lam, 1.0 / lam)
    b = min(t, 1.0)
    if not b > a:
        return 0.0
    v = _quad(a, b, lam) / _k_denominator(lam)
    return math.sqrt(v) if v > 0.0 else 0.0


def j_max(L: int, lam: float) -> int:
    """J_L(lambda): the lowest integer J with lambda^{-J} L <= 1 (Sec. 2.2)."""
    J = 0
    while lam ** J < L:
        J += 1
    return J


def num_scales(L: int, lam: float, J_min: int) -> int:
    """Wavelet scales j = 0..J with J = J_L(lambda) - J_min."""
    return j_max(L, lam) - J_min + 1


def kappa_table(L: int, lam: float, J_min: int) -> np.ndarray:
    """kappa^j(l) = kappa_lambda(lambda^j l / L) (Eq. 15), shape [J+1, L]."""
    J = j_max(L, lam) - J_min
    out = np.zeros((J + 1, L))
    for j in range(J + 1):
        for el in range(L):
            out[j, el] = kappa_lambda(lam ** j * el / L, lam)
    return out


def phi_table(L: int, lam: float, J_min: int) -> np.ndarray:
    """Phi_{l0} = sqrt(k_lambda(lambda^J l / L)) (Eq. 16), shape [L]."""
    J = j_max(L, lam) - J_min
    return np.array([math.sqrt(k_lambda(lam ** J * el / L, lam)) for el in range(L)])


def n_list(N: int) -> list[int]:
    """The n carried by the directionality component: |n| < N and beta_(N,n) = 1 (Eq. 11)."""
    return [n for n in range(-(N - 1), N) if (N + n) % 2 == 1]


def directionality(L: int, N: int) -> np.ndarray:
    """s_{ln} of Eq. 11, shape [L, 2N-1] indexed by n + N - 1 (complex)."""
    eta = 1.0 if (N - 1) % 2 == 0 else 1j
    out = np.zeros((L, 2 * N - 1), dtype=complex)
    for el in range(L):
        gam = min(N - 1, el - (1 + (-1) ** (N + el)) // 2)
        for n in range(-(N - 1), N):
            beta = (1 - (-1) ** (N + n)) // 2
            if beta == 0 or gam < 0 or abs(n) > gam or (gam - n) % 2:
                continue
            out[el, n + N - 1] = eta * math.sqrt(math.comb(gam, (gam - n) // 2) / 2.0 ** gam)
    return out


def wavelets(L: int, N: int, lam: float, J_min: int) -> np.ndarray:
    """Psi^j_{ln} = kappa^j(l) s_{ln} (Eq. 7), shape [J+1, L, 2N-1]."""
    kap = kappa_table(L, lam, J_min)
    s = directionality(L, N)
    return kap[:, :, None] * s[None, :, :]
