"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers in the shape of the paper's workloads;
it holds none of the transform's arithmetic and imports neither the GPU
binding nor the CPU reference.

Signals are band-limited harmonic coefficients f_lm (index l*l + l + m) of a
real signal on the sphere: for l < L and 0 <= m <= l a complex Gaussian with
variance C_l = 1/(l+1)^2 (real and imaginary parts each of variance C_l/2),
the imaginary part of f_l0 set to zero, and f_{l,-m} = (-1)^m conj(f_lm).
Complex (non-real) signals draw every m in -l..l independently with the same variance.
"""
from __future__ import annotations

import numpy as np


def random_flm(L: int, seed: int) -> np.ndarray:
    """Complex128 [L*L] coefficients of a real band-limited signal."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros(L * L, dtype=np.complex128)
    for el in range(L):
        sd = np.sqrt(1.0 / (el + 1) ** 2 / 2.0)
        x = rng.standard_normal(el + 1) * sd
        y = rng.standard_normal(el + 1) * sd
        y[0] = 0.0
        z = x + 1j * y
        base = el * el + el
        f[base: base + el + 1] = z
        m = np.arange(1, el + 1)
        f[base - m] = ((-1.0) ** m) * np.conj(z[1:])
    return f


def random_flm_uniform(L: int, seed: int) -> np.ndarray:
    """The paper's test signal (Sec. 3.4): real and imaginary parts uniform in [-1, 1],
    made real-signal symmetric in the same way."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros(L * L, dtype=np.complex128)
    for el in range(L):
        z = rng.uniform(-1.0, 1.0, el + 1) + 1j * rng.uniform(-1.0, 1.0, el + 1)
        z[0] = z[0].real
        base = el * el + el
        f[base: base + el + 1] = z
        m = np.arange(1, el + 1)
        f[base - m] = ((-1.0) ** m) * np.conj(z[1:])
    return f


def random_flm_complex(L: int, seed: int) -> np.ndarray:
    """Complex128 [L*L] coefficients of a complex band-limited signal (no symmetry)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros(L * L, dtype=np.complex128)
    for el in range(L):
        sd = np.sqrt(1.0 / (el + 1) ** 2 / 2.0)
        n = 2 * el + 1
        f[el * el: el * el + n] = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * sd
    return f


def random_wavelet_samples_complex(S: int, ng: int, nb: int, na: int, seed: int) -> np.ndarray:
    """Arbitrary complex samples on the SO(3) grid, [S][ng][nb][na]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((S, ng, nb, na)) + 1j * rng.standard_normal((S, ng, nb, na))


def random_real_map(nb: int, na: int, seed: int) -> np.ndarray:
    """Arbitrary (not band-limited) real samples, [nb][na]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((nb, na))


def random_wavelet_samples(S: int, ng: int, nb: int, na: int, seed: int) -> np.ndarray:
    """Arbitrary real samples on the SO(3) grid, [S][ng][nb][na]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((S, ng, nb, na))
