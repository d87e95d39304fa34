"""CPU reference ("oracle") for the directional scale-discretized wavelet
transform on the sphere (McEwen, Vandergheynst & Wiaux, SPIE 2013).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference the GPU
library is checked against.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it.  It shares no code with
the GPU library, and the GPU library never calls it.

Layout conventions (the same ones the library's C ABI documents):
  * f_lm: complex [L*L], index l*l + l + m.
  * Wavelet coefficients on the equiangular grid: real [S][2N-1][L][2L-1]
    = [scale j][gamma_g][beta_b][alpha_a], alpha_a = 2 pi a/(2L-1),
    beta_b = pi(2b+1)/(2L-1), gamma_g = 2 pi g/(2N-1).  Scale j = 0 is the
    highest-frequency wavelet.
  * Scaling coefficients: complex harmonic W^Phi_lm, [L*L] (Eq. 31).
  * Complex (non-real) signals: every sum runs over all m and n as written, so
    ``analysis_complex`` gives their complex coefficients and the synthesis
    functions accept complex samples.

Synthesis of samples that are not band-limited: the beta integral is taken of the
unique trigonometric polynomial of degree < L through the samples extended to the
full circle with the parity (-1)^{m+n}; that polynomial times d^l_mn is a polynomial
in cos(beta) only when the extension is consistent at beta = pi, so the integral is
evaluated with a converged Gauss-Legendre rule in beta itself (``beta_rule``).

Functions whose result has a plain definition evaluate it as written
(analysis: Eq. 20 with Eq. 24; scaling: Eq. 31; synthesis: Eq. 32, 33 and
41 with exact quadratures).  See ``orc.c`` for the numerical details.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import tables

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile orc.c into liborc.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "orc.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def _nthreads() -> int:
    return int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _cplx(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


# --------------------------------------------------------------------------- grids

def mw_betas(L: int) -> np.ndarray:
    """beta_b = pi (2b+1)/(2L-1), b < L: the equiangular colatitudes (includes beta = pi)."""
    return np.pi * (2.0 * np.arange(L) + 1.0) / (2.0 * L - 1.0)


def dh_betas(L: int) -> np.ndarray:
    """theta_t = pi (2t+1)/(4L), t < 2L (Sec. 3.1)."""
    return np.pi * (2.0 * np.arange(2 * L) + 1.0) / (4.0 * L)


def beta_rule(L: int) -> tuple[np.ndarray, np.ndarray]:
    """Nodes in [0, pi] and weights (times sin(beta)) of the Gauss-Legendre rule in beta used
    to integrate sin(beta) G(beta) d^l_mn(beta), G a trigonometric polynomial of degree < L:
    4L+16 nodes put the quadrature error of this entire integrand below e^(-5L)."""
    x, w = np.polynomial.legendre.leggauss(4 * L + 16)
    b = 0.5 * np.pi * (x + 1.0)
    return np.ascontiguousarray(b), np.ascontiguousarray(0.5 * np.pi * w * np.sin(b))


def dh_weights(L: int) -> np.ndarray:
    """q(theta_t) = (2/L) sin(theta_t) sum_{k<L} sin((2k+1) theta_t)/(2k+1) (Eq. 18)."""
    th = dh_betas(L)
    k = np.arange(L)
    return (2.0 / L) * np.sin(th) * (np.sin(np.outer(th, 2 * k + 1)) / (2 * k + 1)).sum(axis=1)


# --------------------------------------------------------------------------- Wigner d

def wigner_d(L: int, m: int, n: int, beta: float) -> np.ndarray:
    """d^l_{mn}(beta) for l < L (zero below max(|m|,|n|)); Eq. 24 convention."""
    out = np.zeros(L)
    _load().orc_wigner_d(ctypes.c_int(L), ctypes.c_int(m), ctypes.c_int(n), ctypes.c_double(beta), _dp(out))
    return out


def wigner_d_ext(L: int, m: int, n: int, beta: float) -> tuple[np.ndarray, np.ndarray]:
    """As wigner_d, with the long-double values split as hi + lo."""
    hi = np.zeros(L)
    lo = np.zeros(L)
    _load().orc_wigner_d_ext(ctypes.c_int(L), ctypes.c_int(m), ctypes.c_int(n), ctypes.c_double(beta),
                             _dp(hi), _dp(lo))
    return hi, lo


# --------------------------------------------------------------------------- transforms

def _analysis_raw(flm, psi_sel, nl, L, betas, na, ng, mg):
    S = psi_sel.shape[0]
    f = _cplx(flm).view(np.float64)
    p = _cplx(psi_sel).view(np.float64)
    nla = np.ascontiguousarray(np.array(nl, dtype=np.int32))
    be = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
    out = np.zeros((S, ng, len(be), na), dtype=np.complex128)
    rc = _load().orc_analysis(ctypes.c_int(L), ctypes.c_int(len(nl)), _ip(nla), ctypes.c_int(S), _dp(f), _dp(p),
                              ctypes.c_int(len(be)), _dp(be), ctypes.c_int(na), ctypes.c_int(ng),
                              ctypes.c_int(mg), _dp(out.view(np.float64)), ctypes.c_int(_nthreads()))
    if rc != 0:
        raise MemoryError("oracle analysis failed")
    return out


def _psi_cols(psi: np.ndarray, N: int) -> tuple[np.ndarray, list[int]]:
    nl = tables.n_list(N)
    cols = [n + N - 1 for n in nl]
    return np.ascontiguousarray(psi[:, :, cols]), nl


def analysis_complex(flm, L: int, N: int, lam: float, J_min: int, betas=None, psi=None) -> np.ndarray:
    """W^j(alpha_a, beta_b, gamma_g) by Eq. 20, complex [S][2N-1][nb][2L-1].

    betas: the colatitudes to evaluate (default: the L equiangular ones)."""
    if psi is None:
        psi = tables.wavelets(L, N, lam, J_min)
    ps, nl = _psi_cols(psi, N)
    if betas is None:
        betas = mw_betas(L)
    return _analysis_raw(flm, ps, nl, L, betas, 2 * L - 1, 2 * N - 1, 2 * N - 1)


def analysis(flm, L: int, N: int, lam: float, J_min: int, betas=None, psi=None) -> np.ndarray:
    """Real wavelet coefficients of a real signal, [S][2N-1][nb][2L-1] (Eq. 20)."""
    return analysis_complex(flm, L, N, lam, J_min, betas=betas, psi=psi).real


def analysis_at_complex(flm, L: int, N: int, lam: float, J_min: int, gammas, betas=None,
                        psi=None, nalpha=None) -> np.ndarray:
    """W^j(alpha_a, beta_b, gamma) by Eq. 20 at arbitrary third Euler angles gamma, complex
    [S][len(gammas)][nb][na], alpha_a = 2 pi a/na (na = nalpha, default 2L-1).

    Eq. 20 is a sum over the carried orders n of e^{i n gamma} times a function of (alpha,
    beta) alone; each of those terms is evaluated at gamma = 0 (Eq. 20 with the single order
    n) and the factor e^{i n gamma} is applied here, for every gamma asked."""
    if psi is None:
        psi = tables.wavelets(L, N, lam, J_min)
    ps, nl = _psi_cols(psi, N)
    if betas is None:
        betas = mw_betas(L)
    gammas = np.asarray(gammas, dtype=np.float64).reshape(-1)
    out = None
    for i, n in enumerate(nl):
        h = _analysis_raw(flm, np.ascontiguousarray(ps[:, :, i:i + 1]), [n], L, betas,
                          nalpha or 2 * L - 1, 1, 1)[:, 0]
        t = np.exp(1j * n * gammas)[None, :, None, None] * h[:, None]
        out = t if out is None else out + t
    return out


def analysis_at(flm, L: int, N: int, lam: float, J_min: int, gammas, betas=None, psi=None,
                nalpha=None) -> np.ndarray:
    """Real wavelet coefficients of a real signal at arbitrary gamma, [S][len(gammas)][nb][na]
    (Eq. 20)."""
    return analysis_at_complex(flm, L, N, lam, J_min, gammas, betas=betas, psi=psi, nalpha=nalpha).real


def scale_bandlimits(L: int, lam: float, J_min: int) -> list[int]:
    """Band-limit of each wavelet scale: one more than the largest l with kappa^j(l) > 0
    (0 for a scale with no support).  The wavelet transform of scale j needs no grid finer
    than this band-limit (Sec. 3.2, closing remarks on the compact support of the wavelets)."""
    kap = tables.kappa_table(L, lam, J_min)
    out = []
    for j in range(kap.shape[0]):
        nz = np.nonzero(kap[j] > 0.0)[0]
        out.append(int(nz[-1]) + 1 if len(nz) else 0)
    return out


def analysis_multires(flm, L: int, N: int, lam: float, J_min: int, psi=None) -> list[np.ndarray]:
    """Multiresolution wavelet coefficients: W^j by Eq. 20 on the equiangular grid of the
    scale's own band-limit Lj (alpha 2Lj-1, beta Lj, gamma 2N-1 samples), real
    [2N-1][Lj][2Lj-1] per scale j."""
    if psi is None:
        psi = tables.wavelets(L, N, lam, J_min)
    ps, nl = _psi_cols(psi, N)
    out = []
    for j, Lj in enumerate(scale_bandlimits(L, lam, J_min)):
        if Lj == 0:
            out.append(np.zeros((2 * N - 1, 0, 0)))
            continue
        w = _analysis_raw(flm, np.ascontiguousarray(ps[j:j + 1]), nl, L, mw_betas(Lj), 2 * Lj - 1, 2 * N - 1,
                          2 * N - 1)
        out.append(w[0].real)
    return out


def synthesis_multires(Ws, Wphi, L: int, N: int, lam: float, J_min: int, psi=None, phi=None) -> np.ndarray:
    """Exact synthesis from multiresolution coefficients: each scale's Wigner coefficients
    (Eq. 23) by the quadratures of its own band-limit-Lj grid (zero for l >= Lj, where
    kappa^j vanishes), then Eq. 32 and Eq. 41."""
    bl = scale_bandlimits(L, lam, J_min)
    nn = len(tables.n_list(N))
    wig = np.zeros((len(bl), L, 2 * L - 1, nn), dtype=np.complex128)
    for j, Lj in enumerate(bl):
        if Lj == 0:
            continue
        wj = forward_wigner_mw(np.asarray(Ws[j])[None], Lj, N)[0]
        wig[j, :Lj, L - Lj:L + Lj - 1, :] = wj
    return synthesis_from_wigner(wig, Wphi, L, N, lam, J_min, psi=psi, phi=phi)


def scaling(flm, L: int, lam: float, J_min: int, phi=None) -> np.ndarray:
    """W^Phi_lm = sqrt(4 pi/(2l+1)) f_lm conj(Phi_l0) (Eq. 31), complex [L*L]."""
    if phi is None:
        phi = tables.phi_table(L, lam, J_min)
    f = _cplx(flm)
    out = np.zeros(L * L, dtype=np.complex128)
    for el in range(L):
        sl = slice(el * el, el * el + 2 * el + 1)
        out[sl] = math.sqrt(4.0 * math.pi / (2 * el + 1)) * f[sl] * np.conj(phi[el])
    return out


def inverse_wigner(c: np.ndarray, L: int, nl: list[int], betas, na: int, ng: int, mg: int) -> np.ndarray:
    """g(rho) = sum_{lmn} c[s][l][m+L-1][ni] e^{i m alpha} d^l_mn(beta) e^{i n gamma}; complex [S][ng][nb][na]."""
    c = _cplx(c)
    S = c.shape[0]
    nla = np.ascontiguousarray(np.array(nl, dtype=np.int32))
    be = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
    out = np.zeros((S, ng, len(be), na), dtype=np.complex128)
    rc = _load().orc_inverse_wigner(ctypes.c_int(L), ctypes.c_int(len(nl)), _ip(nla), ctypes.c_int(S),
                                    _dp(c.view(np.float64)), ctypes.c_int(len(be)), _dp(be), ctypes.c_int(na),
                                    ctypes.c_int(ng), ctypes.c_int(mg), _dp(out.view(np.float64)),
                                    ctypes.c_int(_nthreads()))
    if rc != 0:
        raise MemoryError("oracle inverse Wigner failed")
    return out


def forward_wigner_mw(W, L: int, N: int, m_range=None) -> np.ndarray:
    """Wigner coefficients int W D^l_mn (Eq. 23) of samples on the equiangular grid.

    W: [S][2N-1][L][2L-1] (real or complex).  Returns complex [S][L][2L-1][len(n_list(N))];
    with m_range=(lo, hi) only those m columns are computed (others zero)."""
    W = _cplx(W)
    S = W.shape[0]
    nl = tables.n_list(N)
    nla = np.ascontiguousarray(np.array(nl, dtype=np.int32))
    xg, wg = beta_rule(L)
    lo, hi = (-(L - 1), L - 1) if m_range is None else m_range
    out = np.zeros((S, L, 2 * L - 1, len(nl)), dtype=np.complex128)
    rc = _load().orc_forward_wigner_mw(ctypes.c_int(L), ctypes.c_int(len(nl)), _ip(nla), ctypes.c_int(S),
                                       _dp(W.view(np.float64)), ctypes.c_int(2 * L - 1), ctypes.c_int(2 * N - 1),
                                       ctypes.c_int(2 * N - 1), ctypes.c_int(len(xg)), _dp(xg), _dp(wg),
                                       ctypes.c_int(lo), ctypes.c_int(hi), _dp(out.view(np.float64)),
                                       ctypes.c_int(_nthreads()))
    if rc != 0:
        raise MemoryError("oracle forward Wigner failed")
    return out


def alpha_gamma_rules_mw(W, L: int, N: int) -> np.ndarray:
    """First step of forward_wigner_mw for the given rows: W [S][2N-1][nb][2L-1] ->
    complex [S][len(n_list)][nb][2L-1] (Eq. 19 and its gamma analogue)."""
    W = _cplx(W)
    S, _, nb, _ = W.shape
    nl = tables.n_list(N)
    nla = np.ascontiguousarray(np.array(nl, dtype=np.int32))
    out = np.zeros((S, len(nl), nb, 2 * L - 1), dtype=np.complex128)
    rc = _load().orc_alpha_gamma_rules_mw(ctypes.c_int(L), ctypes.c_int(len(nl)), _ip(nla), ctypes.c_int(S),
                                          _dp(W.view(np.float64)), ctypes.c_int(nb), ctypes.c_int(2 * L - 1),
                                          ctypes.c_int(2 * N - 1), ctypes.c_int(2 * N - 1),
                                          _dp(out.view(np.float64)), ctypes.c_int(_nthreads()))
    if rc != 0:
        raise MemoryError("oracle alpha/gamma rules failed")
    return out


def beta_wigner_mw(Gt, L: int, N: int, m_range=None, cols=None) -> np.ndarray:
    """Second step of forward_wigner_mw: Gt [S][len(n_list)][L][2L-1] -> Wigner coefficients of
    the columns m in m_range = (lo, hi), or of the listed columns `cols` (complex
    [S][L][2L-1][len(n_list)], others zero)."""
    Gt = _cplx(Gt)
    S = Gt.shape[0]
    nl = tables.n_list(N)
    nla = np.ascontiguousarray(np.array(nl, dtype=np.int32))
    xg, wg = beta_rule(L)
    out = np.zeros((S, L, 2 * L - 1, len(nl)), dtype=np.complex128)
    if cols is not None:
        ca = np.ascontiguousarray(np.array(cols, dtype=np.int32))
        rc = _load().orc_beta_wigner_mw_cols(ctypes.c_int(L), ctypes.c_int(len(nl)), _ip(nla), ctypes.c_int(S),
                                             _dp(Gt.view(np.float64)), ctypes.c_int(len(xg)), _dp(xg), _dp(wg),
                                             ctypes.c_int(len(ca)), _ip(ca), _dp(out.view(np.float64)),
                                             ctypes.c_int(_nthreads()))
    else:
        rc = _load().orc_beta_wigner_mw(ctypes.c_int(L), ctypes.c_int(len(nl)), _ip(nla), ctypes.c_int(S),
                                        _dp(Gt.view(np.float64)), ctypes.c_int(len(xg)), _dp(xg), _dp(wg),
                                        ctypes.c_int(m_range[0]), ctypes.c_int(m_range[1]),
                                        _dp(out.view(np.float64)), ctypes.c_int(_nthreads()))
    if rc != 0:
        raise MemoryError("oracle beta/Wigner step failed")
    return out


def forward_wigner_dh(W, L: int, N: int) -> np.ndarray:
    """As forward_wigner_mw on the Driscoll-Healy discretisation of Sec. 3.1:
    W [S][N][2L][2L-1] with gamma_g = pi g/N; q weights (Eq. 18), z_n = 1/N (Eq. 39)."""
    W = _cplx(W)
    S = W.shape[0]
    nl = tables.n_list(N)
    nla = np.ascontiguousarray(np.array(nl, dtype=np.int32))
    zw = np.full(len(nl), 1.0 / N)
    qw = np.ascontiguousarray(dh_weights(L))
    out = np.zeros((S, L, 2 * L - 1, len(nl)), dtype=np.complex128)
    rc = _load().orc_forward_wigner_dh(ctypes.c_int(L), ctypes.c_int(len(nl)), _ip(nla), ctypes.c_int(S),
                                       _dp(W.view(np.float64)), ctypes.c_int(2 * L - 1), ctypes.c_int(N),
                                       ctypes.c_int(2 * N), _dp(zw), _dp(qw), _dp(out.view(np.float64)),
                                       ctypes.c_int(_nthreads()))
    if rc != 0:
        raise MemoryError("oracle forward Wigner (DH) failed")
    return out


def analysis_dh(flm, L: int, N: int, lam: float, J_min: int, psi=None) -> np.ndarray:
    """Eq. 20 on the Driscoll-Healy grid of Sec. 3.1: [S][N][2L][2L-1], gamma_g = pi g/N."""
    if psi is None:
        psi = tables.wavelets(L, N, lam, J_min)
    ps, nl = _psi_cols(psi, N)
    return _analysis_raw(flm, ps, nl, L, dh_betas(L), 2 * L - 1, N, 2 * N)


def synthesis_from_wigner(wig: np.ndarray, Wphi, L: int, N: int, lam: float, J_min: int,
                          psi=None, phi=None) -> np.ndarray:
    """f_lm = sum_j sum_n (2l+1)/(8 pi^2) (W^j)^l_mn Psi^j_ln  +  sqrt((2l+1)/(4 pi)) W^Phi_lm Phi_l0
    (Eq. 32 and Eq. 41), complex [L*L]."""
    if psi is None:
        psi = tables.wavelets(L, N, lam, J_min)
    if phi is None:
        phi = tables.phi_table(L, lam, J_min)
    ps, nl = _psi_cols(psi, N)
    f = np.zeros(L * L, dtype=np.complex128)
    for el in range(L):
        norm = (2 * el + 1) / (8.0 * math.pi ** 2)
        ms = np.arange(-el, el + 1)
        # sum over scales and n of (W^j)^l_mn Psi^j_ln
        acc = np.einsum("smn,sn->m", wig[:, el, ms + L - 1, :], ps[:, el, :])
        f[el * el: el * el + 2 * el + 1] = norm * acc
        if Wphi is not None:
            f[el * el: el * el + 2 * el + 1] += (math.sqrt((2 * el + 1) / (4.0 * math.pi))
                                                 * np.asarray(Wphi)[el * el: el * el + 2 * el + 1] * phi[el])
    return f


def synthesis(W, Wphi, L: int, N: int, lam: float, J_min: int, psi=None, phi=None) -> np.ndarray:
    """Exact synthesis of f_lm from the wavelet coefficients on the equiangular grid and
    the harmonic scaling coefficients (Eq. 4 evaluated through Eq. 32, 33 and 41)."""
    wig = forward_wigner_mw(W, L, N)
    return synthesis_from_wigner(wig, Wphi, L, N, lam, J_min, psi=psi, phi=phi)


def synthesis_dh(W, Wphi, L: int, N: int, lam: float, J_min: int, psi=None, phi=None) -> np.ndarray:
    """Exact synthesis from coefficients on the Driscoll-Healy grid (Sec. 3.3, Eq. 32-41)."""
    wig = forward_wigner_dh(W, L, N)
    return synthesis_from_wigner(wig, Wphi, L, N, lam, J_min, psi=psi, phi=phi)


def sht_forward_mw(fmap, L: int) -> np.ndarray:
    """f_lm = int f Y*_lm on the equiangular sphere grid [L][2L-1] (the n = 0, N = 1 case of the
    forward Wigner transform, Y_lm = sqrt((2l+1)/(4 pi)) e^{i m phi} d^l_{m0}(theta))."""
    W = _cplx(fmap)[None, None, :, :]
    wig = forward_wigner_mw(W, L, 1)  # gamma rule with one sample contributes 2 pi
    f = np.zeros(L * L, dtype=np.complex128)
    for el in range(L):
        ms = np.arange(-el, el + 1)
        f[el * el: el * el + 2 * el + 1] = (math.sqrt((2 * el + 1) / (4.0 * math.pi)) / (2.0 * math.pi)
                                            * wig[0, el, ms + L - 1, 0])
    return f


def sht_inverse_mw(flm, L: int, betas=None) -> np.ndarray:
    """f(theta_b, phi_a) = sum f_lm Y_lm on the equiangular sphere grid, complex [nb][2L-1]."""
    c = np.zeros((1, L, 2 * L - 1, 1), dtype=np.complex128)
    f = _cplx(flm)
    for el in range(L):
        ms = np.arange(-el, el + 1)
        c[0, el, ms + L - 1, 0] = math.sqrt((2 * el + 1) / (4.0 * math.pi)) * f[el * el: el * el + 2 * el + 1]
    if betas is None:
        betas = mw_betas(L)
    return inverse_wigner(c, L, [0], betas, 2 * L - 1, 1, 1)[0, 0]
