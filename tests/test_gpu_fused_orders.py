"""The fused alpha and gamma kernels of the prime-factor lengths T = 2047 and T = 4095 for
every count of orders n >= 0 they serve (Nh = 1..4 at T = 2047, 1..2 at T = 4095), with and
without the order n = 0 (odd and even N), in FP64 and in mixed precision: the analysis
(Sec. 3.2, Eq. 29-31) on sampled beta rows against the oracle, and the synthesis
(Sec. 3.3, Eq. 32-41) of arbitrary samples on sampled beta rows, checked on sampled m columns.
Bars: FP64 relative max-error <= 1e-11, mixed <= 1e-5, relative to the largest magnitude of
the oracle's sampled output (per scale for the analysis)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import tables
from paper_1308_5706_amd import s2dw
from paper_1308_5706_amd.inputs import random_flm

from test_gpu_config_parity import oracle_synthesis_columns, rel, sampled_rows_W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "mixed": 1e-5}

CASES = [  # (L, N, J_min, precision): Nh = N - N // 2 orders n >= 0 per transform
    (1024, 1, 4, "fp64"),
    (1024, 2, 4, "mixed"),
    (1024, 3, 4, "fp64"),
    (1024, 6, 4, "fp64"),
    (1024, 5, 4, "mixed"),
    (2048, 1, 6, "fp64"),
    (2048, 2, 6, "mixed"),
    (2048, 3, 6, "mixed"),
]


@pytest.mark.parametrize("L,N,J_min,precision", CASES)
def test_fused_alpha_gamma_orders(L, N, J_min, precision):
    lam = 2.0
    tol = TOL[precision]
    print(f"fused alpha/gamma L={L} N={N} J_min={J_min} {precision}: analysis rows", flush=True)
    f = random_flm(L, 41 + N)
    rows = [0, L - 1]
    W, _ = s2dw.analysis(torch.as_tensor(f).to("cuda"), L, N, lam, J_min, precision=precision, scaling=False)
    got = W[:, :, rows, :].double().cpu().numpy()
    del W
    psi = tables.wavelets(L, N, lam, J_min)
    ref = oracle.analysis(f, L, N, lam, J_min, betas=oracle.mw_betas(L)[rows], psi=psi)
    errs = [rel(got[j], ref[j]) for j in range(ref.shape[0])]
    print("  analysis per-scale rel. error", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) < tol, errs
    print("  synthesis of arbitrary samples on sampled rows and columns", flush=True)
    S = ref.shape[0]
    srows = [0, L // 2, L - 1]
    dtype = np.float64 if precision == "fp64" else np.float32
    Wr, Wf = sampled_rows_W(S, 2 * N - 1, L, srows, 43 + N, dtype=dtype)
    fs = s2dw.synthesis(torch.as_tensor(Wf).to("cuda"), None, L, N, lam, J_min, precision=precision)
    torch.cuda.synchronize()
    fs = fs.cpu().numpy()
    del Wf
    cols = [0, 3, L // 2 + 1, L - 1]
    refs = oracle_synthesis_columns(Wr, srows, L, N, lam, J_min, cols, psi)
    for m in cols:
        e = rel(fs[[el * el + el + m for el in range(m, L)]], refs[m])
        print(f"  m={m}: rel. error {e:.2e}", flush=True)
        assert e < tol, (m, e)
    s2dw.release_caches()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("L,N,J_min", [(1024, 6, 4), (2048, 2, 6)])
def test_alpha_gamma_forms_agree(L, N, J_min):
    # the two-pass form (0), the default (1) and the fused form wherever it applies (2) give
    # the same analysis and synthesis to rounding; with N = 6 at T = 2047 form 2 takes the
    # fused synthesis kernel that sweeps W once per pass, and at T = 4095 form 0 takes the
    # two-pass prime-factor kernels the default does not use
    lam = 2.0
    f = torch.as_tensor(random_flm(L, 51 + N)).to("cuda")
    slots, chunk, fuse = s2dw.get_tuning(L, N, lam, J_min)
    assert fuse == 1
    out = {}
    try:
        for form in (1, 0, 2):
            s2dw.set_tuning(L, N, lam, J_min, slots=slots, chunk=chunk, fuse=form)
            assert s2dw.get_tuning(L, N, lam, J_min) == (slots, chunk, form)
            print(f"L={L} N={N}: form {form}", flush=True)
            W, Wp = s2dw.analysis(f, L, N, lam, J_min)
            fr = s2dw.synthesis(W, Wp, L, N, lam, J_min)
            torch.cuda.synchronize()
            out[form] = (W.cpu().numpy(), fr.cpu().numpy())
            del W, Wp, fr
    finally:
        s2dw.set_tuning(L, N, lam, J_min, slots=slots, chunk=chunk, fuse=1)
    W1, f1 = out[1]
    for form in (0, 2):
        Wf, ff = out[form]
        for j in range(W1.shape[0]):
            assert rel(Wf[j], W1[j]) < 1e-12, (form, j)
        assert rel(ff, f1) < 1e-12, form
        assert rel(ff, f.cpu().numpy()) < 1e-12, form
    s2dw.release_caches()
    torch.cuda.empty_cache()
