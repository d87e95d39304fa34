"""Parity with the CPU oracle at the sizes of the configurations, where the oracle can only
afford sampled outputs:

* FP64 synthesis (Sec. 3.3, Eq. 32-41) of non-band-limited samples at L = 2048, N = 4,
  J_min = 4 and at L = 1024, N = 8, J_min = 1.  W is random on a few beta rows (beta = pi
  among them) and zero elsewhere, so the oracle's alpha/gamma rules run on those rows only;
  its beta integral and Wigner step then run on sampled m columns, including columns whose
  Delta start values lie below the double range (the extended-exponent tiles, m > 1022).
* Mixed precision at L = 512 and L = 1024, N = 8, J_min = 1 and at L = 2048, N = 4,
  J_min = 4 (the FP32 transforms of size 2048, 4096 and the prime-factor lengths 2047, 4095,
  and the FP32 m'-sum): sampled analysis rows and synthesis columns.
* The forward spherical-harmonic transform at L = 1024 on sampled m columns.
* Results of the serving loop (one L = 1024 request among small ones, FP64; one mixed
  request) against the oracle.

Bars: FP64 relative max-error <= 1e-11, mixed <= 1e-5, relative to the largest magnitude of
the oracle's sampled output."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import tables
from paper_1308_5706_amd import s2dw
from paper_1308_5706_amd.inputs import random_flm, random_real_map, random_wavelet_samples

pytestmark = pytest.mark.gpu

TOL = 1e-11
MIXED_TOL = 1e-5


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def sampled_rows_W(S, G, L, rows, seed, dtype=np.float64):
    """Arbitrary samples on the given beta rows, zero elsewhere: (the rows [S][G][len][2L-1],
    the full W [S][G][L][2L-1])."""
    Wr = random_wavelet_samples(S, G, len(rows), 2 * L - 1, seed).astype(dtype)
    W = np.zeros((S, G, L, 2 * L - 1), dtype=dtype)
    W[:, :, rows, :] = Wr
    return Wr, W


def oracle_synthesis_columns(Wrows, rows, L, N, lam, J_min, cols, psi):
    """The oracle's synthesis (wavelet part) on m columns `cols`, for samples that vanish
    outside `rows`: {m: f_lm for l = m..L-1}."""
    Gr = oracle.alpha_gamma_rules_mw(Wrows.astype(np.float64), L, N)
    S, nn = Gr.shape[:2]
    Gt = np.zeros((S, nn, L, 2 * L - 1), dtype=np.complex128)
    Gt[:, :, rows, :] = Gr
    del Gr
    wig = oracle.beta_wigner_mw(Gt, L, N, cols=cols)
    del Gt
    fr = oracle.synthesis_from_wigner(wig, None, L, N, lam, J_min, psi=psi)
    return {m: fr[[el * el + el + m for el in range(m, L)]] for m in cols}


SYN_FULL = [  # (L, N, J_min, m columns)
    (2048, 4, 4, [7, 700, 1100, 1900]),
    (1024, 8, 1, [0, 7, 513, 1000, 1023]),
]


@pytest.mark.parametrize("L,N,J_min,cols", SYN_FULL)
def test_full_size_synthesis_of_arbitrary_samples(L, N, J_min, cols):
    lam = 2.0
    S = tables.num_scales(L, lam, J_min)
    G = 2 * N - 1
    rows = [0, 1, L // 2, L - 2, L - 1]
    print(f"full-size synthesis L={L} N={N} J_min={J_min}: rows {rows}, columns {cols}", flush=True)
    Wr, W = sampled_rows_W(S, G, L, rows, 21)
    Wd = torch.as_tensor(W).to("cuda")
    del W
    got = s2dw.synthesis(Wd, None, L, N, lam, J_min)
    torch.cuda.synchronize()
    fs = got.cpu().numpy()
    del Wd, got
    psi = tables.wavelets(L, N, lam, J_min)
    print("  oracle alpha/gamma rules on the rows, beta/Wigner step on the columns", flush=True)
    ref = oracle_synthesis_columns(Wr, rows, L, N, lam, J_min, cols, psi)
    for m in cols:
        e = rel(fs[[el * el + el + m for el in range(m, L)]], ref[m])
        print(f"  m={m}: rel. error {e:.2e}", flush=True)
        assert e < TOL, (m, e)
    s2dw.release_caches()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("L,N,J_min", [(512, 8, 1), (1024, 8, 1), (2048, 4, 4)])
def test_mixed_precision_at_config_sizes(L, N, J_min):
    lam = 2.0
    print(f"mixed precision L={L} N={N} J_min={J_min}: analysis rows", flush=True)
    f = random_flm(L, 31)
    rows = [0, L // 3, L - 1]
    W, _ = s2dw.analysis(torch.as_tensor(f).to("cuda"), L, N, lam, J_min, precision="mixed", scaling=False)
    assert W.dtype == torch.float32
    got = W[:, :, rows, :].double().cpu().numpy()
    del W
    psi = tables.wavelets(L, N, lam, J_min)
    ref = oracle.analysis(f, L, N, lam, J_min, betas=oracle.mw_betas(L)[rows], psi=psi)
    errs = [rel(got[j], ref[j]) for j in range(ref.shape[0])]
    print("  analysis per-scale rel. error", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) < MIXED_TOL
    print("  synthesis of arbitrary FP32 samples on sampled rows and columns", flush=True)
    S = ref.shape[0]
    srows = [0, L // 2, L - 1]
    Wr, Wf = sampled_rows_W(S, 2 * N - 1, L, srows, 32, dtype=np.float32)
    fs = s2dw.synthesis(torch.as_tensor(Wf).to("cuda"), None, L, N, lam, J_min, precision="mixed")
    torch.cuda.synchronize()
    fs = fs.cpu().numpy()
    cols = [0, 5, L // 2, L - 1]
    refs = oracle_synthesis_columns(Wr, srows, L, N, lam, J_min, cols, psi)
    for m in cols:
        e = rel(fs[[el * el + el + m for el in range(m, L)]], refs[m])
        print(f"  m={m}: rel. error {e:.2e}", flush=True)
        assert e < MIXED_TOL, (m, e)
    s2dw.release_caches()
    torch.cuda.empty_cache()


def test_sht_forward_full_size_columns():
    L = 1024
    print(f"forward SHT L={L} on sampled m columns", flush=True)
    arb = random_real_map(L, 2 * L - 1, 33)
    got = s2dw.sht_forward(torch.as_tensor(arb).to("cuda"), L)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    Gt = oracle.alpha_gamma_rules_mw(arb[None, None, :, :], L, 1)
    cols = [0, 1, 511, 1022, 1023]
    wig = oracle.beta_wigner_mw(Gt, L, 1, cols=cols)
    for m in cols:
        ref = np.array([math.sqrt((2 * el + 1) / (4.0 * math.pi)) / (2.0 * math.pi) * wig[0, el, m + L - 1, 0]
                        for el in range(m, L)])
        e = rel(got[[el * el + el + m for el in range(m, L)]], ref)
        print(f"  m={m}: rel. error {e:.2e}", flush=True)
        assert e < TOL, (m, e)


@pytest.mark.parametrize("precision,big", [("fp64", (1024, 8)), ("mixed", (256, 4))])
def test_served_results_against_oracle(precision, big):
    import time

    from paper_1308_5706_amd.serve import Request, Server
    lam, J_min = 2.0, 1
    tol = TOL if precision == "fp64" else MIXED_TOL
    print(f"served results vs oracle, {precision}, large request L={big[0]} N={big[1]}", flush=True)
    shapes = [(32, 4), big, (64, 1)]
    reqs = [Request(i, L, N, torch.as_tensor(random_flm(L, 700 + i)).to("cuda")) for i, (L, N) in enumerate(shapes)]
    srv = Server(lam=lam, J_min=J_min, precision=precision, streams=2, max_batch=2)
    srv.warm(shapes)
    for r in reqs:
        r.t_arrival = time.perf_counter()
        srv.submit(r)
    done = []
    while not srv.idle():
        done += srv.step()
    assert sorted(r.rid for r in done) == [0, 1, 2]
    for r in sorted(done, key=lambda q: q.rid):
        L, N = r.L, r.N
        rows = [0, L - 1]
        got = r.W[:, :, rows, :].double().cpu().numpy()
        ref = oracle.analysis(r.flm.cpu().numpy(), L, N, lam, J_min, betas=oracle.mw_betas(L)[rows])
        e = max(rel(got[j], ref[j]) for j in range(ref.shape[0]))
        print(f"  request {r.rid} L={L} N={N}: rel. error {e:.2e}", flush=True)
        assert e < tol, (r.rid, e)
        assert rel(r.Wphi.cpu().numpy(), oracle.scaling(r.flm.cpu().numpy(), L, lam, J_min)) < TOL
    del done, reqs, srv
    s2dw.release_caches()
    torch.cuda.empty_cache()
