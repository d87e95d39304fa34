"""The analysis entry point that allocates nothing (fixed per-GPU scratch) against the
allocating one, called through the C ABI: two calls in a row, the second with a smaller
input, each bitwise equal to s2dw_analysis (same kernels) and so within the FP64 bar."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1308_5706_amd import s2dw
from paper_1308_5706_amd.inputs import random_flm

pytestmark = pytest.mark.gpu


def _call(L, N, J_min, f, W, Wp, precision="fp64"):
    p = s2dw.params(L, N, 2.0, J_min, precision)
    return s2dw.lib().s2dw_analysis_noalloc(ctypes.byref(p), ctypes.c_void_p(f.data_ptr()),
                                            ctypes.c_void_p(W.data_ptr()),
                                            ctypes.c_void_p(Wp.data_ptr() if Wp is not None else None),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_analysis_matches_allocating_entry_point():
    for i, (L, N, J_min) in enumerate([(64, 8, 1), (40, 3, 0)]):  # the second call is smaller
        print(f"no-alloc analysis call {i}: L={L} N={N} J_min={J_min}", flush=True)
        f = torch.as_tensor(random_flm(L, 41 + i)).to("cuda")
        W_ref, Wp_ref = s2dw.analysis(f, L, N, 2.0, J_min)  # allocating call: builds the plan
        W = torch.full_like(W_ref, float("nan"))
        Wp = torch.full_like(Wp_ref, float("nan"))
        torch.cuda.synchronize()
        assert _call(L, N, J_min, f, W, Wp) == 0
        torch.cuda.synchronize()
        assert torch.equal(W, W_ref), i
        assert torch.equal(Wp, Wp_ref), i
        err = float((W - W_ref).abs().max() / W_ref.abs().max())
        assert err < 1e-11


def test_noalloc_mixed_and_complex_match():
    from paper_1308_5706_amd.inputs import random_flm_complex
    L, N, J_min = 48, 4, 1
    print("no-alloc analysis, mixed precision and a complex signal", flush=True)
    f = torch.as_tensor(random_flm(L, 51)).to("cuda")
    W_ref, Wp_ref = s2dw.analysis(f, L, N, 2.0, J_min, precision="mixed")
    W = torch.full_like(W_ref, float("nan"))
    assert _call(L, N, J_min, f, W, None, "mixed") == 0
    torch.cuda.synchronize()
    assert torch.equal(W, W_ref)
    fc = torch.as_tensor(random_flm_complex(L, 52)).to("cuda")
    W_ref, Wp_ref = s2dw.analysis(fc, L, N, 2.0, J_min, reality=False)
    W = torch.full_like(W_ref, float("nan"))
    Wp = torch.full_like(Wp_ref, float("nan"))
    s2dw.analysis_noalloc(fc, W, Wp, L, N, 2.0, J_min, reality=False)
    torch.cuda.synchronize()
    assert torch.equal(W, W_ref) and torch.equal(Wp, Wp_ref)


def test_noalloc_refusals():
    # a plan that was never built, and a workspace beyond the fixed scratch
    L, N = 24, 2
    f = torch.zeros(L * L, dtype=torch.complex128, device="cuda")
    W = torch.zeros((s2dw.num_scales(L, 2.0, 3),) + (2 * N - 1, L, 2 * L - 1), dtype=torch.float64, device="cuda")
    assert _call(L, N, 3, f, W, None) == -1  # S2DW_E_ARG: no plan with these parameters yet
    L, N, J_min = 1024, 8, 1
    s2dw.workspace_bytes(L, N, 2.0, J_min)  # builds the plan (host tables only)
    f = torch.zeros(L * L, dtype=torch.complex128, device="cuda")
    W = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert _call(L, N, J_min, f, W, None) == -4  # S2DW_E_UNSUPPORTED: beyond the scratch
    torch.cuda.synchronize()
