"""Python binding of the C ABI in ``include/s2dw.h`` (argument marshalling only).

Every transform runs in the HIP kernels of ``libs2dw.so``; this module only
checks tensor shapes, allocates outputs with torch and passes device pointers
and the current HIP stream.  It raises if the library is not built: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libs2dw.so")

FP64, MIXED = 0, 1
GRID_MW, GRID_MW_MULTIRES, GRID_DH = 0, 1, 2
GRIDS = {"mw": GRID_MW, "multires": GRID_MW_MULTIRES, "dh": GRID_DH}
PRECISIONS = {"fp64": FP64, "mixed": MIXED}

_lib = None


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("N", ctypes.c_int32), ("lam", ctypes.c_double),
                ("J_min", ctypes.c_int32), ("grid", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reality", ctypes.c_int32)]


class Group(ctypes.Structure):
    _fields_ = [("params", Params), ("count", ctypes.c_int32), ("flm", ctypes.c_void_p), ("W", ctypes.c_void_p),
                ("Wphi_lm", ctypes.c_void_p)]


class StageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("ms", ctypes.c_double), ("count", ctypes.c_int64)]


class S2DWError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {lib().s2dw_strerror(code).decode()} ({code})")
        self.code = code


def lib():
    """The loaded libs2dw.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, cp = ctypes.c_void_p, ctypes.POINTER(Params)
        for name, args in [("s2dw_num_scales", [cp, ctypes.POINTER(ctypes.c_int32)]),
                           ("s2dw_grid_shape", [cp, ctypes.POINTER(ctypes.c_int32)]),
                           ("s2dw_wavelet_bytes", [cp, ctypes.POINTER(ctypes.c_uint64)]),
                           ("s2dw_analysis", [cp, vp, vp, vp, vp]),
                           ("s2dw_analysis_noalloc", [cp, vp, vp, vp, vp]),
                           ("s2dw_synthesis", [cp, vp, vp, vp, vp]),
                           ("s2dw_scaling", [cp, vp, vp, vp, vp]),
                           ("s2dw_sht_forward", [cp, vp, vp, vp]),
                           ("s2dw_sht_inverse", [cp, vp, vp, vp]),
                           ("s2dw_analysis_batched", [cp, ctypes.c_int32, vp, vp, vp, vp]),
                           ("s2dw_synthesis_batched", [cp, ctypes.c_int32, vp, vp, vp, vp]),
                           ("s2dw_steer", [cp, ctypes.c_int32, vp, ctypes.c_int32, vp, vp, vp]),
                           ("s2dw_autotune", [cp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)])]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.s2dw_strerror.argtypes = [ctypes.c_int]
        L.s2dw_strerror.restype = ctypes.c_char_p
        L.s2dw_release_caches.argtypes = []
        L.s2dw_release_caches.restype = None
        L.s2dw_scale_grid.argtypes = [cp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_uint64)]
        L.s2dw_scale_grid.restype = ctypes.c_int
        L.s2dw_wavelet_tables.argtypes = [cp, vp, vp, vp]
        L.s2dw_wavelet_tables.restype = ctypes.c_int
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.s2dw_get_tuning.argtypes = [cp, i32p, i32p, i32p]
        L.s2dw_get_tuning.restype = ctypes.c_int
        L.s2dw_set_tuning.argtypes = [cp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.s2dw_set_tuning.restype = ctypes.c_int
        gp = ctypes.POINTER(Group)
        L.s2dw_analysis_persistent.argtypes = [gp, ctypes.c_int32, vp, vp]
        L.s2dw_analysis_persistent.restype = ctypes.c_int
        L.s2dw_synthesis_persistent.argtypes = [gp, ctypes.c_int32, vp, vp]
        L.s2dw_synthesis_persistent.restype = ctypes.c_int
        L.s2dw_persistent_wait_bound.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.s2dw_persistent_wait_bound.restype = ctypes.c_int
        L.s2dw_workspace_bytes.argtypes = [cp, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
        L.s2dw_workspace_bytes.restype = ctypes.c_int
        L.s2dw_cache_bytes.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        L.s2dw_cache_bytes.restype = ctypes.c_int
        L.s2dw_profile.argtypes = [ctypes.c_int]
        L.s2dw_profile.restype = ctypes.c_int
        L.s2dw_profile_read.argtypes = [ctypes.POINTER(StageTime), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.s2dw_profile_read.restype = ctypes.c_int
        L.s2dw_profile_stages.argtypes = [ctypes.c_char_p]
        L.s2dw_profile_stages.restype = ctypes.c_int
        _lib = L
    return _lib


EXPORTED = ["s2dw_num_scales", "s2dw_grid_shape", "s2dw_wavelet_bytes", "s2dw_scale_grid", "s2dw_analysis",
            "s2dw_analysis_noalloc",
            "s2dw_synthesis", "s2dw_analysis_batched", "s2dw_synthesis_batched", "s2dw_steer", "s2dw_autotune", "s2dw_get_tuning", "s2dw_set_tuning",
            "s2dw_analysis_persistent", "s2dw_synthesis_persistent", "s2dw_persistent_wait_bound", "s2dw_workspace_bytes",
            "s2dw_cache_bytes",
            "s2dw_scaling", "s2dw_sht_forward", "s2dw_sht_inverse", "s2dw_wavelet_tables", "s2dw_profile",
            "s2dw_profile_read", "s2dw_profile_stages",
            "s2dw_strerror", "s2dw_release_caches"]


def params(L: int, N: int, lam: float = 2.0, J_min: int = 0, precision: str = "fp64",
           grid: str = "mw", reality: bool = True) -> Params:
    """grid: "mw" (equiangular, every scale at band-limit L), "multires" (each scale on the
    equiangular grid of its own band-limit) or "dh" (the Driscoll-Healy grid of Sec. 3.1);
    reality: real signal (real W) or complex signal (complex W)."""
    if grid not in GRIDS:
        raise ValueError(f"grid must be one of {sorted(GRIDS)}, not {grid!r}")
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}, not {precision!r}")
    return Params(L, N, float(lam), J_min, GRIDS[grid], PRECISIONS[precision], 1 if reality else 0)


def _check(rc: int, what: str):
    if rc != 0:
        raise S2DWError(rc, what)


def num_scales(L: int, lam: float = 2.0, J_min: int = 0) -> int:
    s = ctypes.c_int32()
    _check(lib().s2dw_num_scales(ctypes.byref(params(L, 1, lam, J_min)), ctypes.byref(s)), "num_scales")
    return s.value


def wavelet_tables(L: int, N: int, lam: float = 2.0, J_min: int = 0):
    """Host numpy arrays (kappa [S][L], phi [L], s_ln complex [L][2N-1]) built by the library."""
    import numpy as np
    S = num_scales(L, lam, J_min)
    kap = np.zeros((S, L))
    phi = np.zeros(L)
    s = np.zeros((L, 2 * N - 1), dtype=np.complex128)
    _check(lib().s2dw_wavelet_tables(ctypes.byref(params(L, N, lam, J_min)), ctypes.c_void_p(kap.ctypes.data),
                                     ctypes.c_void_p(phi.ctypes.data), ctypes.c_void_p(s.ctypes.data)),
           "s2dw_wavelet_tables")
    return kap, phi, s


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _as_complex(x: torch.Tensor, n: int, what: str) -> torch.Tensor:
    if not x.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if x.dtype == torch.complex128:
        x = torch.view_as_real(x)
    if x.dtype != torch.float64 or x.numel() != 2 * n:
        raise ValueError(f"{what}: expected {n} complex128 values")
    return x.contiguous()


def _w_dtype(precision: str, reality: bool = True):
    if precision not in ("fp64", "mixed"):
        raise ValueError(f"precision must be 'fp64' or 'mixed', not {precision!r}")
    if reality:
        return torch.float64 if precision == "fp64" else torch.float32
    return torch.complex128 if precision == "fp64" else torch.complex64


def scale_grid(L: int, N: int, lam: float = 2.0, J_min: int = 0, j: int = 0, *, grid: str = "mw"):
    """(shape (n_gamma, n_beta, n_alpha), element offset) of scale j in the W of one map."""
    sh = (ctypes.c_int32 * 3)()
    off = ctypes.c_uint64()
    _check(lib().s2dw_scale_grid(ctypes.byref(params(L, N, lam, J_min, grid=grid)), j, sh,
                                 ctypes.byref(off)), "s2dw_scale_grid")
    return (sh[0], sh[1], sh[2]), off.value


def _w_shape(L, N, lam, J_min, grid):
    """Shape of the W of one map: [S][n_gamma][n_beta][n_alpha], or flat for the
    multiresolution layout."""
    S = num_scales(L, lam, J_min)
    sh, off = scale_grid(L, N, lam, J_min, S - 1, grid=grid)
    if grid != "multires":
        return (S,) + sh
    return (off + sh[0] * sh[1] * sh[2],)


def split_scales(W: torch.Tensor, L: int, N: int, lam: float = 2.0, J_min: int = 0) -> list:
    """Views [(B,) 2N-1, L_j, 2L_j-1] of each scale of multiresolution coefficients W
    ([total] or [B][total])."""
    lead = W.shape[:-1]
    out = []
    for j in range(num_scales(L, lam, J_min)):
        sh, off = scale_grid(L, N, lam, J_min, j, grid="multires")
        n = sh[0] * sh[1] * sh[2]
        out.append(W[..., off:off + n].reshape(lead + sh))
    return out


def _check_w(W, shape, dtype, B, what):
    n = B
    for d in shape:
        n *= d
    if W.dtype != dtype or W.numel() != n or not W.is_cuda or not W.is_contiguous():
        raise ValueError(f"{what}: wrong shape, dtype or layout")


def analysis(flm: torch.Tensor, L: int, N: int, lam: float = 2.0, J_min: int = 0, *, scaling: bool = True,
             out: torch.Tensor | None = None, stream=None, precision: str = "fp64", grid: str = "mw",
             reality: bool = True):
    """Wavelet coefficients W [S][2N-1][L][2L-1] (float64, or float32 with precision="mixed";
    complex128 / complex64 for a complex signal, reality=False; flat in the multiresolution
    layout, see split_scales) and, if scaling, the harmonic scaling coefficients W^Phi_lm
    (complex128 [L*L])."""
    p = params(L, N, lam, J_min, precision, grid, reality)
    wdt = _w_dtype(precision, reality)
    f = _as_complex(flm, L * L, "flm")
    shape = _w_shape(L, N, lam, J_min, grid)
    W = out if out is not None else torch.empty(shape, dtype=wdt, device=f.device)
    _check_w(W, shape, wdt, 1, "W")
    Wp = torch.empty(L * L, dtype=torch.complex128, device=f.device) if scaling else None
    _check(lib().s2dw_analysis(ctypes.byref(p), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(W.data_ptr()),
                               ctypes.c_void_p(Wp.data_ptr() if Wp is not None else None), _stream(stream)),
           "s2dw_analysis")
    return W, Wp


def analysis_noalloc(flm: torch.Tensor, W: torch.Tensor, Wphi: torch.Tensor | None, L: int, N: int,
                     lam: float = 2.0, J_min: int = 0, *, stream=None, precision: str = "fp64", grid: str = "mw",
                     reality: bool = True) -> None:
    """s2dw_analysis into caller-given W (and W^Phi, or None) through the entry point that
    allocates no device memory (the plan must exist, see include/s2dw.h)."""
    p = params(L, N, lam, J_min, precision, grid, reality)
    f = _as_complex(flm, L * L, "flm")
    _check_w(W, _w_shape(L, N, lam, J_min, grid), _w_dtype(precision, reality), 1, "W")
    wp = _as_complex(Wphi, L * L, "Wphi") if Wphi is not None else None
    _check(lib().s2dw_analysis_noalloc(ctypes.byref(p), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(W.data_ptr()),
                                       ctypes.c_void_p(wp.data_ptr() if wp is not None else None), _stream(stream)),
           "s2dw_analysis_noalloc")


def synthesis(W: torch.Tensor, Wphi: torch.Tensor | None, L: int, N: int, lam: float = 2.0, J_min: int = 0, *,
              out: torch.Tensor | None = None, stream=None, precision: str = "fp64",
              grid: str = "mw", reality: bool = True) -> torch.Tensor:
    """f_lm (complex128 [L*L]) from W (float64, or float32 with precision="mixed") and the
    scaling coefficients (or the wavelet part only)."""
    p = params(L, N, lam, J_min, precision, grid, reality)
    W = W.contiguous()
    _check_w(W, _w_shape(L, N, lam, J_min, grid), _w_dtype(precision, reality), 1, "W")
    wp = _as_complex(Wphi, L * L, "Wphi") if Wphi is not None else None
    f = out if out is not None else torch.empty(L * L, dtype=torch.complex128, device=W.device)
    _check(lib().s2dw_synthesis(ctypes.byref(p), ctypes.c_void_p(W.data_ptr()),
                                ctypes.c_void_p(wp.data_ptr() if wp is not None else None),
                                ctypes.c_void_p(f.data_ptr()), _stream(stream)), "s2dw_synthesis")
    return f


def analysis_batched(flm: torch.Tensor, L: int, N: int, lam: float = 2.0, J_min: int = 0, *, scaling: bool = True,
                     out: torch.Tensor | None = None, stream=None, precision: str = "fp64", grid: str = "mw",
                     reality: bool = True):
    """A batch of maps with the same parameters: flm complex128 [B][L*L] -> W [B][S][2N-1][L][2L-1]
    (float64 or float32; [B][total] in the multiresolution layout) and, if scaling, W^Phi
    complex128 [B][L*L]."""
    p = params(L, N, lam, J_min, precision, grid, reality)
    wdt = _w_dtype(precision, reality)
    if flm.dim() != 2 or flm.shape[1] != L * L:
        raise ValueError("flm: expected [B][L*L] complex128")
    B = flm.shape[0]
    f = _as_complex(flm, B * L * L, "flm")
    shape = _w_shape(L, N, lam, J_min, grid)
    W = out if out is not None else torch.empty((B,) + shape, dtype=wdt, device=f.device)
    _check_w(W, shape, wdt, B, "W")
    Wp = torch.empty((B, L * L), dtype=torch.complex128, device=f.device) if scaling else None
    _check(lib().s2dw_analysis_batched(ctypes.byref(p), B, ctypes.c_void_p(f.data_ptr()),
                                       ctypes.c_void_p(W.data_ptr()),
                                       ctypes.c_void_p(Wp.data_ptr() if Wp is not None else None), _stream(stream)),
           "s2dw_analysis_batched")
    return W, Wp


def synthesis_batched(W: torch.Tensor, Wphi: torch.Tensor | None, L: int, N: int, lam: float = 2.0,
                      J_min: int = 0, *, out: torch.Tensor | None = None, stream=None,
                      precision: str = "fp64", grid: str = "mw", reality: bool = True) -> torch.Tensor:
    """A batch of maps: W [B][S][2N-1][L][2L-1] (+ W^Phi [B][L*L]) -> f_lm complex128 [B][L*L]."""
    p = params(L, N, lam, J_min, precision, grid, reality)
    B = W.shape[0]
    W = W.contiguous()
    _check_w(W, _w_shape(L, N, lam, J_min, grid), _w_dtype(precision, reality), B, "W")
    wp = _as_complex(Wphi, B * L * L, "Wphi") if Wphi is not None else None
    f = out if out is not None else torch.empty((B, L * L), dtype=torch.complex128, device=W.device)
    _check(lib().s2dw_synthesis_batched(ctypes.byref(p), B, ctypes.c_void_p(W.data_ptr()),
                                        ctypes.c_void_p(wp.data_ptr() if wp is not None else None),
                                        ctypes.c_void_p(f.data_ptr()), _stream(stream)), "s2dw_synthesis_batched")
    return f


def autotune(L: int, N: int, lam: float = 2.0, J_min: int = 0, *, count: int = 1, precision: str = "fp64",
             stream=None, grid: str = "mw", reality: bool = True):
    """Times the compiled Wigner tile shapes and batch chunks for these parameters and keeps
    the fastest in the library's plan; returns (m' slots per wave, maps per chunk)."""
    sl, ch = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().s2dw_autotune(ctypes.byref(params(L, N, lam, J_min, precision, grid, reality)), count, _stream(stream),
                               ctypes.byref(sl), ctypes.byref(ch)), "s2dw_autotune")
    return sl.value, ch.value


def _groups(items, precision):
    arr = (Group * len(items))()
    for i, (L, N, lam, J_min, f, W, Wp) in enumerate(items):
        arr[i].params = params(L, N, lam, J_min, precision, "mw", True)
        arr[i].count = f.shape[0]
        arr[i].flm = f.data_ptr()
        arr[i].W = W.data_ptr()
        arr[i].Wphi_lm = Wp.data_ptr() if Wp is not None else None
    return arr


def analysis_persistent(groups, *, precision: str = "fp64", stream=None, status: torch.Tensor | None = None,
                        scaling: bool = True):
    """Analyses of several batches, one per parameter set, through the persistent executor (two
    launches).  groups: list of (L, N, lam, J_min, flm complex128 [B][L*L]); returns a list of
    (W [B][S][2N-1][L][2L-1], W^Phi [B][L*L] or None).  The output buffers are allocated on the
    first call with a given list of inputs and reused (the same tensors) on later calls, so
    that the call can be replayed in a graph.  status: optional int32 device tensor of one
    element, set to 0 (or 1: a dependency wait ran out; the results are not valid)."""
    key = ("a", precision, tuple((L, N, lam, J, f.data_ptr(), f.shape[0]) for L, N, lam, J, f in groups))
    outs = _persist_outs.get(key)
    if outs is None:
        outs = []
        for L, N, lam, J_min, f in groups:
            if f.dim() != 2 or f.shape[1] != L * L or f.dtype != torch.complex128 or not f.is_contiguous():
                raise ValueError("flm: expected contiguous [B][L*L] complex128")
            W = torch.empty((f.shape[0],) + _w_shape(L, N, lam, J_min, "mw"), dtype=_w_dtype(precision, True),
                            device=f.device)
            Wp = torch.empty((f.shape[0], L * L), dtype=torch.complex128, device=f.device) if scaling else None
            outs.append((W, Wp))
        _persist_outs[key] = outs
    arr = _groups([(L, N, lam, J, f, W, Wp) for (L, N, lam, J, f), (W, Wp) in zip(groups, outs)], precision)
    _check(lib().s2dw_analysis_persistent(arr, len(groups), ctypes.c_void_p(status.data_ptr() if status is not None
                                                                              else None), _stream(stream)),
           "s2dw_analysis_persistent")
    return outs


def synthesis_persistent(groups, *, precision: str = "fp64", stream=None, status: torch.Tensor | None = None):
    """Syntheses of several batches through the persistent executor.  groups: list of
    (L, N, lam, J_min, W [B][S][2N-1][L][2L-1], W^Phi [B][L*L] or None); returns the list of
    f_lm complex128 [B][L*L] (allocated on the first call with these inputs, then reused)."""
    key = ("s", precision, tuple((L, N, lam, J, W.data_ptr(), Wp.data_ptr() if Wp is not None else 0, W.shape[0])
                                 for L, N, lam, J, W, Wp in groups))
    outs = _persist_outs.get(key)
    if outs is None:
        outs = []
        for L, N, lam, J_min, W, Wp in groups:
            _check_w(W, _w_shape(L, N, lam, J_min, "mw"), _w_dtype(precision, True), W.shape[0], "W")
            outs.append(torch.empty((W.shape[0], L * L), dtype=torch.complex128, device=W.device))
        _persist_outs[key] = outs
    arr = _groups([(L, N, lam, J, f, W, Wp) for (L, N, lam, J, W, Wp), f in zip(groups, outs)], precision)
    _check(lib().s2dw_synthesis_persistent(arr, len(groups), ctypes.c_void_p(status.data_ptr() if status is not None
                                                                               else None), _stream(stream)),
           "s2dw_synthesis_persistent")
    return outs


def persistent_wait_bound(polls: int = 0, never_satisfied: bool = False) -> None:
    """Bound of the persistent executor's dependency waits (polls of ~0.2 us; 0: default);
    never_satisfied (tests only): every wait runs out."""
    _check(lib().s2dw_persistent_wait_bound(polls, 1 if never_satisfied else 0), "s2dw_persistent_wait_bound")


_persist_outs: dict = {}

FUSE_FORMS = {"two-pass": 0, "default": 1, "fused": 2}


def get_tuning(L: int, N: int, lam: float = 2.0, J_min: int = 0, *, precision: str = "fp64", grid: str = "mw",
               reality: bool = True):
    """The plan's tuning: (m' slots per wave, maps per chunk, alpha/gamma form 0..2)."""
    sl, ch, fu = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().s2dw_get_tuning(ctypes.byref(params(L, N, lam, J_min, precision, grid, reality)), ctypes.byref(sl),
                                 ctypes.byref(ch), ctypes.byref(fu)), "s2dw_get_tuning")
    return sl.value, ch.value, fu.value


def set_tuning(L: int, N: int, lam: float = 2.0, J_min: int = 0, *, slots: int, chunk: int, fuse,
               precision: str = "fp64", grid: str = "mw", reality: bool = True) -> None:
    """Applies a tuning (e.g. one autotune found before); fuse is 0..2 or a FUSE_FORMS name."""
    fu = FUSE_FORMS[fuse] if isinstance(fuse, str) else int(fuse)
    _check(lib().s2dw_set_tuning(ctypes.byref(params(L, N, lam, J_min, precision, grid, reality)), slots, chunk, fu),
           "s2dw_set_tuning")


def steer(W: torch.Tensor, gammas, L: int, N: int, lam: float = 2.0, J_min: int = 0, *,
          out: torch.Tensor | None = None, stream=None, grid: str = "mw") -> torch.Tensor:
    """Wavelet coefficients at arbitrary third Euler angles (steerability, Eq. 10).

    W: [S][2N-1][L][2L-1] or [B][S][2N-1][L][2L-1], float64 (or float32: the mixed-precision
    layout); with multires, [total] or [B][total].  gammas: angles in radians (a sequence or
    a float64 tensor).  Returns [(B,) S, Q, L, 2L-1] (multires: [(B,) total_Q] with scale j's
    [Q][L_j][2L_j-1] block at Q/(2N-1) times its offset in W) in W's dtype."""
    if W.dtype not in (torch.float64, torch.float32, torch.complex128, torch.complex64) or not W.is_cuda:
        raise ValueError("W: expected a float64, float32, complex128 or complex64 device tensor")
    precision = "fp64" if W.dtype in (torch.float64, torch.complex128) else "mixed"
    reality = not W.is_complex()
    shape = _w_shape(L, N, lam, J_min, grid)
    per = 1
    for d in shape:
        per *= d
    batched = W.dim() == len(shape) + 1
    if W.numel() == 0 or W.numel() % per != 0 or W.dim() not in (len(shape), len(shape) + 1):
        raise ValueError("W: wrong shape")
    B = W.numel() // per
    W = W.contiguous()
    g = torch.as_tensor(gammas, dtype=torch.float64).reshape(-1).to(W.device).contiguous()
    Q = g.numel()
    G = N if grid == "dh" else 2 * N - 1
    oshape = (per // G * Q,) if grid == "multires" else (shape[0], Q) + shape[2:]
    oshape = ((B,) if batched else ()) + oshape
    o = out if out is not None else torch.empty(oshape, dtype=W.dtype, device=W.device)
    if o.dtype != W.dtype or o.numel() != B * (per // G) * Q or not o.is_contiguous():
        raise ValueError("out: wrong shape, dtype or layout")
    _check(lib().s2dw_steer(ctypes.byref(params(L, N, lam, J_min, precision, grid, reality)), B,
                            ctypes.c_void_p(W.data_ptr()), Q, ctypes.c_void_p(g.data_ptr()),
                            ctypes.c_void_p(o.data_ptr()), _stream(stream)), "s2dw_steer")
    return o


def scaling(flm: torch.Tensor, L: int, N: int = 1, lam: float = 2.0, J_min: int = 0, *, sphere_map: bool = False,
            stream=None):
    """Harmonic scaling coefficients (complex128 [L*L]) and optionally their sphere map [L][2L-1]."""
    p = params(L, N, lam, J_min)
    f = _as_complex(flm, L * L, "flm")
    Wp = torch.empty(L * L, dtype=torch.complex128, device=f.device)
    mp = torch.empty((L, 2 * L - 1), dtype=torch.float64, device=f.device) if sphere_map else None
    _check(lib().s2dw_scaling(ctypes.byref(p), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(Wp.data_ptr()),
                              ctypes.c_void_p(mp.data_ptr() if mp is not None else None), _stream(stream)),
           "s2dw_scaling")
    return Wp, mp


def sht_forward(fmap: torch.Tensor, L: int, stream=None) -> torch.Tensor:
    """f_lm of a real map on the equiangular grid [L][2L-1]."""
    if fmap.dtype != torch.float64 or tuple(fmap.shape) != (L, 2 * L - 1) or not fmap.is_cuda:
        raise ValueError("fmap: expected float64 [L][2L-1] on the device")
    fmap = fmap.contiguous()
    f = torch.empty(L * L, dtype=torch.complex128, device=fmap.device)
    _check(lib().s2dw_sht_forward(ctypes.byref(params(L, 1)), ctypes.c_void_p(fmap.data_ptr()),
                                  ctypes.c_void_p(f.data_ptr()), _stream(stream)), "s2dw_sht_forward")
    return f


def sht_inverse(flm: torch.Tensor, L: int, stream=None) -> torch.Tensor:
    """The real map [L][2L-1] of f_lm on the equiangular grid."""
    f = _as_complex(flm, L * L, "flm")
    m = torch.empty((L, 2 * L - 1), dtype=torch.float64, device=f.device)
    _check(lib().s2dw_sht_inverse(ctypes.byref(params(L, 1)), ctypes.c_void_p(f.data_ptr()),
                                  ctypes.c_void_p(m.data_ptr()), _stream(stream)), "s2dw_sht_inverse")
    return m


def workspace_bytes(L: int, N: int, lam: float = 2.0, J_min: int = 0, *, count: int = 1,
                    precision: str = "fp64", grid: str = "mw", reality: bool = True) -> int:
    """Device bytes of one stream's workspace for a batch of `count` maps."""
    b = ctypes.c_uint64()
    _check(lib().s2dw_workspace_bytes(ctypes.byref(params(L, N, lam, J_min, precision, grid, reality)), count,
                                      ctypes.byref(b)),
           "s2dw_workspace_bytes")
    return b.value


def cache_bytes() -> int:
    """Device bytes held by the library's plans and workspaces."""
    b = ctypes.c_uint64()
    _check(lib().s2dw_cache_bytes(ctypes.byref(b)), "s2dw_cache_bytes")
    return b.value


def profile(enable: bool) -> None:
    """Turn per-kernel stage timing on (clearing totals) or off."""
    _check(lib().s2dw_profile(1 if enable else 0), "s2dw_profile")


def profile_stages(names=None) -> None:
    """Time only the named stages while timing is on (None or empty: every stage)."""
    arg = ",".join(names).encode() if names else None
    _check(lib().s2dw_profile_stages(arg), "s2dw_profile_stages")


def profile_read() -> dict:
    """{stage: (total_ms, launches)} since the last clear (waits for the recorded events)."""
    buf = (StageTime * 64)()
    n = ctypes.c_int32()
    _check(lib().s2dw_profile_read(buf, 64, ctypes.byref(n)), "s2dw_profile_read")
    return {buf[i].name.decode(): (buf[i].ms, buf[i].count) for i in range(min(n.value, 64))}


def release_caches():
    _persist_outs.clear()
    lib().s2dw_release_caches()
