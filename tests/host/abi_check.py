"""Host-only calls into a sanitizer build of the library (path in argv[1]): every query that
needs no GPU over a spread of parameters, and every entry point with invalid arguments,
which must be refused before any device work.  Run in a process of its own with the
sanitizer runtime preloaded; prints "abi_check: N failures" and exits with status 0 when N is 0.
No torch import: only ctypes."""
import ctypes
import math
import sys


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("N", ctypes.c_int32), ("lam", ctypes.c_double),
                ("J_min", ctypes.c_int32), ("grid", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reality", ctypes.c_int32)]


class Group(ctypes.Structure):
    _fields_ = [("params", Params), ("count", ctypes.c_int32), ("flm", ctypes.c_void_p), ("W", ctypes.c_void_p),
                ("Wphi_lm", ctypes.c_void_p)]


def main():
    lib = ctypes.CDLL(sys.argv[1])
    for f in ("s2dw_analysis", "s2dw_synthesis", "s2dw_analysis_batched", "s2dw_synthesis_batched", "s2dw_scaling",
              "s2dw_steer", "s2dw_sht_forward", "s2dw_sht_inverse", "s2dw_analysis_noalloc", "s2dw_autotune",
              "s2dw_workspace_bytes"):
        getattr(lib, f).restype = ctypes.c_int
    lib.s2dw_strerror.restype = ctypes.c_char_p
    fails = 0
    vp = ctypes.c_void_p
    i32 = ctypes.c_int32
    # host-only queries over a spread of parameters (and the refused ones)
    for L in (2, 3, 17, 64, 255, 1024, 2048, 5000):
        for N in (1, 2, 5, 16, 17):
            for lam in (1.0, 1.5, 2.0, 3.0, math.inf, math.nan):
                for J_min in (-1, 0, 1, 3, 12):
                    for grid in (0, 1, 2, 3):
                        p = Params(L, N, lam, J_min, grid, 0, 1)
                        S = i32()
                        lib.s2dw_num_scales(ctypes.byref(p), ctypes.byref(S))
                        sh = (i32 * 3)()
                        lib.s2dw_grid_shape(ctypes.byref(p), sh)
                        b = ctypes.c_uint64()
                        lib.s2dw_wavelet_bytes(ctypes.byref(p), ctypes.byref(b))
                        off = ctypes.c_uint64()
                        for j in (-1, 0, 2, 40):
                            lib.s2dw_scale_grid(ctypes.byref(p), j, sh, ctypes.byref(off))
                        # invalid arguments: refused before device work (null / misaligned /
                        # bad values); valid parameters with null outputs are refused too
                        fake, odd = vp(0x1000), vp(0x1003)
                        if lib.s2dw_analysis(ctypes.byref(p), None, fake, None, None) == 0:
                            fails += 1
                        if lib.s2dw_analysis(ctypes.byref(p), odd, fake, None, None) == 0:
                            fails += 1
                        if lib.s2dw_synthesis(ctypes.byref(p), fake, None, None, None) == 0:
                            fails += 1
                        if lib.s2dw_analysis_batched(ctypes.byref(p), 0, fake, fake, None, None) == 0:
                            fails += 1
                        if lib.s2dw_synthesis_batched(ctypes.byref(p), -3, fake, None, fake, None) == 0:
                            fails += 1
                        if lib.s2dw_steer(ctypes.byref(p), 1, fake, -1, fake, fake, None) == 0:
                            fails += 1
                        if lib.s2dw_scaling(ctypes.byref(p), None, fake, None, None) == 0:
                            fails += 1
                        if lib.s2dw_analysis_noalloc(ctypes.byref(p), odd, fake, None, None) == 0:
                            fails += 1
                        if lib.s2dw_autotune(ctypes.byref(p), 0, None, None, None) == 0:
                            fails += 1
    for L in (1, 5000):
        p = Params(L, 1, 2.0, 0, 0, 0, 1)
        if lib.s2dw_sht_forward(ctypes.byref(p), vp(0x1000), vp(0x1000), None) == 0:
            fails += 1
        if lib.s2dw_sht_inverse(ctypes.byref(p), vp(0x1000), vp(0x1000), None) == 0:
            fails += 1
    # persistent batches refused before any device work (bad groups, mixed precisions, what
    # the executor does not run), and the wait-bound setting
    for f in ("s2dw_analysis_persistent", "s2dw_synthesis_persistent"):
        fn = getattr(lib, f)
        fn.restype = ctypes.c_int
        for gl in ([], [(0, 1, 0, 0x1000)], [(1, 1, 0, 0x1004)], [(1, 1, 0, 0x1000), (1, 1, 1, 0x1000)],
                   [(1, 0, 0, 0x1000)], [(1, 1, 0, 0x1000), (0, 1, 0, 0x1000)]):
            arr = (Group * max(len(gl), 1))()
            for i, (count, reality, precision, ptr) in enumerate(gl):
                arr[i].params = Params(32, 4, 2.0, 0, 0, precision, reality)
                arr[i].count, arr[i].flm, arr[i].W = count, ptr, ptr
            if fn(arr, len(gl), None, None) == 0:
                fails += 1
        if fn(None, 1, None, None) == 0:
            fails += 1
    if lib.s2dw_persistent_wait_bound(-1, 0) == 0 or lib.s2dw_persistent_wait_bound(1, 3) == 0:
        fails += 1
    if lib.s2dw_persistent_wait_bound(0, 0) != 0:
        fails += 1
    # wavelet tables into host buffers
    for (L, N) in ((8, 1), (33, 4), (64, 16)):
        p = Params(L, N, 2.0, 0, 0, 0, 1)
        S = i32()
        lib.s2dw_num_scales(ctypes.byref(p), ctypes.byref(S))
        kap = (ctypes.c_double * (S.value * L))()
        phi = (ctypes.c_double * L)()
        sln = (ctypes.c_double * (2 * L * (2 * N - 1)))()
        if lib.s2dw_wavelet_tables(ctypes.byref(p), kap, phi, sln) != 0:
            fails += 1
    # stage selection names and status texts
    for names in (b"beta_adj,wigner_fwd", b"", None, b"nope", b"beta_adj,,pad", b"x" * 5000):
        lib.s2dw_profile_stages(names)
    lib.s2dw_profile_stages(None)
    for code in range(-8, 2):
        if not lib.s2dw_strerror(code):
            fails += 1
    print(f"abi_check: {fails} failures", flush=True)
    sys.exit(0 if fails == 0 else 1)


if __name__ == "__main__":
    main()
