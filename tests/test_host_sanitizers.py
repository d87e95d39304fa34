"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed):

* the library's host tables (tables.cpp) over a spread of parameters, g++;
* the CPU oracle (orc.c) on small inputs, with its round-trip facts, gcc;
* the library's host code (api.cpp and tables.cpp, the device objects as built) linked into
  a sanitizer build of the library, loaded by a Python process of its own with the sanitizer
  runtime preloaded: every host-only query and every entry point with invalid arguments.

A pass is exit status 0 with no sanitizer report (every check is built with
-fno-sanitize-recover, so a report ends the process with an error)."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1308_5706_amd", "csrc")
HOST = os.path.join(HERE, "host")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(exe, env=None, args=()):
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_host_tables_under_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path / "tables_check")
    subprocess.run([cxx, "-std=c++17", *SAN, "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", f"-I{CSRC}",
                    os.path.join(HOST, "tables_check.cpp"), os.path.join(CSRC, "tables.cpp"), "-o", exe], check=True)
    assert "0 failures" in _run(exe)


def test_oracle_under_sanitizers(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("needs gcc")
    exe = str(tmp_path / "orc_check")
    subprocess.run([cc, "-std=c99", "-fopenmp", *SAN, os.path.join(HOST, "orc_check.c"),
                    os.path.join(ROOT, "oracle", "orc.c"), "-o", exe, "-lm"], check=True)
    assert "0 failures" in _run(exe)


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_library_host_code_under_sanitizers(tmp_path):
    from paper_1308_5706_amd import build as B
    hipcc = B.HIPCC
    rt = _asan_runtime()
    objs = [os.path.join(B.BUILD, n) for n in ("wigner.o", "stages.o", "misc.o", "persist.o")]
    if not os.path.exists(hipcc) or rt is None:
        pytest.skip("needs hipcc and the clang sanitizer runtime")
    if not all(os.path.exists(o) for o in objs):
        B.build()
    host_san = []
    for flag in SAN:  # sanitizers for the host pass only
        host_san += ["-Xarch_host", flag]
    common = ["-x", "hip", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}", "-I", os.path.join(ROOT, "include"),
              "-I", CSRC] + host_san
    san_objs = []
    for src in ("api.cpp", "tables.cpp"):
        o = str(tmp_path / (src + ".o"))
        subprocess.run([hipcc, "-c", os.path.join(CSRC, src), "-o", o] + common, check=True, capture_output=True)
        san_objs.append(o)
    lib = str(tmp_path / "libs2dw_san.so")
    subprocess.run([hipcc, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-o", lib, *san_objs, *objs,
                    "-Xarch_host", "-fsanitize=address,undefined", "-shared-libsan"], check=True, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = _run(sys.executable, env=env, args=(os.path.join(HOST, "abi_check.py"), lib))
    assert "0 failures" in out
