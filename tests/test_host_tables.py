"""Host checks of the Wigner-stage recurrence tables (compiled from the library's own
tables.cpp with the host compiler; no device code runs).

The Wigner kernels run the three-term l-recurrence of Delta^l_{m'm} = d^l_{m'm}(pi/2) on
rescaled values D_l = Delta^l / (g_l(m) h_l(m')) whose Delta^{l-1} coefficient is 1.  This
checks, against the recurrence evaluated in long double with coefficients from their
definitions and exact start values, that the rescaled tables give Delta^l_{m'm} as
accurately as the unscaled recurrence, for start values in and below the double range."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1308_5706_amd", "csrc")
SRC = os.path.join(HERE, "host", "rescaled_recurrence.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path_factory.mktemp("host") / "rescaled_recurrence")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", f"-I{CSRC}", SRC,
                    os.path.join(CSRC, "tables.cpp"), "-o", exe], check=True)
    return exe


def run(exe, L, step):
    out = subprocess.run([exe, str(L), str(step)], check=True, capture_output=True, text=True).stdout.split()
    return {out[i]: float(out[i + 1]) for i in range(0, len(out), 2)}


@pytest.mark.parametrize("L,step", [(64, 1), (300, 3), (2048, 41)])
def test_rescaled_recurrence_matches_delta(checker, L, step):
    e = run(checker, L, step)
    assert e["plain"] < 1e-11 and e["xn"] < 1e-11, e
    # no less accurate than the unscaled recurrence on the same double tables
    assert e["plain"] <= 2.0 * e["orig_plain"] + 1e-13, e
    assert e["xn"] <= 4.0 * e["orig_xn"] + 1e-13, e
