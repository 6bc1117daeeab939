"""The 128-bit fixed-point conversions of the incremental centroid update
(composite vectors D_r of Eqn. 2), compiled for the host from the same header
the HIP kernels use and checked against 128-bit integer arithmetic: exact
truncation of a double times 2^s, and correct rounding back to double.  The
same harness also checks the earlier 64-bit-shift form of the conversion,
and runs once more under the address and undefined-behaviour sanitizers."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("flags", [["-O2"], ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]],
                         ids=["plain", "asan_ubsan"])
def test_fixed128_conversions_exact(tmp_path, flags):
    exe = tmp_path / "fixed128_check"
    subprocess.run(["g++", *flags, "-std=c++17", os.path.join(HERE, "fixed128_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe), "2000000"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mismatches 0, fx_to_double mismatches 0, shift64 form mismatches 0" in r.stdout
    assert "runtime error" not in r.stderr
