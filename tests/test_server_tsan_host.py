"""The serving form's request loop under the thread sanitizer: the library's
host code and a driver (tests/server_tsan.cpp) that submits, waits and reads
statistics from five threads against a dry server (device -1, no GPU work)
are built with -fsanitize=thread on the host side; the run must finish every
job with no sanitizer report.  The device code is compiled unoptimised, only
to satisfy the link (the dry server launches nothing)."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1705_01813_amd", "csrc")
from paper_1705_01813_amd.build import SOURCES  # every source of the library, so the link is whole

FLAGS = ["--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-std=c++17", "-pthread",
         "-Xarch_host", "-fsanitize=thread", "-Xarch_host", "-g"]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_dry_server_under_thread_sanitizer(tmp_path):
    def compile_one(src):
        out = tmp_path / (os.path.basename(src) + ".o")
        r = subprocess.run(["hipcc", *FLAGS, "-c", src, "-o", str(out)], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return str(out)

    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(HERE, "server_tsan.cpp")]
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = tmp_path / "server_tsan"
    r = subprocess.run(["hipcc", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=thread", "-pthread", *objs, "-o",
                        str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ThreadSanitizer" not in r.stderr
    assert "jobs 160 done, 0 errors" in r.stdout
