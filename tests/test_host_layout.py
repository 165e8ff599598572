"""Host-only graph preparation under the address and undefined-behaviour sanitizers.

Builds tests/host_layout_check.cpp with the library's HIP-free layout module
(paper_1908_00210_amd/csrc/gdi_layout.cpp: CSR validation, first-fit colouring,
colour-major relabelling, the halo layout of the grid sweep) using g++ with
-fsanitize=address,undefined, and runs it: the validator must reject every malformed
CSR with its code, and every generated layout must satisfy the invariants the sweep
kernels rely on (each packed entry names its neighbour's bit in the owner's LDS image,
windows and regions inside the image, chunks partitioning each class). No GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_layout_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path / "host_layout_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Wextra", "-Werror", "-o", exe,
           os.path.join(ROOT, "tests", "host_layout_check.cpp"),
           os.path.join(ROOT, "paper_1908_00210_amd", "csrc", "gdi_layout.cpp")]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stdout + b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
    assert int(r.stdout.split()[1]) > 100  # layouts actually checked
