"""Builds libgdi.so (HIP kernels + host library) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgdi.so")
SOURCES = [os.path.join(CSRC, "gdi_kernels.hip"), os.path.join(CSRC, "gdi_halo.hip"),
           os.path.join(CSRC, "gdi_learned.hip"), os.path.join(CSRC, "gdi_host.cpp"),
           os.path.join(CSRC, "gdi_layout.cpp"), os.path.join(CSRC, "gdi_tunecache.cpp")]
HEADERS = [os.path.join(CSRC, "gdi_internal.h"), os.path.join(CSRC, "gdi_device.h"),
           os.path.join(CSRC, "gdi_layout.h"), os.path.join(CSRC, "gdi_tunecache.h"),
           os.path.join(HERE, "..", "include", "gdi.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed FP32 instructions are disabled for all device code
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    """Compiles every source into libgdi.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libgdi.so")
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
