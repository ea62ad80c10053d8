"""Build libhot.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_0907_4027_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, "hot_kernels.hip"), os.path.join(CSRC, "hot_api.cpp")]
OUT = os.path.join(HERE, "libhot.so")
# packed FP32 (v_pk_*_f32) code generation stays off; the host pass warns that it does
# not know the feature, which is harmless
# kernel arguments: the first 16 SGPRs' worth are preloaded at wave launch (no scalar load
# to wait for before the first memory reads of a kernel)
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-kernarg-preload-count=16",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    cmd = [hipcc(), *FLAGS, *SOURCES, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libhot.so")
    if verbose:
        sys.stdout.write(" ".join(cmd) + "\n")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
