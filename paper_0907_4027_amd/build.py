"""Build libhot.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_0907_4027_amd.build

Each source is compiled to an object in its own hipcc process (in parallel), then
the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("hot_kernels.hip", "hot_probes.hip", "hot_scratch.hip", "hot_api.cpp")]
OUT = os.path.join(HERE, "libhot.so")
OBJDIR = os.path.join(HERE, "_build")
# packed FP32 (v_pk_*_f32) code generation stays off; the host pass warns that it does
# not know the feature, which is harmless
# kernel arguments: leading scalar and pointer arguments (up to 14 SGPRs) are preloaded at wave
# launch (a kernel whose argument list starts with an aggregate loads them with scalar loads)
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-kernarg-preload-count=16",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    cc = hipcc()
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        objs.append(obj)
        cmds.append([cc, *FLAGS, "-c", src, "-o", obj])
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        results = list(ex.map(_run, cmds))
    for cmd, res in zip(cmds, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {os.path.basename(cmd[-3])}")
        if verbose:
            sys.stdout.write(" ".join(cmd) + "\n")
    tmp = OUT + ".tmp"
    link = [cc, "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp]
    res = _run(link)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to link libhot.so")
    if verbose:
        sys.stdout.write(" ".join(link) + "\n")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
