"""Build the HIP library for gfx950 (hipcc cross-compiles; no GPU needed)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libtron_mi355x.so")
OBJDIR = os.path.join(LIBDIR, "obj")
SOURCES = ["tron_lib.hip", "lane_br6.hip", "admm.hip", "server.hip", "design.hip", "group.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are switched off for the device code (the host pass of hipcc
# reports that it does not know the feature; the device pass applies it: a float2
# multiply-add compiles to v_pk_fma_f32 without the flag and to v_fma_f32 with it).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# Every source uses the compiler's default instruction scheduler: its alternatives
# (max-ilp, iterative-ilp, max-memory-clause) were measured within 1.5 % of it either way
# on the lane, wave and persistent kernels, none better across them.


def _compile(src, extra):
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *(extra or []), "-c", "-o", obj, os.path.join(CSRC, src)]
    out = subprocess.run(cmd, capture_output=True, text=True)
    if out.returncode != 0:
        raise RuntimeError("HIP build failed:\n" + " ".join(cmd) + "\n" + out.stderr[-20000:])
    return obj, out.stderr


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source (in parallel, one process each) and link the shared library."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    if verbose:
        for _, err in results:
            if err:
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    out = subprocess.run(cmd, capture_output=True, text=True)
    if out.returncode != 0:
        raise RuntimeError("HIP link failed:\n" + " ".join(cmd) + "\n" + out.stderr[-20000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
