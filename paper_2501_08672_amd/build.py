"""Builds libgslivo.so (HIP for gfx950) next to this file with hipcc.

Every .hip translation unit and the host ABI (api.cpp) are compiled in
parallel and linked into one shared library that exports the C ABI of
include/gslivo.h.  Packed FP32 instructions are disabled on the device side.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgslivo.so")
OBJ = os.path.join(ROOT, "_build", "obj")
ARCH = os.environ.get("GSL_OFFLOAD_ARCH", "gfx950")

SOURCES = ["project.hip", "sort.hip", "render.hip", "optim.hip", "window.hip", "sh.hip", "noalloc.hip", "probe.hip", "api.cpp"]
# no packed FP32, and no implicit contraction: every fused multiply-add in the
# kernels is written out, so the same expression rounds the same way in every
# kernel and template instantiation
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off"]


def _compile(src):
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", f"--offload-arch={ARCH}", "-I", INC, "-I", CSRC,
           "-Wall", "-Wno-unused-result"]
    if src.endswith(".hip"):
        cmd += DEVICE_FLAGS + ["-munsafe-fp-atomics"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs))
    return out, msgs


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, m in results:
            for ln in m:
                print(ln)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
