"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds are made in a temporary directory and exercised by
tests/_sanitize_driver.py in a child process with the sanitizer runtime
preloaded:

* the oracle (gsl_oracle.c) with gcc, -fsanitize=address,undefined: a small
  scene's projection, image, adjoint, pose Jacobians (SH colour) and a pixel
  trace;
* the C ABI library with api.cpp's host code built by hipcc with the same
  sanitizers for the host pass only (the device objects are the plain
  build's): camera layouts and workspace sizes of every workload at every
  tile size, rejected shapes, the camera->IMU twist map, both IESKF updates,
  NULL-argument rejection by every device entry point and context creation
  without a GPU.

Any sanitizer report aborts the child (no recovery); the results must also
equal the plain builds' (the same host code at another optimisation level).
"""
import glob
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "_sanitize_driver.py")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(mode, lib, preload=None):
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    if preload:
        env.update(SAN_ENV)
        env["LD_PRELOAD"] = preload
    r = subprocess.run([sys.executable, DRIVER, mode, lib], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, f"{mode} {lib}: rc {r.returncode}\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    for bad in ("AddressSanitizer", "runtime error:", "UndefinedBehaviorSanitizer"):
        assert bad not in r.stderr, r.stderr[-6000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT ")]
    assert line, r.stdout[-2000:]
    return json.loads(line[-1][len("RESULT "):])


def _close(a, b, path=""):
    if isinstance(a, dict):
        assert sorted(a) == sorted(b), path
        for k in a:
            _close(a[k], b[k], f"{path}.{k}")
    elif isinstance(a, list):
        assert len(a) == len(b), path
        for k, (x, y) in enumerate(zip(a, b)):
            _close(x, y, f"{path}[{k}]")
    elif isinstance(a, float):
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (path, a, b)
    else:
        assert a == b, (path, a, b)


def test_oracle_under_asan_ubsan(tmp_path):
    from oracle import oracle as O
    plain = O.build(force=False)
    lib = str(tmp_path / "libgsl_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", lib, O._SRC, "-lm"])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    got = _run("oracle", lib, preload=asan)
    want = _run("oracle", plain)
    _close(got, want)


def test_abi_host_code_under_asan_ubsan(tmp_path):
    from paper_2501_08672_amd import _abi, build
    if not os.path.exists(_abi.LIB_PATH) or not all(
            os.path.exists(os.path.join(build.OBJ, os.path.splitext(s)[0] + ".o")) for s in build.SOURCES):
        build.build()
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("clang AddressSanitizer runtime not found")
    api_o = str(tmp_path / "api_san.o")
    subprocess.check_call(["hipcc", "-O1", "-g", "-std=c++17", "-fPIC", "-fvisibility=hidden",
                           f"--offload-arch={build.ARCH}", "-I", build.INC, "-I", build.CSRC,
                           "-Xarch_host", "-fsanitize=address,undefined",
                           "-Xarch_host", "-fno-sanitize-recover=undefined",
                           "-Xarch_host", "-fno-omit-frame-pointer",
                           "-c", os.path.join(build.CSRC, "api.cpp"), "-o", api_o])
    objs = [os.path.join(build.OBJ, os.path.splitext(s)[0] + ".o") for s in build.SOURCES if s != "api.cpp"]
    lib = str(tmp_path / "libgslivo_san.so")
    subprocess.check_call(["hipcc", "-shared", "-fPIC", f"--offload-arch={build.ARCH}",
                           "-Xarch_host", "-fsanitize=address,undefined", "-shared-libasan",
                           "-o", lib, api_o] + objs)
    got = _run("abi", lib, preload=rts[-1])
    want = _run("abi", _abi.LIB_PATH)
    _close(got, want)
    # sanity of what was exercised
    assert got["null_gsl_render_bwd_noalloc"][0] == -1 and got["vis_bad"] == -1
    assert got["layout_c3_32"][:3] == [0, 0, 0] and got["layout_c3_32"][3] == 8 * 40 * 32
    assert got["bad_tile"][0] == -2 and "tile size 12" in got["bad_tile"][1]
