"""CPU checks of the C ABI library: it loads, exports every function the
header declares, its structs match the ctypes mirrors, and the host-only
entry points validate their arguments.  No compute call is made."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gslivo.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"GSL_API\s+[\w\s\*]*?\b(gsl_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def abi():
    from paper_2501_08672_amd import _abi, build
    if not os.path.exists(_abi.LIB_PATH):
        build.build()
    return _abi


def test_exports_match_header(abi):
    decl = _declared()
    assert len(decl) >= 12
    assert sorted(abi.EXPORTS) == decl
    out = subprocess.run(["nm", "-D", "--defined-only", abi.LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted(set(re.findall(r" T (gsl_\w+)", out)))
    assert exported == decl
    L = abi.lib()
    for name in decl:
        assert getattr(L, name) is not None


def test_struct_layouts_match_header(abi, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gslivo.h"\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gsl_camera), '
                   'sizeof(gsl_opts), sizeof(gsl_gaussians), sizeof(gsl_splat), sizeof(gsl_proj), sizeof(gsl_bins), '
                   'sizeof(gsl_grads), offsetof(gsl_camera, t_cw), offsetof(gsl_bins, capacity_K), sizeof(gsl_binrec), '
                   'sizeof(gsl_adam), sizeof(gsl_adam_state), offsetof(gsl_adam_state, ld)); return 0;}')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(abi.Camera), C.sizeof(abi.Opts), C.sizeof(abi.Gaussians), abi.SPLAT_BYTES,
            C.sizeof(abi.Proj), C.sizeof(abi.Bins), C.sizeof(abi.Grads), abi.Camera.t_cw.offset,
            abi.Bins.capacity_K.offset, 32, C.sizeof(abi.Adam), C.sizeof(abi.AdamState), abi.AdamState.ld.offset]
    assert got == want


def test_default_opts_and_layout(abi):
    import numpy as np
    import scenegen as S
    o = abi.default_opts(16)
    assert o.tile == 16 and abs(o.alpha_max - 0.99) < 1e-7 and abs(o.T_min - 1e-4) < 1e-10
    assert abs(o.alpha_min - 1 / 255) < 1e-9 and o.near_z > 0
    cams = [S.Camera(100, 100, 64, 48, 128, 96, np.eye(3), np.zeros(3)),
            S.Camera(100, 100, 64, 48, 100, 33, np.eye(3), np.zeros(3))]
    arr = abi.camera_array(cams)
    T, P = C.c_int64(), C.c_int64()
    abi.check(abi.lib().gsl_layout(arr, 2, 16, C.byref(T), C.byref(P)))
    assert T.value == 8 * 6 + 7 * 3 and P.value == 128 * 96 + 100 * 33
    with pytest.raises(abi.GslError) as e:
        abi.check(abi.lib().gsl_layout(arr, 2, 12, C.byref(T), C.byref(P)))
    assert e.value.code == abi.GSL_ENOTSUP
    bad = abi.camera_array([S.Camera(100, 100, 0, 0, 0, 10, np.eye(3), np.zeros(3))])
    with pytest.raises(abi.GslError) as e:
        abi.check(abi.lib().gsl_layout(bad, 1, 16, C.byref(T), C.byref(P)))
    assert e.value.code == abi.GSL_EINVAL
    n = C.c_size_t()
    # sizes are host-only: no context needed
    assert abi.lib().gsl_workspace_size(None, arr, 2, 10, C.byref(o), 100, C.byref(n)) == abi.GSL_OK and n.value > 0
    assert abi.lib().gsl_workspace_size(None, arr, 2, 10, C.byref(o), 100, None) == abi.GSL_EINVAL
    # LDS chunk depth: 0 (tuned or the tile's default), 64, 128 or 256
    assert o.chunk == 0
    for ch, rc in ((64, abi.GSL_OK), (128, abi.GSL_OK), (256, abi.GSL_OK), (96, abi.GSL_EINVAL), (512, abi.GSL_EINVAL)):
        oc = abi.default_opts(16, chunk=ch)
        assert abi.lib().gsl_workspace_size(None, arr, 2, 10, C.byref(oc), 100, C.byref(n)) == rc, ch
    assert abi.lib().gsl_window_variant(None, arr, 2, 10, 16, 0, 64) == abi.GSL_EINVAL
    assert abi.lib().gsl_project(None, None, arr, 2, C.byref(o), None, None, 0, None) == abi.GSL_EINVAL
    assert "NULL" in abi.lib().gsl_last_error().decode()


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle, and the oracle never imports the package."""
    pkg = os.path.join(ROOT, "paper_2501_08672_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"(#|//).*", "", txt).replace("oracle-free", ""), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            assert "paper_2501_08672_amd" not in open(os.path.join(ROOT, "oracle", f)).read(), f
