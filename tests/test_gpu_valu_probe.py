"""gsl_valu_probe, the measurement aid behind the compositing kernels'
roofline: finite positive issue rates for every instruction kind, single-cycle
integer min + add issuing at least as fast as fused multiply-adds, and the
host-side rejection of a bad mode and of a host sink pointer."""
import ctypes as C

import pytest

from gpuutil import context, ops

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_probe_rates():
    O = ops()
    ctx = context()
    r = {m: O.valu_probe(ctx, m) for m in O.VALU_PROBE_MODES}
    print("wave64 VALU instructions per CU per 2.4-GHz cycle:", r)
    for m, v in r.items():
        assert 0.05 < v < 16.0, (m, v)
    assert r["umin_add"] >= 0.9 * r["fma"]
    assert r["add"] >= 0.9 * r["fma"]


def test_probe_rejects_bad_arguments():
    from paper_2501_08672_amd import _abi as A
    ctx = context()
    sink = torch.zeros(1, device="cuda")
    out = C.c_double()
    L = A.lib()
    assert L.gsl_valu_probe(ctx.h, 5, C.c_void_p(sink.data_ptr()), C.byref(out)) == A.GSL_EINVAL
    assert "mode" in L.gsl_last_error().decode()
    host = (C.c_float * 1)()
    assert L.gsl_valu_probe(ctx.h, 0, C.cast(host, C.c_void_p), C.byref(out)) == A.GSL_EINVAL
    assert "device memory" in L.gsl_last_error().decode()
