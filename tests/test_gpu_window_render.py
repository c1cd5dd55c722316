"""gsl_window_render, the forward render of a camera set as one unit: the
same projection, binning and compositing as gsl_project + gsl_bin_sort +
gsl_render_fwd, so every output (records, instance lists and ranges, image,
final transmittance, walk lengths) is bit-identical to those three calls',
eager and replayed as a HIP graph; new poses replay the cached graph and give
the three calls' result at those poses; the 1k / 128x96 forward workload."""
import numpy as np
import pytest

import scenegen as S

from gpuutil import context, ops
from test_gpu_parity import _scene_multi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _three_calls(O, ctx, g, cams, o, capacity):
    proj = O.project(ctx, g, cams, o)
    bins = O.bin_sort(ctx, cams, g.N, o, proj, capacity=capacity)
    image, T, nw = O.render_fwd(ctx, cams, g.N, o, proj, bins)
    torch.cuda.synchronize()
    return proj, bins, image, T, nw


def _same(r, ref):
    proj, bins, image, T, nw = ref
    assert r.status() == 0
    K = bins.K
    assert r.bins.K == K
    assert torch.equal(r.image, image)
    assert torch.equal(r.T_final, T)
    assert torch.equal(r.n_walk, nw)
    assert torch.equal(r.bins.tile_ids[:K], bins.tile_ids[:K])
    assert torch.equal(r.bins.gauss_ids[:K], bins.gauss_ids[:K])
    assert torch.equal(r.bins.ranges, bins.ranges)
    for name in ("splats", "binrecs", "depth_keys", "tiles_touched"):
        assert torch.equal(getattr(r.proj, name), getattr(proj, name)), name


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_window_render_is_the_three_calls(tile):
    O = ops()
    ctx = context()
    sc = _scene_multi(4000, 61)
    g, cams, o = O.Gaussians.from_scene(sc), O.CameraSet(sc.cams), O.opts(tile, bg=(0.1, 0.2, 0.3))
    r = O.WindowRender(ctx, g, cams, o)
    ref = _three_calls(O, ctx, g, cams, o, r.bins.capacity)
    r(use_graph=False)
    torch.cuda.synchronize()
    _same(r, ref)
    r(use_graph=True)
    torch.cuda.synchronize()
    n0 = O.graph_count(ctx)
    _same(r, ref)
    r(use_graph=True)  # a replay: no new graph
    torch.cuda.synchronize()
    assert O.graph_count(ctx) == n0
    _same(r, ref)


def test_window_render_sh_colour():
    """SH degree 3 colour (evaluated in the projection) through the recorded
    unit: bit-identical to the three calls."""
    O = ops()
    ctx = context()
    sc = S.with_sh(_scene_multi(3000, 64), 3, 65)
    g, cams, o = O.Gaussians.from_scene(sc), O.CameraSet(sc.cams), O.opts(32)
    r = O.WindowRender(ctx, g, cams, o)
    for _ in range(2):
        r(use_graph=True)
    torch.cuda.synchronize()
    _same(r, _three_calls(O, ctx, g, cams, o, r.bins.capacity))


def test_window_render_graph_follows_new_poses():
    O = ops()
    ctx = context()
    sc = _scene_multi(3000, 62)
    g, cams, o = O.Gaussians.from_scene(sc), O.CameraSet(sc.cams), O.opts(16)
    r = O.WindowRender(ctx, g, cams, o, headroom=2.0)
    r(use_graph=True)
    torch.cuda.synchronize()
    n0 = O.graph_count(ctx)
    rng = np.random.default_rng(63)
    for it in range(3):
        for c in range(cams.C):
            for j in range(3):
                cams.arr[c].t_cw[j] += float(rng.normal(0, 0.01))
        r(use_graph=True)
        torch.cuda.synchronize()
        assert O.graph_count(ctx) == n0, it
        _same(r, _three_calls(O, ctx, g, cams, o, r.bins.capacity))


def test_window_render_forward_workload():
    """1,000 Gaussians, one 128x96 camera, tile 16: the graph's image equals
    the three calls' bit for bit."""
    O = ops()
    ctx = context()
    sc = S.config1()
    g, cams, o = O.Gaussians.from_scene(sc), O.CameraSet(sc.cams), O.opts(16)
    r = O.WindowRender(ctx, g, cams, o)
    for _ in range(2):
        r(use_graph=True)
    torch.cuda.synchronize()
    _same(r, _three_calls(O, ctx, g, cams, o, r.bins.capacity))
