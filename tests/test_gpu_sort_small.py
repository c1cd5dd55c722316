"""Binning of small windows (Sec. II-C, tile-based depth sorting): up to
16384 records one workgroup sorts them by depth, drops those that reach no
tile and scans their tile counts in one launch, and up to an instance
capacity of 16384 one workgroup sorts the instances by tile.

Checked as the full-size sorts are (the instance sequence strictly
increasing in (tile id, depth bits, Gaussian index), each record's instance
count its tiles_touched, the ranges the first and one-past-last position of
every tile), and against the multi-block tile sort of the same records (a
capacity above the one-workgroup bound), bit for bit.  Record counts on both
sides of the bound (16384 and 16385) and a window where nothing reaches a
tile are included.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen as S
from scenegen import Camera

from gpuutil import context, ops

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ONE_BLOCK = 16384


def _cam(W, H, f, seed):
    rng = np.random.default_rng(seed)
    R = Rotation.from_rotvec(rng.normal(0, 0.2, 3)).as_matrix()
    return Camera(f, f * 1.02, W / 2 + 3.3, H / 2 - 2.1, W, H, R, rng.normal(0, 0.3, 3))


def _bins(sc, tile, capacity):
    O = ops()
    ctx = context()
    o = O.opts(tile)
    g = O.Gaussians.from_scene(sc)
    cs = O.CameraSet(sc.cams)
    proj = O.project(ctx, g, cs, o)
    b = O.bin_sort(ctx, cs, g.N, o, proj, capacity=capacity, grow=False)
    torch.cuda.synchronize()
    assert int(b.d_status.item()) == 0
    K = b.K
    return (proj.fields(), K, b.tile_ids[:K].cpu().numpy().view(np.uint32).astype(np.int64),
            b.gauss_ids[:K].cpu().numpy().view(np.uint32).astype(np.int64), b.ranges.cpu().numpy().astype(np.int64))


def _check(sc, tile, f, K, tid, graw, rng):
    C, N = f["depth"].shape
    assert K == int(f["tiles_touched"].astype(np.int64).sum())
    tx = np.array([(c.width + tile - 1) // tile for c in sc.cams], np.int64)
    ty = np.array([(c.height + tile - 1) // tile for c in sc.cams], np.int64)
    toff = np.concatenate([[0], np.cumsum(tx * ty)]).astype(np.int64)
    T_total = int(toff[-1])
    gid = graw & ((1 << 28) - 1)
    if K:
        assert tid.max() < T_total and gid.max() < N
        cam = np.searchsorted(toff, tid, "right") - 1
        dbits = f["depth"].view(np.uint32)[cam, gid].astype(np.int64)
        dt, dd, dg = np.diff(tid), np.diff(dbits), np.diff(gid)
        up = (dt > 0) | ((dt == 0) & ((dd > 0) | ((dd == 0) & (dg > 0))))
        assert np.all(up), f"order broken at {np.nonzero(~up)[0][:5]}"
        cnt = np.bincount(cam * N + gid, minlength=C * N)
        np.testing.assert_array_equal(cnt, f["tiles_touched"].astype(np.int64).ravel())
    starts = np.searchsorted(tid, np.arange(T_total), "left")
    ends = np.searchsorted(tid, np.arange(T_total), "right")
    occ = ends > starts
    np.testing.assert_array_equal(rng[occ, 0], starts[occ])
    np.testing.assert_array_equal(rng[occ, 1], ends[occ])
    assert np.all(rng[~occ, 0] == rng[~occ, 1])


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_one_block_sorts_match_multi_block(tile):
    cams = [_cam(96, 80, 90.0, 41), _cam(130, 70, 110.0, 42), _cam(64, 64, 60.0, 43)]
    sc = S.random_scene(1200, cams[0], 44, zmin=1.0, zmax=4.0)
    sc.cams = cams
    f, K, tid, gid, rng = _bins(sc, tile, ONE_BLOCK)            # both sorts in one workgroup
    print(f"tile {tile}: records {len(cams) * sc.n}, K = {K}")
    assert 0 < K <= ONE_BLOCK
    _check(sc, tile, f, K, tid, gid, rng)
    # the instances by the multi-block sort, and by the one-workgroup sort
    # sized for the capacity just above K (fewer keys per lane)
    for cap in (4 * ONE_BLOCK, K + 1):
        f2, K2, tid2, gid2, rng2 = _bins(sc, tile, cap)
        assert K2 == K
        np.testing.assert_array_equal(tid2, tid)
        np.testing.assert_array_equal(gid2, gid)              # tile parts included
        np.testing.assert_array_equal(rng2, rng)


@pytest.mark.parametrize("n", [700, 1024, 1025, 3000, 7000, ONE_BLOCK, ONE_BLOCK + 1])
def test_depth_sort_at_the_one_block_bound(n):
    # one camera: n records, the depth sort in one workgroup for n <= 16384
    # (with 1, 2, 4, 8 or 16 keys per lane), by the multi-block sort above
    cam = _cam(160, 120, 140.0, 51)
    sc = S.random_scene(n, cam, 52, zmin=1.0, zmax=6.0, smin=0.002, smax=0.02)
    sc.cams = [cam]
    f, K, tid, gid, rng = _bins(sc, 16, 1 << 18)
    print(f"records {n}: K = {K}")
    assert K > 0
    _check(sc, 16, f, K, tid, gid, rng)


def test_one_block_sort_nothing_binned():
    cam = _cam(64, 48, 60.0, 61)
    sc = S.random_scene(500, cam, 62, zmin=1.0, zmax=4.0)
    sc.mean = sc.mean.copy()
    sc.mean[:, 2] = -5.0  # every Gaussian behind the camera
    sc.cams = [cam]
    f, K, tid, gid, rng = _bins(sc, 16, ONE_BLOCK)
    assert K == 0
    _check(sc, 16, f, K, tid, gid, rng)


def test_one_block_tile_sort_over_capacity():
    # more instances than capacity: the emission writes none, the status says
    # so, and every tile's range is empty (nothing reads the unwritten ids)
    cams = [_cam(96, 80, 90.0, 71)]
    sc = S.random_scene(1500, cams[0], 72, zmin=1.0, zmax=4.0)
    sc.cams = cams
    O = ops()
    ctx = context()
    o = O.opts(16)
    g = O.Gaussians.from_scene(sc)
    cs = O.CameraSet(sc.cams)
    proj = O.project(ctx, g, cs, o)
    K = int(proj.fields()["tiles_touched"].astype(np.int64).sum())
    assert K > 2
    b = O.bin_sort(ctx, cs, g.N, o, proj, capacity=K // 2, grow=False)
    torch.cuda.synchronize()
    assert int(b.d_status.item()) == O.A.GSL_ECAPACITY
    assert b.K == K
    assert not b.ranges.cpu().numpy().any()
