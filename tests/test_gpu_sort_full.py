"""Tile binning and the depth/tile radix sort (Sec. II-C, tile-based depth
sorting) at the instance counts the benchmark sorts, bit for bit.

At these sizes the radix passes run over more than 1024 blocks of 4096 keys,
so the row scan of the digit-major histogram carries its running total across
several 1024-block chunks: the 500k window at tiles 32 and 16 (15.7M and
39.6M instances) and the 2M / 16-camera uneven batch at tile 16, whose depth
pass alone sorts 32M records.

Checked against the CPU, without reproducing the sort: the instance sequence
is strictly increasing in (tile id, depth bits, Gaussian index), which is the
one sorted order of its own multiset (no two instances share a (tile,
Gaussian) pair); each record's instance count is its tiles_touched; every
instance's tile lies inside its record's bbox tile span; and the ranges are
the first and one-past-last position of every tile.  The uneven batch also
has records whose tile count does not fit beside the record index in the
depth sort's values, so its last pass looks those counts up.
"""
import numpy as np
import pytest

import scenegen as S

from gpuutil import gpu_forward

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _layout(cams, tile):
    tx = np.array([(c.width + tile - 1) // tile for c in cams], np.int64)
    ty = np.array([(c.height + tile - 1) // tile for c in cams], np.int64)
    toff = np.concatenate([[0], np.cumsum(tx * ty)]).astype(np.int64)
    return tx, ty, toff


def _check_full(sc, tile, min_K):
    st = gpu_forward(sc, sc.cams, tile=tile)
    b = st["bins"]
    assert int(b.d_status.item()) == 0
    K = b.K
    f = st["proj"].fields()
    C, N = f["depth"].shape
    print(f"tile {tile}: K = {K}, records C*N = {C * N}")
    assert K >= min_K
    assert K == int(f["tiles_touched"].astype(np.int64).sum())
    tid = b.tile_ids[:K].cpu().numpy().view(np.uint32).astype(np.int64)
    gid = (b.gauss_ids[:K].cpu().numpy().view(np.uint32) & np.uint32((1 << 28) - 1)).astype(np.int64)
    tx, ty, toff = _layout(sc.cams, tile)
    T_total = int(toff[-1])
    assert tid.max() < T_total and gid.max() < N
    cam = np.searchsorted(toff, tid, "right") - 1
    dbits = f["depth"].view(np.uint32)[cam, gid].astype(np.int64)
    del st
    # strictly increasing (tile, depth bits, index)
    dt, dd, dg = np.diff(tid), np.diff(dbits), np.diff(gid)
    up = (dt > 0) | ((dt == 0) & ((dd > 0) | ((dd == 0) & (dg > 0))))
    bad = np.nonzero(~up)[0]
    assert bad.size == 0, f"order broken at {bad[:5]} (K = {K})"
    del dt, dd, dg, up, dbits
    # each record's instance count is its tiles_touched
    cnt = np.bincount(cam * N + gid, minlength=C * N)
    np.testing.assert_array_equal(cnt, f["tiles_touched"].astype(np.int64).ravel())
    del cnt
    # the depth sort carries tile counts in the free high bits of its values
    # (record indices take ceil(log2(C N)) bits); a count that does not fit
    # is looked up by the last pass: how many records took that path
    ib = max(1, int(np.ceil(np.log2(C * N))))
    cap = (1 << (32 - ib)) - 1 if ib <= 28 else 0
    n_lookup = int((f["tiles_touched"] >= cap).sum()) if cap else int((f["tiles_touched"] > 0).sum())
    print(f"tile {tile}: count field cap {cap}, records whose count is looked up {n_lookup}")
    # every instance's tile is inside the bbox tile span of its record
    local = tid - toff[cam]
    ix, iy = local % tx[cam], local // tx[cam]
    bb = f["bbox"].astype(np.int64)
    for k, (lo, hi) in enumerate(((0, 2), (1, 3))):
        v = ix if k == 0 else iy
        assert np.all(bb[cam, gid, lo] // tile <= v) and np.all(v <= bb[cam, gid, hi] // tile), "tile outside bbox"
    del local, ix, iy
    # ranges: first and one-past-last position of every tile (empty tiles start == end)
    rng = b.ranges.cpu().numpy().astype(np.int64)
    starts = np.searchsorted(tid, np.arange(T_total), "left")
    ends = np.searchsorted(tid, np.arange(T_total), "right")
    occ = ends > starts
    np.testing.assert_array_equal(rng[occ, 0], starts[occ])
    np.testing.assert_array_equal(rng[occ, 1], ends[occ])
    assert np.all(rng[~occ, 0] == rng[~occ, 1])
    return K, n_lookup


@pytest.fixture(scope="module")
def window_scene():
    sc, _ = S.config3()
    return sc


@pytest.mark.parametrize("tile,min_K", [(32, 12_000_000), (16, 30_000_000)])
def test_bin_sort_bench_window_bit_exact(window_scene, tile, min_K):
    # more than 1024 blocks of 4096 keys in every tile pass
    _check_full(window_scene, tile, min_K)


def test_bin_sort_uneven_batch_bit_exact():
    sc, _ = S.config5()
    C, N = len(sc.cams), sc.n
    assert C * N > 1024 * 4096 * 4  # the depth pass spans several row-scan chunks
    _, n_lookup = _check_full(sc, 16, 1024 * 4096 + 1)
    # 32M records leave 7 bits for the count: the records of 127 tiles or
    # more take the look-up path of the last depth pass
    assert n_lookup > 0
