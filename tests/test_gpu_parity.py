"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle.

Sizes span several tiles, several radix-sort blocks and ragged tails; the
full-size workloads are checked on sampled pixels the oracle computes one by
one.  Tolerances are the ones stated in tests/gpuutil.py.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen as S
from scenegen import Camera

from gpuutil import (compare_grads, compare_images, context, gpu_backward, gpu_forward, ops, pixel_tolerance,
                     unpack_np)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rot_cam(W, H, f, seed):
    rng = np.random.default_rng(seed)
    R = Rotation.from_rotvec(rng.normal(0, 0.2, 3)).as_matrix()
    return Camera(f, f * 1.02, W / 2 + 3.3, H / 2 - 2.1, W, H, R, rng.normal(0, 0.3, 3))


def _scene_multi(n, seed):
    """A scene seen by three cameras of different sizes and poses."""
    cams = [_rot_cam(96, 80, 90.0, seed), _rot_cam(130, 70, 110.0, seed + 1), _rot_cam(64, 64, 60.0, seed + 2)]
    sc = S.random_scene(n, cams[0], seed, zmin=1.0, zmax=4.0, unnormalised_quats=True)
    sc.cams = cams
    return sc


# ------------------------------------------------------------------ project

@pytest.mark.parametrize("seed", [1, 2])
def test_project_matches_oracle(oracle, seed):
    sc = _scene_multi(3000, seed)
    st = gpu_forward(sc, sc.cams, tile=16)
    f = st["proj"].fields()
    o = oracle.Opts()
    for c, cam in enumerate(sc.cams):
        p = oracle.project(sc, cam, o)
        kept_g = f["depth"][c] > 0               # projected and not culled
        binned = f["tiles_touched"][c] > 0        # reaches at least one tile
        kept_o = (p["status"] & 1) == 1
        # every splat the GPU keeps, the oracle keeps
        assert not np.any(kept_g & ~kept_o)
        assert not np.any(binned & ~kept_g)
        # a splat the oracle keeps but the GPU does not bin cannot reach alpha_min on any pixel
        only_o = np.nonzero(kept_o & ~binned)[0]
        v, u = np.mgrid[0:cam.height, 0:cam.width]
        for i in only_o[:200]:
            A, B, Cc = p["conic"][i]
            dx, dy = u + 0.5 - p["mean2d"][i, 0], v + 0.5 - p["mean2d"][i, 1]
            a = sc.opacity[i] * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + Cc * dy * dy))
            assert a.max() < o.alpha_min
        k = np.nonzero(kept_g)[0]
        np.testing.assert_allclose(f["mx"][c, k], p["mean2d"][k, 0], atol=2e-5 * max(cam.width, 1) / 64 + 1e-5)
        np.testing.assert_allclose(f["my"][c, k], p["mean2d"][k, 1], atol=2e-5 * max(cam.height, 1) / 64 + 1e-5)
        l11, l12, l22 = (f[n][c, k].astype(np.float64) for n in ("l11", "l12", "l22"))
        conic = np.stack([l11 * l11, l11 * l12, l12 * l12 + l22 * l22], 1)
        scale = np.abs(p["conic"][k]).max(1, keepdims=True)
        np.testing.assert_allclose(conic, p["conic"][k], rtol=0, atol=1e-6 * scale.max())
        assert np.all(np.abs(conic - p["conic"][k]) <= 2e-6 * scale)
        z32 = p["p_cam"][k, 2].astype(np.float32)
        assert np.all(np.abs(f["depth"][c, k] - z32) <= np.spacing(z32))
        # bbox is conservative: every pixel with oracle alpha >= alpha_min lies inside it
        bb = f["bbox"][c]
        for i in k[:400]:
            A, B, Cc = p["conic"][i]
            dx, dy = u + 0.5 - p["mean2d"][i, 0], v + 0.5 - p["mean2d"][i, 1]
            a = np.minimum(o.alpha_max, sc.opacity[i] * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + Cc * dy * dy)))
            hit = a >= o.alpha_min * (1 - 1e-6)
            if hit.any():
                uu, vv = u[hit], v[hit]
                assert bb[i, 0] <= uu.min() and uu.max() <= bb[i, 2], (c, i)
                assert bb[i, 1] <= vv.min() and vv.max() <= bb[i, 3], (c, i)
        # tiles touched: at least one, at most the tile span of the bbox
        T = 16
        span = (bb[k, 2] // T - bb[k, 0] // T + 1) * (bb[k, 3] // T - bb[k, 1] // T + 1)
        assert np.all(f["tiles_touched"][c, k] <= span)
        assert np.all(f["tiles_touched"][c, ~kept_g] == 0)


# ------------------------------------------------------------------ bin_sort

F32 = np.float32


def _ellipse_hits_f32(mx, my, l11, l12, l22, kq, x0, x1, y0, y1):
    """CPU recount of the binning rule in float32 (the kernel's operations in
    its order, except that the kernel fuses the two multiply-adds of each
    quadratic form, which moves `best` by about an ulp): minimum of |L d|^2
    over a rectangle of pixel centres, evaluated on the edges that face the
    centre.  Returns (hit, best) so callers can spot boundary cases (within
    1e-5 of kq, far wider than that rounding)."""
    cc = l12 * l12 + l22 * l22
    kv = -(l11 * l12) / cc
    kh = -l12 / l11
    in_x = (mx >= x0) & (mx <= x1)
    in_y = (my >= y0) & (my <= y1)
    best = np.full(np.shape(x0), F32(3.0e38), F32)
    dx = np.where(mx < x0, x0, x1) - mx
    dy = np.minimum(np.maximum(kv * dx, y0 - my), y1 - my)
    u, w = l11 * dx + l12 * dy, l22 * dy
    best = np.where(in_x, best, u * u + w * w)
    dy = np.where(my < y0, y0, y1) - my
    dx = np.minimum(np.maximum(kh * dy, x0 - mx), x1 - mx)
    u, w = l11 * dx + l12 * dy, l22 * dy
    best = np.where(in_y, best, np.minimum(best, u * u + w * w))
    best = np.where(in_x & in_y, F32(0), best)
    return best <= kq, best


def _gpu_instances(st):
    """Per-instance (tile, Gaussian) of the GPU bins, in the GPU's order."""
    b = st["bins"]
    K = b.K
    return (b.tile_ids[:K].cpu().numpy().astype(np.int64),
            b.gauss_ids[:K].cpu().numpy().view(np.uint32).astype(np.int64) & ((1 << 28) - 1))


def _gpu_bands(st):
    b = st["bins"]
    return b.gauss_ids[:b.K].cpu().numpy().view(np.uint32).astype(np.int64) >> 28


def _tile_layout(cams, tile):
    tiles_x = [(c.width + tile - 1) // tile for c in cams]
    tiles_y = [(c.height + tile - 1) // tile for c in cams]
    toff = np.concatenate([[0], np.cumsum([a * b for a, b in zip(tiles_x, tiles_y)])]).astype(np.int64)
    return tiles_x, tiles_y, toff


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_bin_sort_bit_exact(oracle, tile):
    """Binning and sort: the instance count equals the float32 CPU recount of
    the binning rule (exact-boundary cases aside), every tile where the oracle
    sees alpha >= 1/255 is binned, and the instance order is bit-exact against
    a CPU sort of the same (tile, depth bits, index) keys."""
    sc = _scene_multi(6000, 7)
    st = gpu_forward(sc, sc.cams, tile=tile)
    f = st["proj"].fields()
    b = st["bins"]
    K = b.K
    assert int(b.d_status.item()) == 0
    assert K == int(f["tiles_touched"].sum())
    assert K > 3 * 4096  # several radix-sort blocks plus a ragged tail
    tid, gid = _gpu_instances(st)
    bands = _gpu_bands(st)
    tiles_x, tiles_y, toff = _tile_layout(sc.cams, tile)
    T_total = int(toff[-1])
    cam_of = np.searchsorted(toff, tid, "right") - 1
    # 1. the order: (tile, depth bits, index) ascending, bit-exact
    dbits = np.array([f["depth"][c, i].view(np.uint32) for c, i in zip(cam_of, gid)], np.int64)
    order = np.lexsort((gid, dbits, tid))
    np.testing.assert_array_equal(order, np.arange(K))
    # 2. ranges
    rng = b.ranges.cpu().numpy()
    starts = np.searchsorted(tid, np.arange(T_total), "left")
    ends = np.searchsorted(tid, np.arange(T_total), "right")
    np.testing.assert_array_equal(rng[:, 0][ends > starts], starts[ends > starts])
    np.testing.assert_array_equal(rng[:, 1][ends > starts], ends[ends > starts])
    assert np.all(rng[ends == starts, 0] == rng[ends == starts, 1])
    # 3. per (camera, Gaussian) tile sets: counts, recount, conservativeness
    amin = F32(1.0 / 255.0)
    nboundary = 0
    o = oracle.Opts()
    for c, cam in enumerate(sc.cams):
        sel = cam_of == c
        got, band_of = {}, {}
        for t, i, bm in zip(tid[sel], gid[sel], bands[sel]):
            got.setdefault(int(i), set()).add(int(t - toff[c]))
            band_of[(int(i), int(t - toff[c]))] = int(bm)
        tt = f["tiles_touched"][c]
        for i in np.nonzero(tt)[0]:
            assert len(got.get(int(i), ())) == tt[i]
        assert set(got) == set(np.nonzero(tt)[0].tolist())
        p = oracle.project(sc, cam, o)
        v, u = np.mgrid[0:cam.height, 0:cam.width]
        for i in list(got)[:600]:
            bb = f["bbox"][c, i]
            kq = F32(2.0 * np.log(np.float64(f["opacity"][c, i]) / np.float64(amin)) + 0.01)
            tys, txs = np.mgrid[bb[1] // tile:bb[3] // tile + 1, bb[0] // tile:bb[2] // tile + 1]
            txs, tys = txs.ravel(), tys.ravel()
            x0 = (txs * tile).astype(F32) + F32(0.5)
            x1 = np.minimum((txs + 1) * tile, cam.width).astype(F32) - F32(0.5)
            y0 = (tys * tile).astype(F32) + F32(0.5)
            y1 = np.minimum((tys + 1) * tile, cam.height).astype(F32) - F32(0.5)
            hit, best = _ellipse_hits_f32(f["mx"][c, i], f["my"][c, i], f["l11"][c, i], f["l12"][c, i],
                                          f["l22"][c, i], kq, x0, x1, y0, y1)
            want = {int(ty * tiles_x[c] + tx) for tx, ty, h in zip(txs, tys, hit) if h}
            edge = {int(ty * tiles_x[c] + tx) for tx, ty, bq in zip(txs, tys, best)
                    if abs(float(bq) - float(kq)) <= 1e-5 * float(kq)}
            assert (want ^ got[i]) <= edge, (c, i)
            nboundary += len(want ^ got[i])
            # conservative: every pixel where the oracle's alpha reaches 1/255 is in a binned tile
            A, B, Cc = p["conic"][i]
            dx, dy = u + 0.5 - p["mean2d"][i, 0], v + 0.5 - p["mean2d"][i, 1]
            a = sc.opacity[i] * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + Cc * dy * dy))
            hv, hu = np.nonzero(a >= o.alpha_min * (1 - 1e-6))
            need = {int((y // tile) * tiles_x[c] + x // tile) for y, x in zip(hv, hu)}
            assert need <= got[i], (c, i, need - got[i])
            # ... and its part of that tile is marked: the 16x16 quadrant of a
            # 32x32 tile (bit 2 * row half + column half), the 4-row band of a
            # 16x16 tile; 8x8 tiles carry no mask
            for y, x in zip(hv, hu):
                t = int((y // tile) * tiles_x[c] + x // tile)
                bm = band_of[(int(i), t)]
                if tile == 32:
                    assert bm >> int(2 * ((y % 32) // 16) + (x % 32) // 16) & 1, (c, i, t, y, x)
                elif tile == 16:
                    assert bm >> int((y % 16) // 4) & 1, (c, i, t, y)
                else:
                    assert bm == 0
    assert nboundary <= 2


@pytest.mark.parametrize("tile", [8, 32])
def test_bin_sort_large_splats(tile):
    """Splats that span thousands of tiles among many small ones, on a
    1280x1024 and a 320x200 camera: the wave-wide tile expansion runs over many
    steps with records straddling steps.  The count equals the emitted
    instances, the order is bit-exact, and the tile sets of the largest
    splats (and a sample of the rest) equal the float32 recount."""
    cams = [_rot_cam(1280, 1024, 1000.0, 21), _rot_cam(320, 200, 260.0, 22)]
    big = S.random_scene(24, cams[0], 5, zmin=1.0, zmax=3.0, smin=0.3, smax=1.5)
    small = S.random_scene(20000, cams[0], 6, zmin=1.0, zmax=6.0, smin=0.002, smax=0.05)
    sc = S.Scene(np.concatenate([big.mean, small.mean]), np.concatenate([big.scale, small.scale]),
                 np.concatenate([big.quat, small.quat]), np.concatenate([big.opacity, small.opacity]),
                 np.concatenate([big.color, small.color]), cams)
    st = gpu_forward(sc, sc.cams, tile=tile)
    f = st["proj"].fields()
    b = st["bins"]
    K = b.K
    assert int(b.d_status.item()) == 0
    assert K == int(f["tiles_touched"].sum())
    tid, gid = _gpu_instances(st)
    tiles_x, tiles_y, toff = _tile_layout(sc.cams, tile)
    cam_of = np.searchsorted(toff, tid, "right") - 1
    dbits = np.array(f["depth"][cam_of, gid].view(np.uint32), np.int64)
    order = np.lexsort((gid, dbits, tid))
    np.testing.assert_array_equal(order, np.arange(K))
    amin = F32(1.0 / 255.0)
    rng = np.random.default_rng(3)
    nbig = 0
    for c, cam in enumerate(sc.cams):
        sel = cam_of == c
        tsel, gsel = tid[sel] - toff[c], gid[sel]
        tt = f["tiles_touched"][c]
        cand = np.nonzero(tt)[0]
        pick = np.concatenate([cand[cand < 24], rng.choice(cand[cand >= 24], 40, replace=False)])
        for i in pick:
            got = set(tsel[gsel == i].tolist())
            assert len(got) == tt[i]
            bb = f["bbox"][c, i]
            kq = F32(2.0 * np.log(np.float64(f["opacity"][c, i]) / np.float64(amin)) + 0.01)
            tys, txs = np.mgrid[bb[1] // tile:bb[3] // tile + 1, bb[0] // tile:bb[2] // tile + 1]
            txs, tys = txs.ravel(), tys.ravel()
            nbig = max(nbig, len(txs))
            x0 = (txs * tile).astype(F32) + F32(0.5)
            x1 = np.minimum((txs + 1) * tile, cam.width).astype(F32) - F32(0.5)
            y0 = (tys * tile).astype(F32) + F32(0.5)
            y1 = np.minimum((tys + 1) * tile, cam.height).astype(F32) - F32(0.5)
            hit, best = _ellipse_hits_f32(f["mx"][c, i], f["my"][c, i], f["l11"][c, i], f["l12"][c, i],
                                          f["l22"][c, i], kq, x0, x1, y0, y1)
            want = {int(ty * tiles_x[c] + tx) for tx, ty, h in zip(txs, tys, hit) if h}
            edge = {int(ty * tiles_x[c] + tx) for tx, ty, bq in zip(txs, tys, best)
                    if abs(float(bq) - float(kq)) <= 1e-5 * float(kq)}
            assert (want ^ got) <= edge, (c, i)
    assert nbig > 64 * 16  # some record spans many expansion steps


def test_size_limits_rejected():
    """Limits the host checks before any launch: N < 2^28 (the instance id
    keeps 4 band bits), C*N < 2^32, 1 <= C <= 1024, image sides <= 32767,
    tile in {8, 16, 32}, capacity < 2^32; the largest accepted sizes pass."""
    O = ops()
    A = O.A
    ctx = context()
    cams = O.CameraSet([S.Camera(100, 100, 64, 48, 128, 96, np.eye(3), np.zeros(3))])
    o = O.opts(16)

    def code(fn):
        with pytest.raises(A.GslError) as e:
            fn()
        return e.value.code

    assert O.workspace_size(ctx, cams, (1 << 28) - 1, o, 0) > 0
    assert code(lambda: O.workspace_size(ctx, cams, 1 << 28, o, 0)) == A.GSL_EINVAL
    assert code(lambda: O.workspace_size(ctx, cams, -1, o, 0)) == A.GSL_EINVAL
    assert code(lambda: O.workspace_size(ctx, cams, 100, o, 1 << 32)) == A.GSL_EINVAL
    many = O.CameraSet([S.Camera(100, 100, 64, 48, 128, 96, np.eye(3), np.zeros(3))] * 17)
    assert code(lambda: O.workspace_size(ctx, many, (1 << 28) - 1, o, 0)) == A.GSL_EINVAL  # C*N >= 2^32
    too_many = O.CameraSet([S.Camera(100, 100, 4, 4, 8, 8, np.eye(3), np.zeros(3))] * 1025)
    assert code(lambda: O.workspace_size(ctx, too_many, 10, o, 0)) == A.GSL_ENOTSUP
    wide = O.CameraSet([S.Camera(100, 100, 64, 48, 32768, 8, np.eye(3), np.zeros(3))])
    assert code(lambda: O.workspace_size(ctx, wide, 10, o, 0)) == A.GSL_EINVAL
    widest = O.CameraSet([S.Camera(100, 100, 64, 48, 32767, 8, np.eye(3), np.zeros(3))])
    assert O.workspace_size(ctx, widest, 10, o, 0) > 0
    bad = O.opts(16)
    bad.tile = 12
    assert code(lambda: O.workspace_size(ctx, cams, 10, bad, 0)) == A.GSL_ENOTSUP
    bad = O.opts(16)
    bad.alpha_min = 0.995
    assert code(lambda: O.workspace_size(ctx, cams, 10, bad, 0)) == A.GSL_EINVAL


def test_bin_sort_capacity_overflow():
    O = ops()
    sc = _scene_multi(4000, 3)
    ctx = context()
    o = O.opts(16)
    g = O.Gaussians.from_scene(sc)
    cs = O.CameraSet(sc.cams)
    proj = O.project(ctx, g, cs, o)
    small = O.bin_sort(ctx, cs, g.N, o, proj, capacity=100, grow=False)
    torch.cuda.synchronize()
    assert int(small.d_status.item()) == -3  # GSL_ECAPACITY
    K = small.K
    assert K > 100
    full = O.bin_sort(ctx, cs, g.N, o, proj, capacity=K, grow=False)
    assert int(full.d_status.item()) == 0 and full.K == K


# ------------------------------------------------------------------ render_fwd

def test_render_fwd_config1(oracle):
    sc = S.config1()
    st = gpu_forward(sc, sc.cams, tile=16)
    img = unpack_np(st["cams"], st["image"])[0]
    r = oracle.render_image(sc, sc.cams[0], oracle.Opts())
    compare_images(img, r["image"], r["flags"], name="config1")
    T = unpack_np(st["cams"], st["T"], 1)[0]
    ok = r["flags"] == 0
    assert np.abs(T[ok] - r["T"][ok]).max() <= 1e-4


def test_render_fwd_multicam_background(oracle):
    sc = _scene_multi(4000, 11)
    bg = (0.25, 0.5, 0.125)
    st = gpu_forward(sc, sc.cams, tile=16, bg=bg)
    imgs = unpack_np(st["cams"], st["image"])
    for c, cam in enumerate(sc.cams):
        r = oracle.render_image(sc, cam, oracle.Opts(bg=bg))
        compare_images(imgs[c], r["image"], r["flags"], name=f"cam{c}", bg=bg)


def test_render_last_contributor_matches(oracle):
    """The Gaussian at the end of each pixel's walk is the oracle's last contributor."""
    sc = S.config1(seed=3)
    st = gpu_forward(sc, sc.cams, tile=16)
    cam = sc.cams[0]
    nw = unpack_np(st["cams"], st["n_walk"], 1)[0]
    r = oracle.render_image(sc, cam, oracle.Opts())
    rng = st["bins"].ranges.cpu().numpy()
    gids = st["bins"].gauss_ids.cpu().numpy().view(np.uint32) & ((1 << 28) - 1)
    tx = (cam.width + 15) // 16
    ok = r["flags"] == 0
    for v in range(cam.height):
        for u in range(cam.width):
            if not ok[v, u]:
                continue
            t = (v // 16) * tx + u // 16
            n = nw[v, u]
            got = gids[rng[t, 0] + n - 1] if n > 0 else -1
            assert got == r["last"][v, u], (u, v)


def test_render_tile_size_invariance():
    sc = _scene_multi(3000, 5)
    imgs = [gpu_forward(sc, sc.cams, tile=t)["image"].cpu().numpy() for t in (8, 16, 32)]
    np.testing.assert_array_equal(imgs[0], imgs[1])
    np.testing.assert_array_equal(imgs[1], imgs[2])


def test_render_permutation_invariance():
    sc = _scene_multi(3000, 6)
    perm = np.random.default_rng(0).permutation(sc.n)
    sp = sc.permuted(perm)
    sp.cams = sc.cams
    a = gpu_forward(sc, sc.cams)["image"].cpu().numpy()
    b = gpu_forward(sp, sc.cams)["image"].cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_render_config2_sampled(oracle):
    """Full-size 100k / 640x512 workload: 3000 sampled pixels."""
    sc, _ = S.config2()
    st = gpu_forward(sc, sc.cams, tile=16)
    img = unpack_np(st["cams"], st["image"])[0]
    cam = sc.cams[0]
    rng = np.random.default_rng(0)
    pix = np.stack([rng.integers(0, cam.width, 3000), rng.integers(0, cam.height, 3000)], 1).astype(np.int32)
    r = oracle.render(sc, cam, oracle.Opts(), pixels=pix)
    got = img[:, pix[:, 1], pix[:, 0]]
    tl = pixel_tolerance(r["flags"])
    err = np.abs(got.T - r["rgb"]).max(1)
    assert np.all(err <= tl), (err - tl).max()
    print(f"config2 sampled: {int(np.isinf(tl).sum())} flag-1 pixels of {len(tl)}")
    assert np.isinf(tl).sum() <= 0.002 * len(tl) + 1


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_render_stats_counts(oracle, tile):
    """gsl_render_stats: the contributing pairs are the oracle's contributor
    counts summed over pixels (threshold-ambiguous pixels may differ by one
    each); contributors <= backward pairs <= forward pairs evaluated."""
    O = ops()
    sc = S.config1()
    st = gpu_forward(sc, sc.cams, tile=tile)
    ev_f, n_c, ev_b = O.render_stats(st["ctx"], st["cams"], sc.n, st["opts"], st["proj"], st["bins"])
    r = oracle.render_image(sc, sc.cams[0], oracle.Opts())
    amb = int((r["flags"] != 0).sum())
    assert abs(n_c - int(r["n"].sum())) <= amb
    assert n_c <= ev_b <= ev_f
    assert ev_f <= st["bins"].K * tile * tile


def test_render_empty_and_degenerate():
    O = ops()
    # all Gaussians behind the camera: background everywhere, K = 0
    cam = Camera(50.0, 50.0, 20.0, 15.0, 40, 30, np.eye(3), np.zeros(3))
    sc = S.random_scene(500, cam, 1)
    sc.mean[:, 2] = -sc.mean[:, 2]
    st = gpu_forward(sc, [cam], tile=16, bg=(0.1, 0.2, 0.3))
    assert st["bins"].K == 0
    img = unpack_np(st["cams"], st["image"])[0]
    np.testing.assert_allclose(img, np.broadcast_to(np.float32([0.1, 0.2, 0.3])[:, None, None], img.shape))
    # a single-pixel camera and a camera smaller than one tile
    cams = [Camera(5.0, 5.0, 0.5, 0.5, 1, 1, np.eye(3), np.zeros(3)),
            Camera(20.0, 20.0, 3.0, 2.5, 7, 5, np.eye(3), np.zeros(3))]
    sc2 = S.random_scene(300, cams[1], 2, smin=0.05, smax=0.3)
    st2 = gpu_forward(sc2, cams, tile=32)
    assert np.isfinite(st2["image"].cpu().numpy()).all()


# ------------------------------------------------------------------ backward

def _cotangent(oracle, sc, cams, seed, o_kw=None):
    """Random cotangents, zero on pixels the oracle flags as ambiguous."""
    rng = np.random.default_rng(seed)
    vs = []
    for cam in cams:
        r = oracle.render_image(sc, cam, oracle.Opts(**(o_kw or {})))
        v = rng.normal(size=(3, cam.height, cam.width))
        v[:, (r["flags"] & 3) != 0] = 0.0  # alpha-threshold or clamp ambiguity
        vs.append(v)
    return vs


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_render_bwd_config1(oracle, tile):
    sc = S.config1()
    st = gpu_forward(sc, sc.cams, tile=tile)
    vs = _cotangent(oracle, sc, sc.cams, 0)
    v_packed = torch.from_numpy(np.concatenate([v.astype(np.float32).ravel() for v in vs])).cuda()
    gg = gpu_backward(st, v_packed)
    go = oracle.render_bwd(sc, sc.cams, vs, oracle.Opts())
    compare_grads(gg, go, keys=("mean", "scale", "quat", "opacity", "color", "pose"), name=f"config1 tile {tile}")


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_render_bwd_multicam_pose(oracle, tile):
    sc = _scene_multi(2500, 21)
    bg = (0.2, 0.1, 0.3)
    st = gpu_forward(sc, sc.cams, tile=tile, bg=bg)
    vs = _cotangent(oracle, sc, sc.cams, 1, {"bg": bg})
    v_packed = torch.from_numpy(np.concatenate([v.astype(np.float32).ravel() for v in vs])).cuda()
    gg = gpu_backward(st, v_packed)
    go = oracle.render_bwd(sc, sc.cams, vs, oracle.Opts(bg=bg))
    compare_grads(gg, go, keys=("mean", "scale", "quat", "opacity", "color", "pose"), name=f"multicam tile {tile}")


def test_render_bwd_accumulate():
    sc = _scene_multi(1500, 22)
    st = gpu_forward(sc, sc.cams, tile=16)
    v = torch.randn(3 * st["cams"].P_total, device="cuda")
    a = gpu_backward(st, v)
    O = ops()
    gr = O.render_bwd(st["ctx"], st["g"], st["cams"], st["opts"], st["proj"], st["bins"], st["T"], st["n_walk"], v)
    O.render_bwd(st["ctx"], st["g"], st["cams"], st["opts"], st["proj"], st["bins"], st["T"], st["n_walk"], v,
                 accumulate=True, out=gr)
    torch.cuda.synchronize()
    np.testing.assert_allclose(gr.mean.cpu().numpy().T, 2 * a["mean"], rtol=1e-5, atol=1e-6 * np.abs(a["mean"]).max())
    # the 2D gradients come from float atomics, so two runs differ in summation order
    np.testing.assert_allclose(gr.pose.cpu().numpy(), 2 * a["pose"], rtol=1e-5, atol=1e-6 * np.abs(a["pose"]).max())


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_render_bwd_config2_sampled(oracle, tile):
    """Full-size 100k / 640x512 with the cotangent non-zero on 400 sampled pixels."""
    sc, _ = S.config2()
    cam = sc.cams[0]
    st = gpu_forward(sc, sc.cams, tile=tile)
    rng = np.random.default_rng(5)
    pix = np.stack([rng.integers(0, cam.width, 400), rng.integers(0, cam.height, 400)], 1).astype(np.int32)
    pix = np.unique(pix, axis=0)
    r = oracle.render(sc, cam, oracle.Opts(), pixels=pix)
    assert int(((r["flags"] & 1) != 0).sum()) <= 1
    pix = pix[(r["flags"] & 3) == 0]
    v = rng.normal(size=(len(pix), 3))
    vimg = np.zeros((3, cam.height, cam.width), np.float32)
    vimg[:, pix[:, 1], pix[:, 0]] = v.T
    gg = gpu_backward(st, torch.from_numpy(vimg.ravel()).cuda())
    go = oracle.render_bwd(sc, [cam], [v], oracle.Opts(), pixels=[pix])
    compare_grads(gg, go, keys=("mean", "scale", "quat", "opacity", "color", "pose"), name=f"config2 tile {tile}")


# ------------------------------------------------------------------ window

def _window(sc, target_packed, tile, loss, keep_image=True):
    O = ops()
    ctx = context()
    g = O.Gaussians.from_scene(sc)
    cs = O.CameraSet(sc.cams)
    w = O.Window(ctx, g, cs, O.opts(tile), target_packed, loss=loss, keep_image=keep_image)
    return w


def test_window_step_matches_separate_calls():
    """Fused forward + loss gradient + backward equals render_fwd, the loss
    gradient formed on the host side, and render_bwd."""
    sc = _scene_multi(4000, 31)
    tgt_scene = S.jitter_means(sc, 0.02, 5)
    tgt_scene.cams = sc.cams
    tgt = gpu_forward(tgt_scene, sc.cams)["image"]
    for loss in ("l2", "l1"):
        w = _window(sc, tgt, 16, loss)
        w.step(use_graph=False)
        torch.cuda.synchronize()
        st = gpu_forward(sc, sc.cams, tile=16)
        np.testing.assert_array_equal(w.image.cpu().numpy(), st["image"].cpu().numpy())
        r = st["image"] - tgt
        if loss == "l2":
            v = r
            want_loss = 0.5 * float((r.double() ** 2).sum())
        else:
            inv = torch.cat([torch.full((3 * h * wd,), 1.0 / (3 * h * wd), device="cuda")
                             for h, wd in st["cams"].sizes])
            v = torch.sign(r) * inv
            want_loss = float((r.abs().double() * inv.double()).sum())
        gg = gpu_backward(st, v.float())
        got = {"mean": w.grads.mean.cpu().numpy().T, "scale": w.grads.scale.cpu().numpy().T,
               "quat": w.grads.quat.cpu().numpy().T, "opacity": w.grads.opacity.cpu().numpy(),
               "color": w.grads.color.cpu().numpy().T, "pose": w.grads.pose.cpu().numpy()}
        compare_grads(got, gg, rel=1e-5, keys=("mean", "scale", "quat", "opacity", "color", "pose"),
                      elem_rel=1e-4, name=f"window {loss}")
        assert abs(float(w.d_loss.item()) - want_loss) <= 1e-5 * abs(want_loss)


def test_window_graph_replay_and_variants():
    sc = _scene_multi(3000, 41)
    tgt = torch.rand(3 * sum(c.width * c.height for c in sc.cams), device="cuda")
    w = _window(sc, tgt, 16, "l2")
    w.step(use_graph=False)
    torch.cuda.synchronize()
    ref = (w.grads.mean.clone(), w.grads.pose.clone(), w.d_loss.clone(), w.image.clone())
    for _ in range(3):
        w.step(use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(w.image, ref[3])
        assert abs(float(w.d_loss.item()) - float(ref[2].item())) <= 1e-9 * abs(float(ref[2].item()))
        torch.testing.assert_close(w.grads.mean, ref[0], rtol=1e-5, atol=1e-6 * float(ref[0].abs().max()))
        # float32 atomics add the 2D gradients in a different order on every run
        torch.testing.assert_close(w.grads.pose, ref[1], rtol=1e-5, atol=1e-6 * float(ref[1].abs().max()))
        # eager work between replays
        _ = (w.target * 2).sum().item()
    tile, times = w.tune()
    assert tile in (8, 16, 32)
    w.step(use_graph=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(w.image.cpu().numpy(), ref[3].cpu().numpy())


def test_window_graph_follows_new_poses():
    """New keyframe poses replay the cached graph (no new capture) and give
    what an eager step at those poses gives: the camera table is uploaded
    before each launch, not baked into the graph."""
    O = ops()
    sc = _scene_multi(3000, 47)
    tgt = torch.rand(3 * sum(c.width * c.height for c in sc.cams), device="cuda")
    w = _window(sc, tgt, 16, "l1")
    w.step(use_graph=True)
    torch.cuda.synchronize()
    n0 = O.graph_count(w.ctx)
    rng = np.random.default_rng(48)
    for it in range(3):
        for c in range(w.cams.C):
            for j in range(3):
                w.cams.arr[c].t_cw[j] += float(rng.normal(0, 0.01))
        w.step(use_graph=True)
        torch.cuda.synchronize()
        assert w.status() == 0
        assert O.graph_count(w.ctx) == n0, it
        got = (w.image.clone(), float(w.d_loss.item()), w.grads.mean.clone(), w.grads.pose.clone())
        w.step(use_graph=False)
        torch.cuda.synchronize()
        assert torch.equal(got[0], w.image), it
        assert abs(got[1] - float(w.d_loss.item())) <= 1e-9 * abs(got[1])
        torch.testing.assert_close(got[2], w.grads.mean, rtol=1e-5, atol=1e-6 * float(got[2].abs().max()))
        torch.testing.assert_close(got[3], w.grads.pose, rtol=1e-5, atol=1e-6 * float(got[3].abs().max()))


def test_profiled_steps_time_the_same_work():
    """The profiling hook on eager steps and on replays of the profiling
    graph: five positive stage times whose first four add up to the fifth,
    and the same image, loss and gradients as an unprofiled step."""
    sc = _scene_multi(3000, 45)
    tgt = torch.rand(3 * sum(c.width * c.height for c in sc.cams), device="cuda")
    w = _window(sc, tgt, 16, "l1")
    w.step(use_graph=True)
    torch.cuda.synchronize()
    ref = (w.image.clone(), float(w.d_loss.item()), w.grads.mean.clone(), w.grads.pose.clone())
    for graph in (False, True, True):
        ms = w.profiled_step(graph=graph)
        torch.cuda.synchronize()
        assert len(ms) == 5 and all(x > 0.0 for x in ms), ms
        assert abs(sum(ms[:4]) - ms[4]) <= 1e-3 * ms[4] + 2e-3, ms
        assert torch.equal(w.image, ref[0])
        assert abs(float(w.d_loss.item()) - ref[1]) <= 1e-9 * abs(ref[1])
        torch.testing.assert_close(w.grads.mean, ref[2], rtol=1e-5, atol=1e-6 * float(ref[2].abs().max()))
        torch.testing.assert_close(w.grads.pose, ref[3], rtol=1e-5, atol=1e-6 * float(ref[3].abs().max()))
    # the plain graph still runs unprofiled after the profiling graph
    w.step(use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(w.image, ref[0])


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_window_variants_agree(tile):
    """Every fused-kernel variant (plain, persistent, longest first, both,
    XCD-chunked) at every LDS chunk depth gives the same image, loss and
    gradients."""
    sc = _scene_multi(3000, 43)
    tgt = torch.rand(3 * sum(c.width * c.height for c in sc.cams), device="cuda")
    w = _window(sc, tgt, tile, "l1")
    res = []
    for variant, chunk in [(v, ch) for v in range(5) for ch in (64, 128, 256)]:
        w.set_variant(variant, chunk)
        w.step(use_graph=False)
        torch.cuda.synchronize()
        res.append((w.image.clone(), float(w.d_loss.item()), w.grads.mean.clone(), w.grads.pose.clone()))
    for img, loss, gm, gp in res[1:]:
        assert torch.equal(img, res[0][0])
        assert abs(loss - res[0][1]) <= 1e-9 * abs(res[0][1])
        torch.testing.assert_close(gm, res[0][2], rtol=1e-5, atol=1e-6 * float(res[0][2].abs().max()))
        # float32 atomics add the 2D gradients in a variant-dependent order
        torch.testing.assert_close(gp, res[0][3], rtol=1e-5, atol=1e-6 * float(res[0][3].abs().max()))


def test_rasterize_autograd():
    O = ops()
    from paper_2501_08672_amd.autograd import rasterize
    sc = _scene_multi(2000, 51)
    ctx = context()
    cs = O.CameraSet(sc.cams)
    g = O.Gaussians.from_scene(sc)
    params = [t.clone().requires_grad_(True) for t in (g.mean, g.scale, g.quat, g.opacity, g.color)]
    pose = torch.zeros((cs.C, 6), dtype=torch.float64, device="cuda", requires_grad=True)
    img, T = rasterize(*params, cs, ctx, O.opts(16), pose)
    wgt = torch.randn_like(img)
    (img * wgt).sum().backward()
    st = gpu_forward(sc, sc.cams)
    gg = gpu_backward(st, wgt)
    np.testing.assert_allclose(params[0].grad.cpu().numpy().T, gg["mean"], rtol=1e-5,
                               atol=1e-6 * np.abs(gg["mean"]).max())
    np.testing.assert_allclose(pose.grad.cpu().numpy(), gg["pose"], rtol=1e-5, atol=1e-9)


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("variant", [0, 4, 2])
def test_window_step_bins_equal_bin_sort(variant, use_graph):
    """Whatever the fused variant, the window step leaves bins bit-identical
    to gsl_bin_sort's for the same projection."""
    O = ops()
    ctx = context()
    sc = _scene_multi(5000, 61)
    tgt = torch.rand(3 * sum(c.width * c.height for c in sc.cams), device="cuda")
    w = _window(sc, tgt, 16, "l1")
    w.set_variant(variant)
    for _ in range(2):
        w.step(use_graph=use_graph)
    torch.cuda.synchronize()
    assert w.status() == 0
    proj = O.project(ctx, w.g, w.cams, w.opts)
    b = O.bin_sort(ctx, w.cams, w.g.N, w.opts, proj, capacity=w.bins.capacity, grow=False)
    torch.cuda.synchronize()
    K = b.K
    assert w.bins.K == K
    assert torch.equal(w.bins.tile_ids[:K], b.tile_ids[:K])
    assert torch.equal(w.bins.gauss_ids[:K], b.gauss_ids[:K])
    assert torch.equal(w.bins.ranges, b.ranges)


def test_window_step_capacity_overflow():
    """A capacity below the instance count: the window step reports
    GSL_ECAPACITY through the status word and runs to the end; with enough
    capacity the graph path succeeds."""
    O = ops()
    sc = _scene_multi(5000, 62)
    tgt = torch.rand(3 * sum(c.width * c.height for c in sc.cams), device="cuda")
    w = _window(sc, tgt, 16, "l1")
    w.step(use_graph=False)
    torch.cuda.synchronize()
    K = w.bins.K
    for cap in (K // 3, (2 * K) // 3, K - 1):
        w2 = O.Window(w.ctx, w.g, w.cams, w.opts, tgt, loss="l1", capacity=max(cap, 1))
        w2.step(use_graph=False)
        torch.cuda.synchronize()
        assert w2.status() == O.A.GSL_ECAPACITY, cap
    w3 = O.Window(w.ctx, w.g, w.cams, w.opts, tgt, loss="l1", capacity=K)
    w3.step(use_graph=True)
    torch.cuda.synchronize()
    assert w3.status() == 0 and w3.bins.K == K
