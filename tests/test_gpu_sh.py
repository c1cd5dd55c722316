"""View-dependent colour (SH degrees 1-3, Sec. II-B) and the bilinear colour
initialisation on the GPU against the oracle: per-record colours, images,
gradients (coefficients, means through the view direction, poses through the
camera centre), Adam over the coefficient rows, and gsl_color_init."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import scenegen as S
from scenegen import Camera
from scenegen.scenes import frustum_points

from gpuutil import compare_grads, compare_images, context, gpu_backward, gpu_forward, ops

pytestmark = pytest.mark.gpu


def _cam(W, H, f, seed):
    rng = np.random.default_rng(seed)
    R = Rotation.from_rotvec(rng.normal(0, 0.2, 3)).as_matrix()
    return Camera(f, f * 1.02, W / 2 + 3.3, H / 2 - 2.1, W, H, R, rng.normal(0, 0.3, 3))


def _scene(n, seed, degree):
    cams = [_cam(96, 80, 90.0, seed), _cam(130, 70, 110.0, seed + 1), _cam(64, 64, 60.0, seed + 2)]
    sc = S.random_scene(n, cams[0], seed, zmin=1.0, zmax=4.0, unnormalised_quats=True)
    sc.cams = cams
    return S.with_sh(sc, degree, seed + 7, sigma=0.2)


def _cmax(oracle, sc):
    return max(float(np.abs(oracle.sh_colour(sc, c)).max()) for c in sc.cams)


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_sh_record_colours_match_oracle(oracle, degree):
    sc = _scene(3000, 11 + degree, degree)
    st = gpu_forward(sc, sc.cams)
    f = st["proj"].fields()
    for c, cam in enumerate(sc.cams):
        want = oracle.sh_colour(sc, cam)
        kept = f["depth"][c] > 0
        assert kept.sum() > 100
        got = np.stack([f["r"][c], f["g"][c], f["b"][c]], 1)
        np.testing.assert_allclose(got[kept], want[kept], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("degree,tile", [(1, 16), (2, 8), (3, 32)])
def test_sh_images_match_oracle(oracle, degree, tile):
    sc = _scene(2500, 21, degree)
    bg = (0.2, 0.1, 0.3)
    st = gpu_forward(sc, sc.cams, tile=tile, bg=bg)
    imgs = [t.cpu().numpy() for t in st["cams"].unpack(st["image"])]
    cm = _cmax(oracle, sc)
    for c, cam in enumerate(sc.cams):
        r = oracle.render_image(sc, cam, oracle.Opts(bg=bg))
        compare_images(imgs[c].reshape(3, cam.height, cam.width), r["image"], r["flags"], name=f"cam{c}", bg=bg,
                       cmax=cm)


@pytest.mark.parametrize("degree,tile", [(1, 16), (3, 16), (1, 8), (3, 32)])
def test_sh_gradients_match_oracle(oracle, degree, tile):
    """Coefficients, means (now also through the view direction), colours,
    the other parameters and the camera poses (now also through the camera
    centre), to the gradient tolerance."""
    sc = _scene(2500, 31, degree)
    bg = (0.2, 0.1, 0.3)
    st = gpu_forward(sc, sc.cams, tile=tile, bg=bg)
    rng = np.random.default_rng(5)
    vs = []
    for cam in sc.cams:
        r = oracle.render_image(sc, cam, oracle.Opts(bg=bg))
        v = rng.normal(size=(3, cam.height, cam.width))
        v[:, (r["flags"] & 3) != 0] = 0.0
        vs.append(v)
    v_packed = torch.from_numpy(np.concatenate([v.astype(np.float32).ravel() for v in vs])).cuda()
    gg = gpu_backward(st, v_packed)
    go = oracle.render_bwd(sc, sc.cams, vs, oracle.Opts(bg=bg))
    compare_grads(gg, go, keys=("mean", "scale", "quat", "opacity", "color", "sh", "pose"), name=f"sh{degree} tile {tile}")


def test_sh_window_step_matches_separate_calls():
    """The fused window step with SH colour equals project + bin_sort +
    render_fwd + render_bwd of the same L2 loss, and its graph replays agree."""
    O = ops()
    ctx = context()
    sc = _scene(3000, 41, 3)
    cs = O.CameraSet(sc.cams)
    g = O.Gaussians.from_scene(sc)
    o = O.opts(16)
    tgt_sc = S.jitter_means(sc, 0.02, 3)
    tgt_sc.sh = sc.sh
    gt = O.Gaussians.from_scene(tgt_sc)
    pt = O.project(ctx, gt, cs, o)
    bt = O.bin_sort(ctx, cs, gt.N, o, pt)
    target, _, _ = O.render_fwd(ctx, cs, gt.N, o, pt, bt)
    win = O.Window(ctx, g, cs, o, target, loss="l2", keep_image=True)
    win.step(use_graph=False)
    torch.cuda.synchronize()
    eager = {k: getattr(win.grads, k).clone() for k in ("mean", "color", "sh", "pose")}
    proj = O.project(ctx, g, cs, o)
    bins = O.bin_sort(ctx, cs, g.N, o, proj)
    img, T, nw = O.render_fwd(ctx, cs, g.N, o, proj, bins)
    gr = O.render_bwd(ctx, g, cs, o, proj, bins, T, nw, (img - target).contiguous())
    torch.cuda.synchronize()
    for k in ("mean", "color", "sh"):
        a, b = eager[k], getattr(gr, k)
        assert torch.allclose(a, b, rtol=1e-4, atol=1e-5 * float(b.abs().max())), k
    assert torch.allclose(eager["pose"], gr.pose, rtol=1e-5, atol=1e-6 * float(gr.pose.abs().max()))
    for _ in range(3):
        win.step(use_graph=True)
        torch.cuda.synchronize()
        assert torch.allclose(win.grads.sh, eager["sh"], rtol=1e-5, atol=1e-6 * float(eager["sh"].abs().max()))


def test_sh_adam_rows_match_oracle(oracle):
    """Adam over 14 + 3K raw rows: the SH rows take lr_sh and the identity
    activation; act.sh receives them."""
    O = ops()
    ctx = context()
    N, degree = 4000, 2
    K = O.sh_count(degree)
    rng = np.random.default_rng(12)
    raw = rng.normal(size=(14 + 3 * K, N)).astype(np.float32)
    raw[3:6] = rng.uniform(-4, -1, (3, N))
    st = O.AdamState(torch.from_numpy(raw).cuda())
    assert st.sh_degree == degree
    z = lambda *s: torch.zeros(*s, dtype=torch.float32, device="cuda")
    g = O.Gaussians(z(3, N), z(3, N), z(4, N), z(N), z(3, N), z(3 * K, N))
    grads = O.Grads(N, 1, "cuda", degree)
    lr = (1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3)
    lr_sh = 3e-4
    hp = O.adam_hparams(lr=lr, eps=1e-8, lr_sh=lr_sh)
    f32 = lambda x: float(np.float32(x))
    row_lr = np.array([f32(lr[0])] * 3 + [f32(lr[1])] * 3 + [f32(lr[2])] * 4 + [f32(lr[3])] + [f32(lr[4])] * 3
                      + [f32(lr_sh)] * (3 * K))
    x, m, v = raw.astype(np.float64), np.zeros(raw.shape), np.zeros(raw.shape)
    for t in (1, 2, 3):
        ga = {k: rng.normal(size=(r, N)).astype(np.float32) for k, r in
              (("mean", 3), ("scale", 3), ("quat", 4), ("opacity", 1), ("color", 3), ("sh", 3 * K))}
        for k in ("mean", "scale", "quat", "color", "sh"):
            getattr(grads, k).copy_(torch.from_numpy(ga[k]))
        grads.opacity.copy_(torch.from_numpy(ga["opacity"][0]))
        O.adam_step(ctx, st, hp, grads, g)
        gr = oracle.raw_gradient(x, {k: a.astype(np.float64) for k, a in ga.items()})
        x, m, v = oracle.adam_step(x, m, v, gr, t, row_lr, beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-8))
    torch.cuda.synchronize()
    np.testing.assert_allclose(st.raw.cpu().numpy(), x, rtol=0, atol=1e-5)
    np.testing.assert_allclose(g.sh.cpu().numpy(), x[14:], rtol=0, atol=1e-5)
    np.testing.assert_allclose(g.scale.cpu().numpy(), np.exp(x[3:6]), rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("W,H", [(96, 80), (17, 11)])
def test_color_init_matches_oracle(oracle, W, H):
    """Bilinear colours of means in front of and behind the camera, inside
    and outside the image, on a plain and a strided (capacity) layout."""
    O = ops()
    ctx = context()
    cam = _cam(W, H, 0.9 * W, 61)
    rng = np.random.default_rng(62)
    n = 5000
    pts = frustum_points(rng, cam, n, 0.5, 6.0)
    pts[:300] += rng.normal(0, 3.0, (300, 3))  # some outside the image or behind
    pts = pts.astype(np.float32)
    img = rng.uniform(size=(3, H, W)).astype(np.float32)
    want, ok = oracle.bilinear_colour(pts, cam, img, near_z=0.2)
    assert ok.sum() > 4000 and (~ok).sum() > 10
    o = O.opts(16)
    mean = torch.from_numpy(np.ascontiguousarray(pts.T)).cuda()
    col, valid = O.color_init(ctx, mean, cam, torch.from_numpy(img).cuda(), o)
    torch.cuda.synchronize()
    assert np.array_equal(valid.cpu().numpy().astype(bool), ok)
    np.testing.assert_allclose(col.cpu().numpy().T[ok], want[ok], rtol=0, atol=1e-6)
    assert np.all(col.cpu().numpy().T[~ok] == 0.0)
    # the same into rows of a capacity-strided block (e.g. the window's raw colour rows)
    cap = n + 123
    block = torch.full((17, cap), 7.0, dtype=torch.float32, device="cuda")
    block[0:3, :n] = mean
    col2, valid2 = O.color_init(ctx, block[0:3, :n], cam, torch.from_numpy(img).cuda(), o, color=block[11:14, :n])
    torch.cuda.synchronize()
    got = block[11:14, :n].cpu().numpy().T
    np.testing.assert_array_equal(got[ok], col.cpu().numpy().T[ok])
    assert np.all(got[~ok] == 7.0)
