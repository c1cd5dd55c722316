"""GPU checks at the full sizes of the larger workloads, through the C ABI.

* 200k surfels, 640x512, 32 perturbed poses batched: the pose gradient of
  1/2 sum r^2 (r = render at the perturbed pose - render at the true pose)
  against the oracle on sampled pixels, and against central differences of
  the twist evaluated with the GPU forward.
* 500k surfels, 8 keyframes 1280x1024: sampled pixels of the window image and
  the gradient of a sparse cotangent against the oracle.
* 2M surfels, 16 cameras 320x256 .. 1920x1080: sampled pixels against the
  oracle, and the batched window step against per-camera steps.
* the benchmark's launch configuration (500k, 8 x 1280x1024, tile 32, fused
  window step replayed as a graph): its image equals gsl_render_fwd's bit for
  bit and its gradients equal gsl_render_bwd's with the loss cotangent; the
  same window with SH degree 3 colour on sampled pixels against the oracle.
* the window update at its benchmark size (500k Gaussians, 100k points per
  frame), two frames, bit for bit against the oracle.
"""
import numpy as np
import pytest

import scenegen as S

from gpuutil import compare_grads, context, gpu_backward, gpu_forward, ops, pixel_tolerance, unpack_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _sample(cam, n, rng):
    p = np.stack([rng.integers(0, cam.width, n), rng.integers(0, cam.height, n)], 1).astype(np.int32)
    return np.unique(p, axis=0)


@pytest.fixture(scope="module")
def pose_batch():
    sc, true_cam, cams, tw = S.config4()
    ref = gpu_forward(sc, [true_cam], tile=16)
    I_true = unpack_np(ref["cams"], ref["image"])[0]
    st = gpu_forward(sc, cams, tile=16)
    return sc, true_cam, cams, tw, I_true, st


def test_pose_batch_vs_oracle(oracle, pose_batch):
    """32 poses in one batch; cotangent r = I(T_pert) - I(T_true) on 96 sampled
    pixels per pose (oracle-unambiguous ones), elsewhere 0."""
    sc, true_cam, cams, tw, I_true, st = pose_batch
    rng = np.random.default_rng(1)
    imgs = unpack_np(st["cams"], st["image"])
    vs, pix_list, v_packed = [], [], []
    sel = [0, 5, 11, 17, 23, 31]  # oracle on a subset of the 32 poses keeps the test short
    for c, cam in enumerate(cams):
        v = np.zeros((3, cam.height, cam.width), np.float32)
        if c in sel:
            pix = _sample(cam, 96, rng)
            r = oracle.render(sc, cam, oracle.Opts(), pixels=pix)
            pix = pix[(r["flags"] & 3) == 0]
            res = imgs[c][:, pix[:, 1], pix[:, 0]] - I_true[:, pix[:, 1], pix[:, 0]]
            v[:, pix[:, 1], pix[:, 0]] = res
            vs.append(res.T.astype(np.float64))
            pix_list.append(pix)
        v_packed.append(v.ravel())
    gg = gpu_backward(st, torch.from_numpy(np.concatenate(v_packed)).cuda())
    go = oracle.render_bwd(sc, [cams[c] for c in sel], vs, oracle.Opts(), pixels=pix_list)
    compare_grads({"pose": gg["pose"][sel]}, {"pose": go["pose"]}, keys=("pose",), name="pose batch")
    # poses with a zero cotangent get an exactly zero gradient
    others = [c for c in range(len(cams)) if c not in sel]
    assert np.all(gg["pose"][others] == 0)


def test_pose_batch_vs_twist_differences(pose_batch):
    """Directional central differences of L(xi) = 1/2 sum (I(Exp(xi) T) - I_true)^2
    with the GPU forward.  L jumps wherever a Gaussian crosses the 1/255 skip
    or the cutoff at some pixel, and the analytic gradient is the derivative
    of its smooth part; so the check is made on the pixels whose central
    differences at steps h and 2h agree (no jump within +-2h), with the
    gradient taken for the loss of those same pixels."""
    sc, true_cam, cams, tw, I_true, st = pose_batch
    imgs = unpack_np(st["cams"], st["image"])
    rng = np.random.default_rng(2)
    for c in (0, 7):
        d = rng.normal(size=6)
        d[:3] *= 1e-4 / np.linalg.norm(d[:3])
        d[3:] *= 2e-4 / np.linalg.norm(d[3:])

        def render(h):
            cam = S.perturb_camera(cams[c], h * d[:3], h * d[3:])
            s2 = gpu_forward(sc, [cam], tile=16)
            return unpack_np(s2["cams"], s2["image"])[0].astype(np.float64)

        I0 = imgs[c].astype(np.float64)
        D1 = (render(1.0) - render(-1.0)) / 2.0
        D2 = (render(2.0) - render(-2.0)) / 4.0
        smooth = (np.abs(D1 - D2) <= 0.05 * np.abs(D1) + 1e-6).all(0)
        assert smooth.mean() > 0.5, smooth.mean()
        r = I0 - I_true
        fd = float((r * D1)[:, smooth].sum())
        v = []
        for k, cam in enumerate(cams):
            vk = np.zeros((3, cam.height, cam.width), np.float32)
            if k == c:
                vk[:, smooth] = r[:, smooth]
            v.append(vk.ravel())
        gg = gpu_backward(st, torch.from_numpy(np.concatenate(v)).cuda())
        an = float(gg["pose"][c] @ d)
        assert abs(fd - an) <= 1e-2 * abs(an), (c, fd, an, smooth.mean())


def test_window_500k_sampled(oracle):
    sc, _ = S.config3()
    st = gpu_forward(sc, sc.cams, tile=16)
    imgs = unpack_np(st["cams"], st["image"])
    rng = np.random.default_rng(3)
    vparts, pix_l, vs = [], [], []
    for c, cam in enumerate(sc.cams):
        pix = _sample(cam, 48, rng)
        r = oracle.render(sc, cam, oracle.Opts(), pixels=pix)
        got = imgs[c][:, pix[:, 1], pix[:, 0]].T
        assert np.all(np.abs(got - r["rgb"]).max(1) <= pixel_tolerance(r["flags"]))
        nf = int(((r["flags"] & 1) != 0).sum())
        print(f"window 500k cam {c}: {nf} flag-1 pixels of {len(pix)}")
        assert nf <= 1, (c, nf)  # at most one excluded pixel per sampled keyframe
        pix = pix[(r["flags"] & 3) == 0]
        v = rng.normal(size=(len(pix), 3))
        vi = np.zeros((3, cam.height, cam.width), np.float32)
        vi[:, pix[:, 1], pix[:, 0]] = v.T
        vparts.append(vi.ravel())
        pix_l.append(pix)
        vs.append(v)
    gg = gpu_backward(st, torch.from_numpy(np.concatenate(vparts)).cuda())
    go = oracle.render_bwd(sc, sc.cams, vs, oracle.Opts(), pixels=pix_l)
    compare_grads(gg, go, keys=("mean", "scale", "quat", "opacity", "color", "pose"), name="window 500k")


@pytest.fixture(scope="module")
def uneven():
    sc, tgt = S.config5()
    return sc, tgt


def test_uneven_batch_sampled(oracle, uneven):
    sc, _ = uneven
    st = gpu_forward(sc, sc.cams, tile=8)
    imgs = unpack_np(st["cams"], st["image"])
    rng = np.random.default_rng(4)
    for c in (0, 5, 15):
        cam = sc.cams[c]
        pix = _sample(cam, 24, rng)
        r = oracle.render(sc, cam, oracle.Opts(), pixels=pix)
        got = imgs[c][:, pix[:, 1], pix[:, 0]].T
        assert np.all(np.abs(got - r["rgb"]).max(1) <= pixel_tolerance(r["flags"])), c
        nf = int(((r["flags"] & 1) != 0).sum())
        print(f"uneven batch cam {c}: {nf} flag-1 pixels of {len(pix)}")
        assert nf <= 1, (c, nf)


def test_uneven_batch_window_vs_per_camera(uneven):
    """One batched window step over 16 mixed-size cameras equals 16
    single-camera steps: images bit-identical, per-camera losses and pose
    gradients equal, Gaussian gradients equal to their sum."""
    O = ops()
    sc, tgt_sc = uneven
    ctx = context()
    cs = O.CameraSet(sc.cams)
    g = O.Gaussians.from_scene(sc)
    tgt = gpu_forward(tgt_sc, sc.cams, tile=16)["image"]
    w = O.Window(ctx, g, cs, O.opts(16), tgt, loss="l1", keep_image=True)
    w.step(use_graph=True)
    torch.cuda.synchronize()
    tot_mean = torch.zeros_like(w.grads.mean)
    loss = 0.0
    for c, cam in enumerate(sc.cams):
        c1 = O.CameraSet([cam])
        w1 = O.Window(ctx, g, c1, O.opts(16), cs.unpack(tgt)[c].reshape(-1).contiguous(), loss="l1",
                      keep_image=True)
        w1.step(use_graph=False)
        torch.cuda.synchronize()
        assert torch.equal(w1.image, cs.unpack(w.image)[c].reshape(-1))
        # the 2D gradients are summed with float atomics in a different order;
        # the pose is a sum over all Gaussians with cancellation
        scale = float(w.grads.pose[c].abs().max())
        torch.testing.assert_close(w1.grads.pose[0], w.grads.pose[c], rtol=1e-4, atol=1e-4 * scale)
        tot_mean += w1.grads.mean
        loss += float(w1.d_loss.item())
        del w1
    assert abs(loss - float(w.d_loss.item())) <= 1e-6 * abs(loss)
    torch.testing.assert_close(tot_mean, w.grads.mean, rtol=1e-4, atol=1e-5 * float(tot_mean.abs().max()))


def test_bench_window_step_is_the_separate_path():
    """The fused tile-32 window step (graph) at the benchmark size: the image
    it keeps equals gsl_render_fwd's bit for bit, and its L2-loss gradients
    are gsl_render_bwd's for the cotangent image - target.  Both add float32
    2D gradients with atomics in run-dependent order, up to thousands of adds
    per record at this size: 1e-4 of each tensor's largest entry (measured
    4e-5 on the scales), 1e-3 per large element."""
    O = ops()
    ctx = context()
    sc, tgt_sc = S.config3()
    cs = O.CameraSet(sc.cams)
    g = O.Gaussians.from_scene(sc)
    target = gpu_forward(tgt_sc, sc.cams, tile=32)["image"]
    w = O.Window(ctx, g, cs, O.opts(32), target, loss="l2", keep_image=True)
    for _ in range(2):
        w.step(use_graph=True)
    torch.cuda.synchronize()
    assert w.status() == 0
    st = gpu_forward(sc, sc.cams, tile=32)
    assert torch.equal(w.image, st["image"])
    gg = gpu_backward(st, (st["image"] - target).contiguous())
    got = {"mean": w.grads.mean.cpu().numpy().T, "scale": w.grads.scale.cpu().numpy().T,
           "quat": w.grads.quat.cpu().numpy().T, "opacity": w.grads.opacity.cpu().numpy(),
           "color": w.grads.color.cpu().numpy().T, "pose": w.grads.pose.cpu().numpy()}
    compare_grads(got, gg, rel=1e-4, keys=("mean", "scale", "quat", "opacity", "color", "pose"), elem_rel=1e-3,
                  name="bench window")


def test_bench_window_sh3_sampled(oracle):
    """The benchmark window with SH degree 3 colour at tile 32: sampled
    pixels of every keyframe against the oracle."""
    sc, _ = S.config3()
    sc = S.with_sh(sc, 3, 33)
    st = gpu_forward(sc, sc.cams, tile=32)
    imgs = unpack_np(st["cams"], st["image"])
    rng = np.random.default_rng(7)
    cm = max(float(np.abs(oracle.sh_colour(sc, c)).max()) for c in sc.cams)
    for c, cam in enumerate(sc.cams):
        pix = _sample(cam, 32, rng)
        r = oracle.render(sc, cam, oracle.Opts(), pixels=pix)
        got = imgs[c][:, pix[:, 1], pix[:, 0]].T
        assert np.all(np.abs(got - r["rgb"]).max(1) <= pixel_tolerance(r["flags"], cmax=cm)), c
        nf = int(((r["flags"] & 1) != 0).sum())
        print(f"SH3 window cam {c}: {nf} flag-1 pixels of {len(pix)}")
        assert nf <= 1, (c, nf)


def test_window_update_bench_size(oracle):
    """Two frames of the benchmark's window update (500k Gaussians x 42 rows,
    capacity 2^20, 100k points, 0.5 m voxels), bit for bit against the oracle."""
    O = ops()
    ctx = context()
    n, P, cap, vs, R = 500_000, 100_000, 1 << 20, 0.5, 42
    frames, means = S.lidar_stream(71, 3, P, n)
    k, ok = oracle.voxel_key(means, vs)
    win_keys = np.where(ok, k, np.uint64(0xFFFFFFFFFFFFFFFF))
    win_rows = np.random.default_rng(72).normal(size=(R, n)).astype(np.float32)
    sw = O.SlidingWindow(ctx, cap, vs)
    sw.keys[:n] = O.voxel_keys(ctx, torch.from_numpy(means).cuda(), vs)
    sw.block[:, :n] = torch.from_numpy(win_rows).cuda()
    sw.n = n
    for f in (1, 2):
        rng = np.random.default_rng(100 + f)
        made = {}

        def fetch(add_vox):
            made["vox"] = add_vox.numpy().view(np.uint64).copy()
            ak = np.repeat(made["vox"], 15)
            ar = rng.normal(size=(R, len(ak))).astype(np.float32)
            made["k"], made["r"] = ak, ar
            return torch.from_numpy(ak.view(np.int64).copy()), torch.from_numpy(ar)

        ek, er = sw.update(torch.from_numpy(frames[f]).cuda(), fetch)
        torch.cuda.synchronize()
        # the oracle's own classification decides its side; the GPU's ADD list must equal it
        pk, pok = oracle.voxel_key(frames[f], vs)
        _, add_o = oracle.window_classify(win_keys, pk, pok)
        assert np.array_equal(made["vox"], add_o)
        win_keys, win_rows, ek_w, er_w = oracle.window_maintain(win_keys, win_rows, pk[pok], np.repeat(add_o, 15),
                                                                made["r"])
        assert sw.n == len(win_keys)
        assert np.array_equal(sw.keys[:sw.n].cpu().numpy().view(np.uint64), win_keys)
        assert np.array_equal(sw.block[:, :sw.n].cpu().numpy().view(np.uint32), win_rows.view(np.uint32))
        assert np.array_equal(ek.cpu().numpy().view(np.uint64), ek_w)
        assert np.array_equal(er.cpu().numpy().view(np.uint32), er_w.view(np.uint32))
