"""Pose Jacobians of the IESKF visual update on the GPU (gsl_pose_jacobian)
against the FP64 oracle: per-pixel dI/dxi, the rendered colour, the per-camera
normal equations, the adjoint identity with the reverse-mode pose gradient,
and one Gauss-Newton/IESKF step that moves a perturbed camera towards the
true pose."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import scenegen as S
from scenegen import Camera

from gpuutil import gpu_backward, gpu_forward, ops, unpack_np

pytestmark = pytest.mark.gpu


def _cams(seed):
    rng = np.random.default_rng(seed)
    out = []
    for (W, H, f) in ((96, 80, 90.0), (130, 70, 110.0)):
        R = Rotation.from_rotvec(rng.normal(0, 0.15, 3)).as_matrix()
        out.append(Camera(f, f * 1.02, W / 2 + 1.7, H / 2 - 0.9, W, H, R, rng.normal(0, 0.2, 3)))
    return out


def _scene(seed, n=3000):
    cams = _cams(seed)
    sc = S.random_scene(n, cams[0], seed, zmin=1.0, zmax=4.0, smin=0.02, smax=0.15, unnormalised_quats=True)
    sc.cams = cams
    return sc


def _run(sc, tile, target=None, weight=None, bg=(0.0, 0.0, 0.0)):
    O = ops()
    st = gpu_forward(sc, sc.cams, tile=tile, bg=bg)
    tgt = None if target is None else torch.from_numpy(target.astype(np.float32)).cuda()
    wgt = None if weight is None else torch.from_numpy(weight.astype(np.float32)).cuda()
    pj = O.pose_jacobian(st["ctx"], st["g"], st["cams"], st["opts"], st["proj"], st["bins"], target=tgt,
                         weight=wgt, want_image=True, want_jac=True)
    torch.cuda.synchronize()
    return st, pj


def _jac_per_camera(st, pj):
    cs = st["cams"]
    out = []
    for c, (h, w) in enumerate(cs.sizes):
        o = int(cs.pix_offsets[c])
        J = pj.jac[:, o:o + h * w].cpu().numpy().astype(np.float64)  # (18, P)
        out.append(J.reshape(3, 6, h * w).transpose(2, 0, 1))       # (P, 3, 6)
    return out


@pytest.mark.parametrize("tile,degree", [(8, 0), (16, 0), (32, 0), (16, 3), (32, 2)])
def test_pose_jacobian_matches_oracle(oracle, tile, degree):
    """Per pixel, per twist direction: |GPU - oracle| <= 1e-3 max |oracle| on
    the pixels the oracle does not flag; the colour equals gsl_render_fwd's
    bit for bit (same walk, same decisions).  With SH colour the colours'
    dependence on the camera centre is part of the Jacobian."""
    sc = S.with_sh(_scene(3), degree, 33, sigma=0.2)
    bg = (0.1, 0.2, 0.3)
    st, pj = _run(sc, tile, bg=bg)
    img_fwd = st["image"].cpu().numpy()
    assert np.array_equal(pj.image.cpu().numpy(), img_fwd)
    jg = _jac_per_camera(st, pj)
    o = oracle.Opts(bg=bg)
    nflag = 0
    for c, cam in enumerate(sc.cams):
        r = oracle.render_jvp(sc, cam, o)
        fl = oracle.render(sc, cam, o)["flags"]
        ok = fl == 0
        nflag += int((~ok).sum())
        for j in range(6):
            ref = r["jac"][:, :, j]
            m = np.abs(ref[ok]).max()
            d = np.abs(jg[c][:, :, j] - ref)[ok].max()
            assert d <= 1e-3 * m, (c, j, d, m)
    assert nflag <= 0.02 * sum(c.width * c.height for c in sc.cams)


@pytest.mark.parametrize("weighted", [False, True])
def test_pose_normal_equations_match_oracle(oracle, weighted):
    """Per camera H^T R^-1 H, H^T R^-1 z and z^T R^-1 z (z = I - target) from
    the device reduction against the oracle's sums over all pixels of its own
    Jacobians and colours: entrywise within 1e-3 of the largest entry."""
    sc = _scene(5)
    rng = np.random.default_rng(2)
    tgt_sc = S.jitter_means(sc, 0.01, 9)
    tgt_sc.cams = sc.cams
    targets = [oracle.render_image(tgt_sc, cam)["image"] for cam in sc.cams]
    target = np.concatenate([t.reshape(-1) for t in targets])
    P_total = sum(c.width * c.height for c in sc.cams)
    weight = rng.uniform(0.2, 2.0, P_total) if weighted else None
    st, pj = _run(sc, 16, target=target, weight=weight)
    off = 0
    for c, cam in enumerate(sc.cams):
        r = oracle.render_jvp(sc, cam)
        n = cam.width * cam.height
        res = r["rgb"] - targets[c].reshape(3, -1).T
        w = None if weight is None else weight[off:off + n]
        HtH, Htz, zz = oracle.normal_equations(r["jac"], res, w)
        off += n
        np.testing.assert_allclose(pj.HtH[c].cpu().numpy(), HtH, rtol=0, atol=1e-3 * np.abs(HtH).max())
        np.testing.assert_allclose(pj.Htz[c].cpu().numpy(), Htz, rtol=0, atol=1e-3 * np.abs(Htz).max())
        assert abs(float(pj.zz[c]) - zz) <= 1e-3 * zz
        g = pj.HtH[c].cpu().numpy()
        assert np.array_equal(g, g.T)


@pytest.mark.parametrize("degree", [0, 3])
def test_pose_jacobian_adjoint_identity_on_gpu(degree):
    """GPU forward mode against GPU reverse mode: sum_p <v_p, dI_p/dxi> equals
    gsl_render_bwd's pose gradient for the same cotangent v (with SH colour
    both include the colours' dependence on the camera centre)."""
    sc = S.with_sh(_scene(8), degree, 18, sigma=0.2)
    st, pj = _run(sc, 16)
    rng = np.random.default_rng(4)
    v = rng.normal(size=3 * st["cams"].P_total).astype(np.float32)
    g = gpu_backward(st, torch.from_numpy(v).cuda())
    jg = _jac_per_camera(st, pj)
    vs = unpack_np(st["cams"], torch.from_numpy(v))
    for c in range(len(sc.cams)):
        vp = vs[c].reshape(3, -1).T.astype(np.float64)
        lhs = np.einsum("pc,pcj->j", vp, jg[c])
        np.testing.assert_allclose(lhs, g["pose"][c], rtol=0, atol=2e-3 * np.abs(g["pose"][c]).max())


def test_ieskf_step_moves_camera_towards_truth(oracle):
    """A camera perturbed by a small left twist from the pose that rendered
    the target: one update from the GPU normal equations (flat prior) cuts
    the pose error by more than half, and agrees with the oracle's update
    from its own normal equations at the same estimate."""
    O = ops()
    sc, cam_true, _, _ = S.config4(n_planes=6, per_plane=3000, n_poses=1, width=160, height=128, f=125.0)
    target = oracle.render_image(sc, cam_true)["image"]
    xi_err = np.array([0.004, -0.003, 0.002, 0.01, -0.008, 0.006])
    cam_hat = S.perturb_camera(cam_true, xi_err[:3], xi_err[3:])
    sc.cams = [cam_hat]
    st, pj = _run(sc, 16, target=target.reshape(-1))
    P = np.eye(6) * 1e6
    delta, _ = O.ieskf_pose_update(pj.HtH[0].cpu().numpy(), pj.Htz[0].cpu().numpy(), P)
    # the update is a left twist of T_CW; the remaining error is that of T_true T_new^-1
    R_hat, t_hat = cam_hat.R_cw.astype(np.float64), cam_hat.t_cw.astype(np.float64)
    E2 = Rotation.from_rotvec(delta[:3]).as_matrix()
    R_new, t_new = E2 @ R_hat, E2 @ t_hat + delta[3:]
    Rt, tt = cam_true.R_cw.astype(np.float64), cam_true.t_cw.astype(np.float64)
    dR = Rotation.from_matrix(Rt @ R_new.T).as_rotvec()
    dt = tt - (Rt @ R_new.T) @ t_new
    before, after = np.linalg.norm(xi_err), np.linalg.norm(np.concatenate([dR, dt]))
    assert after < 0.5 * before, (before, after, delta)
    r = oracle.render_jvp(sc, cam_hat)
    HtH, Htz, _ = oracle.normal_equations(r["jac"], r["rgb"] - target.reshape(3, -1).T)
    d_orc, _ = oracle.ieskf_pose_update(HtH, Htz, P)
    np.testing.assert_allclose(delta, d_orc, rtol=0, atol=2e-2 * np.abs(d_orc).max())
