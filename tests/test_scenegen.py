"""The seeded input generators: deterministic, and shaped as stated (frustum
depth range, surfel geometry, keyframe spacing, perturbation sizes)."""
import numpy as np

import scenegen as S


def test_seeded_and_float32():
    a, b = S.config1(), S.config1()
    assert a.digest() == b.digest()
    assert S.config1(seed=2).digest() != a.digest()
    for arr in (a.mean, a.scale, a.quat, a.opacity, a.color):
        assert arr.dtype == np.float32


def test_config1_distributions():
    sc = S.config1()
    cam = sc.cams[0]
    z = sc.mean[:, 2].astype(np.float64)
    assert z.min() >= 1.0 - 1e-6 and z.max() <= 5.0 + 1e-6
    u = cam.fx * sc.mean[:, 0] / z + cam.cx
    v = cam.fy * sc.mean[:, 1] / z + cam.cy
    assert np.all((u > -1e-3) & (u < cam.width + 1e-3) & (v > -1e-3) & (v < cam.height + 1e-3))
    assert sc.scale.min() >= 0.01 - 1e-7 and sc.scale.max() <= 0.1 + 1e-7
    np.testing.assert_allclose(np.linalg.norm(sc.quat, axis=1), 1, atol=1e-6)
    assert 0 < sc.opacity.min() and sc.opacity.max() < 1


def test_surfels_are_flat_along_the_normal():
    cam = S.Camera(500, 500, 320, 256, 640, 512, np.eye(3), np.zeros(3))
    rng = np.random.default_rng(0)
    sc = S.surface_scene(3, 200, 7, S.scenes.frustum_points(rng, cam, 3, 2, 4))
    assert np.all(sc.scale[:, 2] == np.float32(1e-3))
    # the third rotation axis is the patch normal: all surfels of a patch share it (up to sign)
    from scipy.spatial.transform import Rotation
    q = sc.quat.astype(np.float64)
    R = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1)).as_matrix()
    n = R[:, :, 2]
    for p in range(3):
        blk = n[p * 200:(p + 1) * 200]
        assert np.all(np.abs(blk @ blk[0]) > 1 - 1e-5)


def test_trajectory_spacing():
    cams = S.trajectory_cameras(8, 1280, 1024, 1000.0, seed=3)
    centres = [-c.R_cw.astype(np.float64).T @ c.t_cw.astype(np.float64) for c in cams]
    for a, b, ca, cb in zip(centres, centres[1:], cams, cams[1:]):
        np.testing.assert_allclose(np.linalg.norm(b - a), 0.3, rtol=1e-5)
        Rrel = ca.R_cw.astype(np.float64) @ cb.R_cw.astype(np.float64).T
        ang = np.degrees(np.arccos(np.clip((np.trace(Rrel) - 1) / 2, -1, 1)))
        np.testing.assert_allclose(ang, 5.0, rtol=1e-3)


def test_config4_perturbations():
    sc, true_cam, cams, tw = S.config4(n_planes=2, per_plane=100)
    assert len(cams) == 32 and tw.shape == (32, 6)
    assert np.abs(tw[:, 3:]).max() < 0.05 * 5 and np.abs(np.degrees(tw[:, :3])).max() < 5
