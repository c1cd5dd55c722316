"""Pins for the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (single Gaussian on the optical axis, two Gaussians), library routines
for special cases (scipy rotations), invariants (rigid motion, permutation,
partition of unity, monotone transmittance), brute-force evaluation of the
compositing sum as an explicit product, and central finite differences of the
forward for every gradient, including the camera twist.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen as S
from dataclasses import replace

from scenegen import Camera, Scene

pytestmark = pytest.mark.filterwarnings("ignore")


def _cam(W=32, H=24, f=30.0, R=np.eye(3), t=np.zeros(3), cx=None, cy=None):
    return Camera(f, f * 1.1, W / 2 if cx is None else cx, H / 2 if cy is None else cy, W, H, R, t)


def _scene(mean, scale, quat, opac, color, cams):
    return Scene(np.array(mean), np.array(scale), np.array(quat), np.array(opac), np.array(color), cams)


def _wxyz_to_scipy(q):
    q = np.asarray(q, np.float64)
    return Rotation.from_quat(np.concatenate([q[..., 1:], q[..., :1]], -1))


# ---------------------------------------------------------------- projection

def test_projection_on_axis_closed_form(oracle):
    """Gaussian at (0, 0, z) under an identity camera: mean2d = (cx, cy) and
    Sigma2D = (f/z)^2 (R S^2 R^T)[:2, :2] + eps I, with R from scipy."""
    cam = _cam(W=64, H=48, f=80.0)
    rng = np.random.default_rng(0)
    n = 20
    z = rng.uniform(1, 4, n)
    mean = np.stack([np.zeros(n), np.zeros(n), z], 1)
    scale = rng.uniform(0.01, 0.2, (n, 3))
    quat = rng.normal(size=(n, 4))
    sc = _scene(mean, scale, quat, np.full(n, 0.5), np.ones((n, 3)), [cam])
    o = oracle.Opts(eps2d=0.3)
    p = oracle.project(sc, cam, o)
    assert np.all(p["status"] & 1)
    np.testing.assert_allclose(p["mean2d"], np.tile([cam.cx, cam.cy], (n, 1)), rtol=0, atol=1e-12)
    m, s = sc.mean.astype(np.float64), sc.scale.astype(np.float64)
    R = _wxyz_to_scipy(sc.quat.astype(np.float64)).as_matrix()
    for i in range(n):
        Sig = R[i] @ np.diag(s[i] ** 2) @ R[i].T
        J = np.diag([cam.fx / m[i, 2], cam.fy / m[i, 2]])
        S2 = J @ Sig[:2, :2] @ J + 0.3 * np.eye(2)
        np.testing.assert_allclose(p["cov2d"][i], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-12)
        Q = np.linalg.inv(S2)
        np.testing.assert_allclose(p["conic"][i], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-10)


def test_projection_roll_swaps_axes(oracle):
    """A 90 degree rotation of the Gaussian about the optical axis swaps the
    2D covariance axes (square pixels)."""
    cam = Camera(50.0, 50.0, 16, 12, 32, 24, np.eye(3), np.zeros(3))
    q0 = [1, 0, 0, 0]
    q90 = [np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)]
    sc = _scene([[0, 0, 2.0], [0, 0, 2.0]], [[0.1, 0.03, 0.05]] * 2, [q0, q90], [0.5, 0.5], np.ones((2, 3)),
                [cam])
    p = oracle.project(sc, cam, oracle.Opts(eps2d=0.0))
    a, b = p["cov2d"]
    np.testing.assert_allclose([a[0], a[2]], [b[2], b[0]], rtol=1e-6)
    np.testing.assert_allclose(a[0], (50 * float(np.float32(0.1)) / 2) ** 2, rtol=1e-6)


def test_projection_matches_linearised_pinhole(oracle):
    """Off-axis Gaussians under a rotated camera: mean2d is the pinhole image
    of R_cw p + t computed with scipy, and Sigma2D - eps I equals J Sigma_C J^T
    where J is a central-difference Jacobian of the pinhole map."""
    rng = np.random.default_rng(1)
    Rc = Rotation.from_rotvec(rng.normal(0, 0.3, 3)).as_matrix()
    cam = Camera(70.0, 65.0, 33.0, 21.0, 64, 48, Rc, rng.normal(0, 0.5, 3))
    sc = S.random_scene(30, cam, seed=7, zmin=1.5, zmax=4)
    p = oracle.project(sc, cam, oracle.Opts(eps2d=0.3))
    Rcw, t = cam.R_cw.astype(np.float64), cam.t_cw.astype(np.float64)

    def pinhole(pc):
        return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])

    R = _wxyz_to_scipy(sc.quat.astype(np.float64)).as_matrix()
    for i in range(sc.n):
        pc = Rcw @ sc.mean[i].astype(np.float64) + t
        np.testing.assert_allclose(p["p_cam"][i], pc, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(p["mean2d"][i], pinhole(pc), rtol=1e-12)
        h = 1e-6
        Jn = np.stack([(pinhole(pc + h * e) - pinhole(pc - h * e)) / (2 * h) for e in np.eye(3)], 1)
        s = sc.scale[i].astype(np.float64)
        SigC = Rcw @ R[i] @ np.diag(s ** 2) @ R[i].T @ Rcw.T
        S2 = Jn @ SigC @ Jn.T
        np.testing.assert_allclose(p["cov2d"][i], [S2[0, 0] + 0.3, S2[0, 1], S2[1, 1] + 0.3], rtol=1e-6)


def test_projection_culls_near_and_guard(oracle):
    cam = _cam(W=40, H=30, f=40.0)
    mean = [[0, 0, 0.1], [0, 0, 0.25], [100.0, 0, 1.0], [0.5, 0, 1.0]]
    sc = _scene(mean, [[0.05] * 3] * 4, [[1, 0, 0, 0]] * 4, [0.5] * 4, np.ones((4, 3)), [cam])
    st = oracle.project(sc, cam, oracle.Opts())["status"]
    assert list(st & 1) == [0, 1, 0, 1]


def test_rigid_motion_invariance(oracle):
    """Moving the scene and the camera by the same rigid motion leaves the
    projection and the image unchanged."""
    cam = _cam(W=40, H=30, f=35.0)
    sc = S.random_scene(40, cam, seed=3, zmin=1.5, zmax=4.0)
    r0 = Rotation.from_rotvec([0.3, -0.5, 0.9])
    t0 = np.array([1.0, -2.0, 0.5])
    m2 = r0.apply(sc.mean.astype(np.float64)) + t0
    q2 = (r0 * _wxyz_to_scipy(sc.quat)).as_quat()  # scipy (x, y, z, w)
    q2 = np.concatenate([q2[:, 3:], q2[:, :3]], 1) * np.linalg.norm(sc.quat.astype(np.float64), axis=1,
                                                                    keepdims=True)
    R2 = cam.R_cw.astype(np.float64) @ r0.as_matrix().T
    t2 = cam.t_cw.astype(np.float64) - R2 @ t0
    # keep everything exactly representable: compare against the float32-rounded moved scene
    sc2 = _scene(m2, sc.scale, q2, sc.opacity, sc.color, [])
    cam2 = Camera(cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, R2, t2)
    a = oracle.render_image(sc, cam, oracle.Opts())
    b = oracle.render_image(sc2, cam2, oracle.Opts())
    # float32 rounding of the moved inputs perturbs values at the 1e-6 level
    ok = (a["flags"] == 0) & (b["flags"] == 0)
    assert ok.mean() > 0.95
    np.testing.assert_allclose(a["image"][:, ok], b["image"][:, ok], atol=2e-5)


# ---------------------------------------------------------------- compositing

def test_single_gaussian_closed_form(oracle):
    """One Gaussian on the axis: I(x) = c min(0.99, sigma G(x)) + (1 - a) bg
    where a >= 1/255, else bg, with G the axis-aligned 2D Gaussian."""
    cam = _cam(W=48, H=40, f=60.0)
    sc = _scene([[0, 0, 2.0]], [[0.08, 0.05, 0.1]], [[1, 0, 0, 0]], [0.9], [[0.3, 0.6, 0.9]], [cam])
    bg = (0.1, 0.2, 0.05)
    o = oracle.Opts(bg=bg, eps2d=0.3)
    r = oracle.render_image(sc, cam, o)
    s = sc.scale[0].astype(np.float64)
    sxx = (cam.fx * s[0] / 2.0) ** 2 + 0.3
    syy = (cam.fy * s[1] / 2.0) ** 2 + 0.3
    v, u = np.mgrid[0:cam.height, 0:cam.width]
    dx, dy = u + 0.5 - cam.cx, v + 0.5 - cam.cy
    G = np.exp(-0.5 * (dx ** 2 / sxx + dy ** 2 / syy))
    a = np.minimum(0.99, float(np.float32(0.9)) * G)
    a = np.where(a >= 1 / 255, a, 0.0)
    for ch in range(3):
        want = float(sc.color[0, ch]) * a + (1 - a) * bg[ch]
        np.testing.assert_allclose(r["image"][ch], want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["T"], 1 - a, atol=1e-12)
    assert np.all(r["n"] == (a > 0))


def test_two_gaussian_closed_form(oracle):
    """Front and back Gaussian: I = c_f a_f + c_b a_b (1 - a_f), the front one
    chosen by depth whatever the index order."""
    cam = _cam(W=24, H=20, f=40.0)
    sc = _scene([[0.02, 0, 3.0], [0, 0.01, 1.5]], [[0.1, 0.1, 0.1], [0.05, 0.07, 0.05]],
                [[1, 0, 0, 0], [1, 0, 0, 0]], [0.7, 0.6], [[1, 0, 0], [0, 1, 0]], [cam])
    o = oracle.Opts(eps2d=0.3)
    r = oracle.render_image(sc, cam, o)
    p = oracle.project(sc, cam, o)
    v, u = np.mgrid[0:cam.height, 0:cam.width]
    al = []
    for i in range(2):
        dx, dy = u + 0.5 - p["mean2d"][i, 0], v + 0.5 - p["mean2d"][i, 1]
        A, B, Cc = p["conic"][i]
        a = np.minimum(0.99, float(sc.opacity[i]) * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + Cc * dy * dy)))
        al.append(np.where(a >= 1 / 255, a, 0.0))
    front, back = al[1], al[0]  # index 1 is nearer
    want = np.stack([back * (1 - front), front, np.zeros_like(front)])
    np.testing.assert_allclose(r["image"], want, atol=1e-12)


def test_partition_of_unity(oracle):
    """All colours 1 and background 0: every channel equals 1 - T_final."""
    cam = _cam(W=40, H=32, f=30.0)
    sc = S.random_scene(200, cam, seed=11, zmin=1, zmax=3, smin=0.05, smax=0.3)
    sc.color[:] = 1.0
    r = oracle.render_image(sc, cam, oracle.Opts())
    for ch in range(3):
        np.testing.assert_allclose(r["image"][ch], 1 - r["T"], atol=1e-12)
    assert r["T"].min() >= 1e-4  # the walk stops before crossing the cutoff
    assert r["T"].max() <= 1.0


def test_transmittance_monotone_and_explicit_product(oracle):
    """Brute force on a tiny scene: the contributor set is exactly the
    Gaussians in (float depth, index) order whose alpha reaches 1/255, cut
    before the transmittance would drop below 1e-4; the image equals the
    explicit sum of c_i a_i prod_{j<i}(1 - a_j) over that set."""
    cam = _cam(W=16, H=12, f=14.0)
    sc = S.random_scene(16, cam, seed=5, zmin=1, zmax=2, smin=0.05, smax=0.3)
    o = oracle.Opts()
    p = oracle.project(sc, cam, o)
    r = oracle.render_image(sc, cam, o)
    z32 = p["p_cam"][:, 2].astype(np.float32)
    order = sorted([i for i in range(sc.n) if p["status"][i] & 1], key=lambda i: (z32[i], i))
    for vv in range(cam.height):
        for uu in range(cam.width):
            ids, al, Ts = oracle.pixel_trace(sc, cam, uu, vv, o)
            assert np.all(np.diff(Ts) <= 0) and np.all(Ts <= 1)
            # brute-force contributor set
            T = 1.0
            want_ids, want_al = [], []
            for i in order:
                dx, dy = uu + 0.5 - p["mean2d"][i, 0], vv + 0.5 - p["mean2d"][i, 1]
                A, B, Cc = p["conic"][i]
                a = min(0.99, float(sc.opacity[i]) * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + Cc * dy * dy)))
                if a < 1 / 255:
                    continue
                if T * (1 - a) < 1e-4:
                    break
                want_ids.append(i)
                want_al.append(a)
                T *= 1 - a
            assert list(ids) == want_ids
            np.testing.assert_allclose(al, want_al, rtol=1e-13)
            # explicit product form of the compositing sum
            c = sc.color.astype(np.float64)
            val = sum(c[i] * a * np.prod([1 - b for b in want_al[:k]]) for k, (i, a) in
                      enumerate(zip(want_ids, want_al)))
            np.testing.assert_allclose(r["image"][:, vv, uu], val if len(want_ids) else np.zeros(3),
                                       atol=1e-12)


def test_permutation_invariance(oracle):
    cam = _cam(W=40, H=30, f=35.0)
    sc = S.random_scene(300, cam, seed=21, smin=0.03, smax=0.2)
    perm = np.random.default_rng(0).permutation(sc.n)
    a = oracle.render_image(sc, cam, oracle.Opts())
    b = oracle.render_image(sc.permuted(perm), cam, oracle.Opts())
    np.testing.assert_array_equal(a["image"], b["image"])
    np.testing.assert_array_equal(a["T"], b["T"])


# ---------------------------------------------------------------- gradients

def _loss(oracle, sc, cams, Ws, o):
    tot = 0.0
    for cam, W in zip(cams, Ws):
        tot += float(np.sum(oracle.render_image(sc, cam, o)["image"] * W))
    return tot


def _flags(oracle, sc, cams, o):
    return [oracle.render_image(sc, c, o)["flags"] for c in cams]


def _fd_scene(seed, n=6, W=20, H=16, clamp=False):
    cam = _cam(W=W, H=H, f=18.0)
    sc = S.random_scene(n, cam, seed=seed, zmin=1.0, zmax=2.0, smin=0.08, smax=0.3, unnormalised_quats=True)
    if clamp:  # opacities near 1: the alpha clamp is active around the centres
        sc.opacity[:] = np.float32(0.995)
    else:  # opacities away from the clamp so that no alpha sits on it
        sc.opacity[:] = np.float32(0.3) + np.float32(0.5) * sc.opacity
    return sc, cam


@pytest.mark.parametrize("seed,clamp", [(1, False), (2, False), (3, True)])
def test_gradients_match_central_differences(oracle, seed, clamp):
    """Analytic gradients for L = <W, I> against FP64 central differences of
    the forward, for every parameter of every Gaussian (with and without
    pixels where the alpha clamp holds)."""
    sc, cam = _fd_scene(seed, clamp=clamp)
    o = oracle.Opts(bg=(0.2, 0.1, 0.3))
    rng = np.random.default_rng(seed)
    Wimg = rng.normal(size=(3, cam.height, cam.width))
    fl = _flags(oracle, sc, [cam], o)[0]
    Wimg[:, fl != 0] = 0.0
    g = oracle.render_bwd(sc, [cam], [Wimg], o)
    base = {k: getattr(sc, k).astype(np.float64).copy() for k in ("mean", "scale", "quat", "opacity", "color")}

    def L_with(name, val):
        params = {k: v.copy() for k, v in base.items()}
        params[name] = val
        s2 = Scene(params["mean"], params["scale"], params["quat"], params["opacity"], params["color"], [cam])
        # bypass float32 rounding: the oracle works on float64 copies
        for k in params:
            setattr(s2, k, params[k])
        return _loss(oracle, s2, [cam], [Wimg], o)

    for name in ("mean", "scale", "quat", "opacity", "color"):
        a = base[name]
        fd = np.zeros_like(a)
        for idx in np.ndindex(a.shape):
            h = 1e-6 * max(1.0, abs(a[idx]))
            ap, am = a.copy(), a.copy()
            ap[idx] += h
            am[idx] -= h
            fd[idx] = (L_with(name, ap) - L_with(name, am)) / (2 * h)
        an = g[name]
        scale = np.abs(fd).max()
        np.testing.assert_allclose(an, fd, atol=2e-6 * scale + 1e-9, rtol=2e-5, err_msg=name)


def _rodrigues(w):
    return Rotation.from_rotvec(w).as_matrix()


class Cam64:
    """A camera holding float64 pose values (exactly orthonormal rotations)."""

    def __init__(self, like, R, t):
        self.fx, self.fy, self.cx, self.cy = like.fx, like.fy, like.cx, like.cy
        self.width, self.height = like.width, like.height
        self.R_cw = np.asarray(R, np.float64)
        self.t_cw = np.asarray(t, np.float64)


def test_pose_gradient_matches_twist_differences(oracle):
    """dL/d(dphi, dt) for T_CW <- Exp(dphi, dt) T_CW against central
    differences, with the exponential taken from scipy."""
    rng = np.random.default_rng(4)
    Rc = Rotation.from_rotvec([0.1, -0.2, 0.05]).as_matrix()
    cam0 = Camera(18.0, 19.0, 10.0, 8.0, 20, 16, Rc, [0.1, -0.05, 0.2])
    sc = S.random_scene(8, cam0, seed=9, zmin=1.0, zmax=2.0, smin=0.08, smax=0.3)
    sc.opacity[:] = np.float32(0.3) + np.float32(0.5) * sc.opacity
    o = oracle.Opts()
    Wimg = rng.normal(size=(3, cam0.height, cam0.width))
    Wimg[:, oracle.render_image(sc, cam0, o)["flags"] != 0] = 0

    def cam_at(xi):
        E = _rodrigues(xi[:3])
        return Cam64(cam0, E @ cam0.R_cw.astype(np.float64), E @ cam0.t_cw.astype(np.float64) + xi[3:])

    g = oracle.render_bwd(sc, [cam0], [Wimg], o)["pose"][0]
    fd = np.zeros(6)
    for k in range(6):
        h = 1e-6
        e = np.zeros(6)
        e[k] = h
        fd[k] = (_loss(oracle, sc, [cam_at(e)], [Wimg], o) - _loss(oracle, sc, [cam_at(-e)], [Wimg], o)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=2e-5, atol=1e-6 * np.abs(fd).max())


def test_pose_gradient_rigid_identities(oracle):
    """Exact identities: translating the camera by dt moves every camera-frame
    mean by dt, so dL/ddt = R_cw sum_i dL/dp_W,i; rotating it by dphi rotates
    every camera-frame mean and orientation, so dL/ddphi is the matching sum of
    mean and quaternion gradients."""
    rng = np.random.default_rng(8)
    Rc = Rotation.from_rotvec([0.2, 0.1, -0.3]).as_matrix()
    cam32 = Camera(40.0, 42.0, 20.0, 16.0, 40, 32, Rc, [0.3, 0.1, -0.2])
    sc = S.random_scene(60, cam32, seed=13, zmin=1.0, zmax=3.0, smin=0.03, smax=0.2, unnormalised_quats=True)
    cam = Cam64(cam32, Rc, [0.3, 0.1, -0.2])
    o = oracle.Opts()
    Wimg = rng.normal(size=(3, cam.height, cam.width))
    g = oracle.render_bwd(sc, [cam], [Wimg], o)
    W = cam.R_cw.astype(np.float64)
    np.testing.assert_allclose(g["pose"][0, 3:], W @ g["mean"].sum(0), rtol=1e-10,
                               atol=1e-12 * np.abs(g["mean"]).max())
    pC = sc.mean.astype(np.float64) @ W.T + cam.t_cw.astype(np.float64)
    q = sc.quat.astype(np.float64)
    want = np.zeros(3)
    for k in range(3):
        phi = np.zeros(3)
        phi[k] = 1.0
        # camera-frame means move by phi x p_C; in world coordinates W^T (phi x p_C)
        dm = np.cross(phi, pC) @ W
        # orientations turn by the world-frame vector W^T phi: dq = 1/2 (0, w) (x) q
        w = W.T @ phi
        dq = 0.5 * np.stack([-(w[0] * q[:, 1] + w[1] * q[:, 2] + w[2] * q[:, 3]),
                             w[0] * q[:, 0] + w[1] * q[:, 3] - w[2] * q[:, 2],
                             w[1] * q[:, 0] + w[2] * q[:, 1] - w[0] * q[:, 3],
                             w[2] * q[:, 0] + w[0] * q[:, 2] - w[1] * q[:, 1]], 1)
        want[k] = np.sum(g["mean"] * dm) + np.sum(g["quat"] * dq)
    np.testing.assert_allclose(g["pose"][0, :3], want, rtol=1e-9, atol=1e-12 * np.abs(want).max())


def test_single_gaussian_gradient_closed_forms(oracle):
    """One unclamped Gaussian, background 0: dI_ch/dc_ch = a and
    dI/dsigma = c G at every pixel."""
    cam = _cam(W=24, H=20, f=30.0)
    sc = _scene([[0, 0, 2.0]], [[0.08, 0.05, 0.1]], [[1, 0, 0, 0]], [0.6], [[0.3, 0.6, 0.9]], [cam])
    o = oracle.Opts()
    p = oracle.project(sc, cam, o)
    v, u = np.mgrid[0:cam.height, 0:cam.width]
    dx, dy = u + 0.5 - p["mean2d"][0, 0], v + 0.5 - p["mean2d"][0, 1]
    A, B, Cc = p["conic"][0]
    G = np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + Cc * dy * dy))
    a = float(sc.opacity[0]) * G
    on = a >= 1 / 255
    for ch in range(3):
        Wimg = np.zeros((3, cam.height, cam.width))
        Wimg[ch] = 1.0
        g = oracle.render_bwd(sc, [cam], [Wimg], o)
        np.testing.assert_allclose(g["color"][0, ch], a[on].sum(), rtol=1e-12)
        np.testing.assert_allclose(g["opacity"][0], float(sc.color[0, ch]) * G[on].sum(), rtol=1e-12)


def test_alpha_threshold_flip_bound(oracle):
    """A Gaussian whose alpha sits on the 1/255 skip threshold, once with
    nothing in front of it and once behind two occluders (T = 0.01 * 0.5).
    Taking the decision either way moves the pixel by alpha T |c - bg| at
    most, well inside 2 alpha T (max c + bg): the oracle flags the pixel when
    that bound exceeds the 5e-5 budget (open view) and leaves it unflagged
    when it does not (occluded), in which case the two sides of the threshold
    agree to the budget."""
    cam = _cam(W=9, H=9, f=20.0, cx=4.5, cy=4.5)
    probe = dict(mean=[0, 0, 3.0], scale=[0.3, 0.3, 0.3], color=[1.0, 0.0, 0.5])
    occ_mean, occ_scale = [[0, 0, 1.0], [0, 0, 1.5]], [[1.0, 1.0, 1.0], [1.0, 1.0, 1.0]]
    pix = np.array([[4, 4]], np.int32)
    o = oracle.Opts()
    for occluded in (False, True):
        res = []
        for side in (-1, 1):
            mean = ([probe["mean"]] + (occ_mean if occluded else []))
            scale = ([probe["scale"]] + (occ_scale if occluded else []))
            n = len(mean)
            sc = _scene(mean, scale, [[1, 0, 0, 0]] * n, [1.0] + [0.99, 0.5][: n - 1],
                        [probe["color"]] + [[0.2, 0.2, 0.2]] * (n - 1), [cam])
            p = oracle.project(sc, cam, o)
            A, B, Cc = p["conic"][0]
            d = 4.5 - p["mean2d"][0]
            G = np.exp(-0.5 * (A * d[0] ** 2 + 2 * B * d[0] * d[1] + Cc * d[1] ** 2))
            sc.opacity[0] = np.float32((1 / 255) / G * (1 + side * 1e-6))
            res.append(oracle.render(sc, cam, o, pixels=pix))
        lo, hi = res
        assert hi["n"][0] == lo["n"][0] + 1  # the probe is skipped on one side only
        dev = float(np.abs(hi["rgb"] - lo["rgb"]).max())
        T = 1.0 if not occluded else (1 - 0.99) * (1 - 0.5)
        assert dev <= (1 / 255) * T * 1.0 * (1 + 1e-5)
        if occluded:
            assert (lo["flags"][0] & 1) == 0 and (hi["flags"][0] & 1) == 0  # (2: the occluder sits on the clamp)
            assert dev <= o.amb_ignore
            assert oracle.render(sc, cam, oracle.Opts(amb_ignore=0.0), pixels=pix)["flags"][0] & 1
        else:
            assert lo["flags"][0] & 1 and hi["flags"][0] & 1


# ---------------------------------------------------------------- pose Jacobians and the IESKF update

def _twist_scene(seed):
    Rc = Rotation.from_rotvec([0.1, -0.2, 0.05]).as_matrix()
    cam0 = Camera(18.0, 19.0, 10.0, 8.0, 20, 16, Rc, [0.1, -0.05, 0.2])
    sc = S.random_scene(10, cam0, seed=seed, zmin=1.0, zmax=2.0, smin=0.08, smax=0.3)
    sc.opacity[:] = np.float32(0.3) + np.float32(0.5) * sc.opacity
    return sc, cam0


@pytest.mark.parametrize("degree", [0, 3])
def test_pose_jvp_matches_twist_differences(oracle, degree):
    """Per-pixel dI/d(dphi, dt) against central differences of the rendered
    colour under T_CW <- Exp(dphi, dt) T_CW (exponential from scipy), on the
    pixels where the steps h and 2h agree (no threshold crossed); with SH
    colour the camera centre's motion changes the colours too."""
    sc, cam0 = _twist_scene(9)
    sc = S.with_sh(sc, degree, 19, sigma=0.3)
    o = oracle.Opts(bg=(0.2, 0.1, 0.3))
    J = oracle.render_jvp(sc, cam0, o)
    flags = oracle.render(sc, cam0, o)["flags"]

    def cam_at(xi):
        E = _rodrigues(xi[:3])
        return Cam64(cam0, E @ cam0.R_cw.astype(np.float64), E @ cam0.t_cw.astype(np.float64) + xi[3:])

    h = 1e-6
    checked = 0
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        fd1 = (oracle.render(sc, cam_at(e), o)["rgb"] - oracle.render(sc, cam_at(-e), o)["rgb"]) / (2 * h)
        fd2 = (oracle.render(sc, cam_at(2 * e), o)["rgb"] - oracle.render(sc, cam_at(-2 * e), o)["rgb"]) / (4 * h)
        smooth = (np.abs(fd1 - fd2).max(1) <= 1e-4 * (1 + np.abs(fd1).max(1))) & (flags == 0)
        scale = np.abs(fd1[smooth]).max()
        np.testing.assert_allclose(J["jac"][smooth, :, k], fd1[smooth], rtol=1e-4, atol=1e-6 * scale)
        checked += int(smooth.sum())
    assert checked > 0.8 * 6 * cam0.width * cam0.height


@pytest.mark.parametrize("seed,degree", [(3, 0), (17, 0), (23, 2)])
def test_pose_jvp_adjoint_identity(oracle, seed, degree):
    """Forward and reverse mode are two separate derivations of one Jacobian:
    sum_p <v_p, dI_p/dxi> equals the pose gradient of L = sum_p <v_p, I_p>
    for any cotangent v, with background, clamped alphas and cut-off walks."""
    rng = np.random.default_rng(seed)
    Rc = Rotation.from_rotvec(rng.normal(0, 0.2, 3)).as_matrix()
    cam = Cam64(Camera(30.0, 33.0, 16.0, 12.0, 32, 24, Rc, [0, 0, 0]), Rc, rng.normal(0, 0.2, 3))
    sc = S.random_scene(120, cam, seed=seed, zmin=1.0, zmax=3.0, smin=0.05, smax=0.3, unnormalised_quats=True)
    sc.opacity[:20] = 0.999  # clamped at 0.99 near their centres
    sc = S.with_sh(sc, degree, seed + 1, sigma=0.3)
    o = oracle.Opts(bg=(0.3, 0.6, 0.1))
    J = oracle.render_jvp(sc, cam, o)
    r = oracle.render(sc, cam, o)
    assert np.array_equal(J["rgb"], r["rgb"])
    v = rng.normal(size=(cam.width * cam.height, 3))
    g = oracle.render_bwd(sc, [cam], [v], o)["pose"][0]
    lhs = np.einsum("pc,pcj->j", v, J["jac"])
    np.testing.assert_allclose(lhs, g, rtol=1e-9, atol=1e-12 * np.abs(g).max())


def test_imu_to_camera_twist_matches_perturbation_model(oracle):
    """xi_cam = A xi_imu against central differences of the exact relation
    T(xi_c) T_CW = T_CI (T_WI [+] xi_i)^-1 with (R_WI Exp(dphi), t_WI + dt)."""
    rng = np.random.default_rng(5)
    R_CI = _rodrigues(rng.normal(0, 1, 3))
    t_CI = rng.normal(0, 0.3, 3)
    R_WI = _rodrigues(rng.normal(0, 1, 3))
    t_WI = rng.normal(0, 2, 3)

    def T_CW_of(R_wi, t_wi):
        # T_CW = T_CI T_WI^-1
        R_iw, t_iw = R_wi.T, -R_wi.T @ t_wi
        return R_CI @ R_iw, R_CI @ t_iw + t_CI

    R_CW, t_CW = T_CW_of(R_WI, t_WI)
    A = oracle.imu_to_camera_twist(R_CI, t_CI, R_CW)

    def xi_c(xi_i):
        Rp, tp = T_CW_of(R_WI @ _rodrigues(xi_i[:3]), t_WI + xi_i[3:])
        E = Rp @ R_CW.T
        phi = Rotation.from_matrix(E).as_rotvec()
        return np.concatenate([phi, tp - E @ t_CW])

    h = 1e-6
    fd = np.zeros((6, 6))
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        fd[:, k] = (xi_c(e) - xi_c(-e)) / (2 * h)
    np.testing.assert_allclose(A, fd, atol=1e-7)


def test_ieskf_update_matches_gain_form(oracle):
    """The information-form update from H^T R^-1 H and H^T R^-1 z equals the
    gain form K = P H^T (H P H^T + R)^-1 on an explicit stacked model, and
    the posterior covariance equals (H^T R^-1 H + P^-1)^-1."""
    rng = np.random.default_rng(11)
    m = 40
    H = rng.normal(size=(m, 6))
    Rd = rng.uniform(0.5, 2.0, m)
    z = rng.normal(size=m)
    L = rng.normal(size=(6, 6))
    P = L @ L.T + 0.5 * np.eye(6)
    dxp = rng.normal(0, 0.1, 6)
    HtRH = H.T @ (H / Rd[:, None])
    HtRz = H.T @ (z / Rd)
    delta, Pn = oracle.ieskf_pose_update(HtRH, HtRz, P, dxp)
    K = P @ H.T @ np.linalg.inv(H @ P @ H.T + np.diag(Rd))
    np.testing.assert_allclose(delta, -K @ z - (np.eye(6) - K @ H) @ dxp, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Pn, (np.eye(6) - K @ H) @ P, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Pn, np.linalg.inv(HtRH + np.linalg.inv(P)), rtol=1e-9, atol=1e-12)
    # the normal equations of the oracle's per-pixel form agree with the explicit stacking
    jac = H[: 3 * (m // 3)].reshape(-1, 3, 6)
    res = z[: 3 * (m // 3)].reshape(-1, 3)
    w = rng.uniform(0.5, 2.0, m // 3)
    A, b, zz = oracle.normal_equations(jac, res, w)
    Hs = jac.reshape(-1, 6)
    ws = np.repeat(w, 3)
    np.testing.assert_allclose(A, sum(ws[i] * np.outer(Hs[i], Hs[i]) for i in range(len(ws))), rtol=1e-12)
    np.testing.assert_allclose(b, sum(ws[i] * Hs[i] * res.reshape(-1)[i] for i in range(len(ws))), rtol=1e-12)


def test_ieskf_visual_update_matches_stacked_imu_model(oracle):
    """The IMU-pose update from the camera's normal equations equals the gain
    form on an explicitly stacked model in the IMU twist: H_imu = H_cam A row
    by row, R = noise_var I, K = P H_imu^T (H_imu P H_imu^T + R)^-1."""
    rng = np.random.default_rng(13)
    m = 45
    H_cam = rng.normal(size=(m, 6))
    z = rng.normal(size=m)
    from scipy.spatial.transform import Rotation
    A = oracle.imu_to_camera_twist(Rotation.from_rotvec(rng.normal(size=3)).as_matrix(), rng.normal(0, 0.2, 3),
                                   Rotation.from_rotvec(rng.normal(size=3)).as_matrix())
    L = rng.normal(size=(6, 6))
    P = L @ L.T + 0.3 * np.eye(6)
    dxp = rng.normal(0, 0.05, 6)
    nv = 0.7
    delta, Pn = oracle.ieskf_visual_update(H_cam.T @ H_cam, H_cam.T @ z, A, P, dxp, noise_var=nv)
    H = np.stack([A.T @ h for h in H_cam])  # each row h_imu = h_cam A
    K = P @ H.T @ np.linalg.inv(H @ P @ H.T + nv * np.eye(m))
    np.testing.assert_allclose(delta, -K @ z - (np.eye(6) - K @ H) @ dxp, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Pn, (np.eye(6) - K @ H) @ P, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------- Adam

def test_deactivate_inverts_activate(oracle):
    """deactivate is the inverse of activate (round trips both ways, with SH
    rows), and hand-worked values: scale 1 -> 0, e -> 1; opacity 1/2 -> 0,
    1 / (1 + e^-2) -> 2, 1 / (1 + e^3) -> -3."""
    rng = np.random.default_rng(5)
    raw = rng.normal(size=(14 + 9, 6))
    back = oracle.deactivate(oracle.activate(raw))
    np.testing.assert_allclose(back, raw, rtol=0, atol=1e-12)
    act = oracle.activate(raw)
    again = oracle.activate(oracle.deactivate(act))
    for k in act:
        np.testing.assert_allclose(again[k], act[k], rtol=1e-13, atol=1e-15)
    e = np.e
    act = {"mean": np.zeros((3, 3)), "scale": np.array([[1.0, e, e * e]] * 3), "quat": np.ones((4, 3)),
           "opacity": np.array([[0.5, 1.0 / (1.0 + e ** -2), 1.0 / (1.0 + e ** 3)]]), "color": np.full((3, 3), 0.25)}
    r = oracle.deactivate(act)
    np.testing.assert_allclose(r[3:6], [[0.0, 1.0, 2.0]] * 3, atol=1e-15)
    np.testing.assert_allclose(r[10], [0.0, 2.0, -3.0], atol=1e-14)
    np.testing.assert_array_equal(r[11:14], act["color"])

def test_adam_constant_gradient_closed_form(oracle):
    """For a gradient that stays g, the bias-corrected moments are exactly g
    and g^2, so every step moves by -lr g / (|g| + eps); the first step of any
    gradient sequence is the same."""
    rng = np.random.default_rng(2)
    raw = rng.normal(size=(14, 7))
    g = rng.normal(size=(14, 7))
    lr = np.linspace(1e-3, 1e-2, 14)
    m = np.zeros_like(raw)
    v = np.zeros_like(raw)
    x = raw.copy()
    for t in range(1, 6):
        x, m, v = oracle.adam_step(x, m, v, g, t, lr, eps=1e-8)
        want = raw - t * lr[:, None] * g / (np.abs(g) + 1e-8)
        np.testing.assert_allclose(x, want, rtol=1e-12, atol=1e-12)


def test_adam_matches_scalar_recursion(oracle):
    """A changing gradient, against the recursion written for one scalar."""
    rng = np.random.default_rng(3)
    gs = rng.normal(size=12)
    x, m, v = 0.5, 0.0, 0.0
    X, M, V = np.full((14, 1), 0.5), np.zeros((14, 1)), np.zeros((14, 1))
    for t, g in enumerate(gs, 1):
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        x = x - 0.01 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-15)
        X, M, V = oracle.adam_step(X, M, V, np.full((14, 1), g), t, 0.01)
    np.testing.assert_allclose(X[:, 0], x, rtol=1e-13)


@pytest.mark.parametrize("rows", [14, 14 + 9])
def test_activation_chain_matches_differences(oracle, rows):
    """raw_gradient against central differences of a linear functional of the
    activated parameters (with SH coefficient rows after the colour)."""
    rng = np.random.default_rng(4)
    raw = rng.normal(size=(rows, 5))
    W = {k: rng.normal(size=(b - a, 5)) for k, (a, b) in oracle.RAW_ROWS.items()}
    if rows > 14:
        W["sh"] = rng.normal(size=(rows - 14, 5))

    def f(r):
        act = oracle.activate(r)
        return sum(float((W[k] * act[k]).sum()) for k in W)

    g = oracle.raw_gradient(raw, W)
    h = 1e-6
    fd = np.zeros_like(raw)
    for idx in np.ndindex(*raw.shape):
        e = np.zeros_like(raw)
        e[idx] = h
        fd[idx] = (f(raw + e) - f(raw - e)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)  # central-difference rounding at h = 1e-6


# ---------------------------------------------------------------- window maintenance

def test_window_maintain_worked_example(oracle):
    """Eight Gaussians, keys 10..17, field of view {10, 12, 13, 15, 16, 17, 99}:
    11 and 14 are deleted (D = 2); the holes before n - D = 6 are slots 1 and 4,
    filled by the kept Gaussians of the rear [6, 8) in order (16 -> 1, 17 -> 4);
    then 20 and 21 are appended."""
    keys = np.arange(10, 18, dtype=np.uint64)
    rows = np.stack([keys.astype(np.float32), -keys.astype(np.float32)])
    k, r, ek, er = oracle.window_maintain(keys, rows, [10, 12, 13, 15, 16, 17, 99], np.array([20, 21], np.uint64),
                                          np.array([[20, 21], [-20, -21]], np.float32))
    assert k.tolist() == [10, 16, 12, 13, 17, 15, 20, 21]
    assert r[0].tolist() == [10, 16, 12, 13, 17, 15, 20, 21] and r[1].tolist() == [-x for x in r[0].tolist()]
    assert ek.tolist() == [11, 14] and er[0].tolist() == [11, 14]


def test_window_maintain_invariants(oracle):
    """Random windows: the kept keys are exactly the window keys in the field
    of view, front Gaussians that are kept do not move, every Gaussian keeps
    its own parameters, evicted are the rest in window order."""
    rng = np.random.default_rng(8)
    for trial in range(20):
        n = int(rng.integers(0, 200))
        keys = rng.permutation(10_000)[:n].astype(np.uint64)
        rows = rng.normal(size=(3, n)).astype(np.float32)
        rows[0] = keys
        fov = rng.choice(10_000, 5000, replace=False)
        add = np.arange(20_000, 20_000 + int(rng.integers(0, 30)), dtype=np.uint64)
        add_rows = np.stack([add.astype(np.float32), np.zeros(len(add), np.float32), np.ones(len(add), np.float32)])
        k, r, ek, er = oracle.window_maintain(keys, rows, fov, add, add_rows)
        inf = np.isin(keys, fov)
        D = int((~inf).sum())
        assert sorted(k[: n - D].tolist()) == sorted(keys[inf].tolist())
        assert k[n - D:].tolist() == add.tolist()
        front_kept = np.nonzero(inf[: n - D])[0]
        assert np.array_equal(k[front_kept], keys[front_kept])
        np.testing.assert_array_equal(r[0], k.astype(np.float32))
        assert ek.tolist() == keys[~inf].tolist()
        np.testing.assert_array_equal(er, rows[:, ~inf])


def _unpack(key):
    m = (1 << 21) - 1
    return ((int(key) >> 42) & m) - (1 << 20), ((int(key) >> 21) & m) - (1 << 20), (int(key) & m) - (1 << 20)


def test_voxel_key_floor_and_packing(oracle):
    """floor, not truncation, on negative coordinates; a coordinate exactly on
    a voxel face belongs to the voxel above; the packed fields decode to the
    indices; out-of-range and non-finite points have no key."""
    pts = np.array([[0.26, -0.1, 1.0], [-0.5, 0.0, 0.49], [6.0e5, 0, 0], [np.nan, 0, 0]], np.float32)  # 6e5 / 0.5 >= 2^20
    k, ok = oracle.voxel_key(pts, 0.5)
    assert ok.tolist() == [True, True, False, False]
    assert _unpack(k[0]) == (0, -1, 2)
    assert _unpack(k[1]) == (-1, 0, 0)
    assert int(k[0]) == (1 << 62) | ((1 << 20) - 1 << 21) | ((1 << 20) + 2)
    assert k[2] == 0 and k[3] == 0


def test_voxel_key_cell_contains_point(oracle):
    """The voxel a key names contains the point: i v_s <= p < (i + 1) v_s per
    axis, exactly (float32 inputs make fp64 products and the quotient's floor
    exact), and two points share a key iff they share every index."""
    rng = np.random.default_rng(3)
    pts = (rng.normal(size=(400, 3)) * 40).astype(np.float32)
    pts[:50] = np.round(pts[:50] / 0.4) * np.float32(0.4)  # near voxel faces
    for vs in (0.4, 1.0, 0.25):
        k, ok = oracle.voxel_key(pts, vs)
        assert ok.all()
        v = float(np.float32(vs))
        for j in range(len(pts)):
            idx = _unpack(k[j])
            for a in range(3):
                assert idx[a] * v <= float(pts[j, a]) < (idx[a] + 1) * v
        i_all = np.floor(pts.astype(np.float64) / v).astype(np.int64)
        same_key = k[:, None] == k[None, :]
        same_idx = (i_all[:, None, :] == i_all[None, :, :]).all(-1)
        assert np.array_equal(same_key, same_idx)


def test_window_classify_worked_example(oracle):
    """Window keys [5, 7, 5, 9, 11]; frame keys [7, 3, 7, 12, 5, 3, x(invalid)]:
    the field of view is {3, 5, 7, 12}; 9 and 11 are DELETE; ADD is 3 then 12
    (order of first appearance), each once."""
    d, add = oracle.window_classify(np.array([5, 7, 5, 9, 11], np.uint64),
                                    np.array([7, 3, 7, 12, 5, 3, 9], np.uint64),
                                    np.array([1, 1, 1, 1, 1, 1, 0], bool))
    assert d.tolist() == [False, False, False, True, True]
    assert add.tolist() == [3, 12]


def test_window_classify_set_identities(oracle):
    """ADD and the kept window keys partition the field of view; ADD keys are
    unique, absent from the window, and ordered by first appearance."""
    rng = np.random.default_rng(5)
    for trial in range(10):
        win = rng.integers(0, 300, int(rng.integers(0, 400))).astype(np.uint64)
        pk = rng.integers(100, 500, int(rng.integers(0, 600))).astype(np.uint64)
        ok = rng.random(len(pk)) > 0.1
        d, add = oracle.window_classify(win, pk, ok)
        fov = set(pk[ok].tolist())
        kept = set(win[~d].tolist())
        assert kept <= fov and set(win[d].tolist()).isdisjoint(fov)
        assert len(set(add.tolist())) == len(add) and set(add.tolist()).isdisjoint(set(win.tolist()))
        assert kept | set(add.tolist()) == fov
        first = [int(np.nonzero((pk == a) & ok)[0][0]) for a in add]
        assert first == sorted(first)


# ---------------------------------------------------------------- view-dependent colour

def _real_sh_scipy(l, m, u):
    """Real orthonormal Y_lm from scipy's complex harmonics (with the
    Condon-Shortley phase), made real as sqrt(2) (-1)^m Re / Im."""
    from scipy.special import sph_harm_y
    theta = np.arccos(np.clip(u[:, 2], -1, 1))
    phi = np.arctan2(u[:, 1], u[:, 0])
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    Y = sph_harm_y(l, abs(m), theta, phi)
    return np.sqrt(2.0) * (-1) ** m * (Y.real if m > 0 else Y.imag)


def _unit(rng, n):
    u = rng.normal(size=(n, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def test_sh_basis_matches_scipy(oracle):
    """The Cartesian polynomials against scipy's spherical harmonics, every
    (l, m) up to degree 3, times Y_00 = 1 / (2 sqrt(pi))."""
    u = _unit(np.random.default_rng(1), 200)
    B = oracle.sh_basis(u, 3) * (0.5 / np.sqrt(np.pi))
    k = 0
    for l in range(1, 4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(B[:, k], _real_sh_scipy(l, m, u), atol=1e-12, err_msg=f"l={l} m={m}")
            k += 1
    assert oracle.sh_basis(u, 1).shape == (200, 3) and oracle.sh_basis(u, 2).shape == (200, 8)


def test_sh_basis_orthogonal_on_sphere(oracle):
    """Gauss-Legendre in cos(theta) x uniform phi (exact for these degrees):
    the integral of B_i B_j over the sphere is 4 pi delta_ij, and of B_i is 0."""
    xg, wg = np.polynomial.legendre.leggauss(10)
    nphi = 16
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    u = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    B = oracle.sh_basis(u, 3)
    G = (B * w[:, None]).T @ B
    np.testing.assert_allclose(G, 4 * np.pi * np.eye(15), atol=1e-11)
    np.testing.assert_allclose(w @ B, np.zeros(15), atol=1e-11)


def test_sh_basis_grad_matches_differences(oracle):
    rng = np.random.default_rng(2)
    u = rng.normal(size=(50, 3))
    g = oracle.sh_basis_grad(u, 3)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (oracle.sh_basis(u + e, 3) - oracle.sh_basis(u - e, 3)) / (2 * h)
        np.testing.assert_allclose(g[:, :, a], fd, rtol=1e-7, atol=1e-8)


def _sh_scene(seed, degree, n=6, W=20, H=16):
    sc, cam = _fd_scene(seed, n=n, W=W, H=H)
    return S.with_sh(sc, degree, seed + 100, sigma=0.3), cam


@pytest.mark.parametrize("degree", [1, 3])
def test_sh_colour_vjp_matches_differences(oracle, degree):
    """The adjoint of the view-dependent colour against central differences
    in the coefficients, the means and the camera translation."""
    sc, cam = _sh_scene(5, degree)
    Rc = Rotation.from_rotvec([0.2, -0.1, 0.3]).as_matrix()
    cam = Cam64(cam, Rc, [0.3, -0.2, 0.1])
    rng = np.random.default_rng(6)
    gc = rng.normal(size=(sc.n, 3))
    gcol, gsh, gm, gdt = oracle.sh_colour_vjp(sc, cam, gc)
    f = lambda s, c: float(np.sum(oracle.sh_colour(s, c) * gc))
    base = {k: np.asarray(getattr(sc, k), np.float64).copy() for k in ("mean", "color", "sh")}
    h = 1e-6
    for name, an in (("mean", gm), ("color", gcol), ("sh", gsh)):
        fd = np.zeros_like(base[name])
        for idx in np.ndindex(base[name].shape):
            vals = []
            for sgn in (1, -1):
                s2 = replace(sc)
                for k in base:
                    setattr(s2, k, base[k].copy())
                getattr(s2, name)[idx] += sgn * h
                vals.append(f(s2, cam))
            fd[idx] = (vals[0] - vals[1]) / (2 * h)
        np.testing.assert_allclose(an, fd, rtol=1e-6, atol=1e-8, err_msg=name)
    s64 = replace(sc)
    for k in base:
        setattr(s64, k, base[k].copy())
    fd = np.zeros(3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd[a] = (f(s64, Cam64(cam, cam.R_cw, cam.t_cw + e)) - f(s64, Cam64(cam, cam.R_cw, cam.t_cw - e))) / (2 * h)
    np.testing.assert_allclose(gdt, fd, rtol=1e-6, atol=1e-8)
    # a rotation about the camera centre leaves the view directions unchanged
    E = _rodrigues([1e-3, -2e-3, 5e-4])
    np.testing.assert_allclose(oracle.sh_colour(s64, Cam64(cam, E @ cam.R_cw, E @ cam.t_cw)),
                               oracle.sh_colour(s64, cam), atol=1e-12)


def test_sh_render_gradients_match_differences(oracle):
    """Through the whole render: the SH coefficients, the means (whose colour
    now depends on the view direction) and the pose translation."""
    sc, cam0 = _sh_scene(7, 2, n=5)
    Rc = Rotation.from_rotvec([0.05, -0.1, 0.02]).as_matrix()
    cam = Cam64(cam0, Rc, [0.05, -0.02, 0.1])
    o = oracle.Opts(bg=(0.2, 0.1, 0.3))
    rng = np.random.default_rng(8)
    Wimg = rng.normal(size=(3, cam.height, cam.width))
    Wimg[:, oracle.render_image(sc, cam, o)["flags"] != 0] = 0
    g = oracle.render_bwd(sc, [cam], [Wimg], o)
    base = {k: np.asarray(getattr(sc, k), np.float64).copy() for k in ("mean", "scale", "quat", "opacity", "color",
                                                                       "sh")}

    def L(params, c=cam):
        s2 = replace(sc)
        for k in params:
            setattr(s2, k, params[k])
        return _loss(oracle, s2, [c], [Wimg], o)

    h = 1e-6
    for name in ("sh", "mean", "color"):
        fd = np.zeros_like(base[name])
        for idx in np.ndindex(base[name].shape):
            vals = []
            for sgn in (1, -1):
                p = {k: v.copy() for k, v in base.items()}
                p[name][idx] += sgn * h
                vals.append(L(p))
            fd[idx] = (vals[0] - vals[1]) / (2 * h)
        np.testing.assert_allclose(g[name], fd, atol=2e-6 * np.abs(fd).max() + 1e-9, rtol=2e-5, err_msg=name)
    fd = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        cams = []
        for sgn in (1, -1):
            E = _rodrigues(sgn * e[:3])
            cams.append(Cam64(cam, E @ cam.R_cw, E @ cam.t_cw + sgn * e[3:]))
        fd[k] = (L(base, cams[0]) - L(base, cams[1])) / (2 * h)
    np.testing.assert_allclose(g["pose"][0], fd, rtol=2e-5, atol=1e-6 * np.abs(fd).max())


def _backproject(cam, u, v, z):
    """World points that project to pixel coordinates (u, v) at depth z."""
    pc = np.stack([(u - cam.cx) / cam.fx * z, (v - cam.cy) / cam.fy * z, z], -1)
    R = np.asarray(cam.R_cw, np.float64)
    return (pc - np.asarray(cam.t_cw, np.float64)) @ R


def test_bilinear_colour_pixel_centres_and_affine_images(oracle):
    """At a pixel centre the colour is that pixel; an image affine in (u, v)
    per channel is reproduced exactly anywhere between centres; the midpoint
    of four centres gives their mean."""
    rng = np.random.default_rng(9)
    Rc = Rotation.from_rotvec([0.1, 0.2, -0.1]).as_matrix()
    cam = Cam64(_cam(W=17, H=11, f=20.0), Rc, [0.1, 0.0, -0.2])
    img = rng.uniform(size=(3, 11, 17))
    ii, jj = rng.integers(0, 17, 30), rng.integers(0, 11, 30)
    pts = _backproject(cam, ii + 0.5, jj + 0.5, rng.uniform(1, 5, 30))
    c, ok = oracle.bilinear_colour(pts, cam, img)
    assert ok.all()
    np.testing.assert_allclose(c, img[:, jj, ii].T, atol=1e-12)
    # affine image: c_ch(u, v) = a_ch + b_ch (u - 1/2) + d_ch (v - 1/2) at the pixel centres
    a, b, d = rng.normal(size=3), rng.normal(size=3), rng.normal(size=3)
    V, U = np.mgrid[0:11, 0:17]
    aff = a[:, None, None] + b[:, None, None] * U + d[:, None, None] * V
    u = rng.uniform(0.5, 16.5, 200)
    v = rng.uniform(0.5, 10.5, 200)
    c, ok = oracle.bilinear_colour(_backproject(cam, u, v, rng.uniform(1, 5, 200)), cam, aff)
    assert ok.all()
    want = a[None] + b[None] * (u - 0.5)[:, None] + d[None] * (v - 0.5)[:, None]
    np.testing.assert_allclose(c, want, atol=1e-9)
    # midpoint of the centres of (3, 4), (4, 4), (3, 5), (4, 5)
    c, _ = oracle.bilinear_colour(_backproject(cam, np.array([4.0]), np.array([5.0]), np.array([2.0])), cam, img)
    np.testing.assert_allclose(c[0], img[:, 4:6, 3:5].mean((1, 2)), atol=1e-12)


def test_bilinear_colour_borders_and_invalid(oracle):
    """Between the image border and the outer pixel centres the edge pixel
    value holds (clamp); behind the near plane or outside the image nothing."""
    cam = _cam(W=8, H=6, f=10.0)
    rng = np.random.default_rng(10)
    img = rng.uniform(size=(3, 6, 8))
    pts = _backproject(cam, np.array([0.2, 7.9, 0.1, 4.0]), np.array([0.3, 5.9, 3.0, -0.5]), np.array([2.0] * 4))
    c, ok = oracle.bilinear_colour(pts, cam, img)
    assert ok.tolist() == [True, True, True, False]
    np.testing.assert_allclose(c[0], img[:, 0, 0], atol=1e-12)
    np.testing.assert_allclose(c[1], img[:, 5, 7], atol=1e-12)
    np.testing.assert_allclose(c[2], 0.5 * (img[:, 2, 0] + img[:, 3, 0]), atol=1e-12)
    behind = _backproject(cam, np.array([4.0]), np.array([3.0]), np.array([0.1]))
    assert not oracle.bilinear_colour(behind, cam, img)[1][0]
