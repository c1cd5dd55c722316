"""Seeded synthetic Gaussian scenes and camera sets.

Every array is produced in float64 by numpy's PCG64 generator and then rounded
to float32 once, so that the GPU path (which reads float32) and the FP64
oracle (which widens the same float32 values) start from identical inputs.

Shapes follow the paper's workloads: LiDAR-initialised surfel Gaussians
(Sec. II-B: a thin scale along the surface normal, rotation built from the
normal) and the evaluation settings of Sec. III (640x480 with a
100k-Gaussian window, 256x216 with a 20k window on the embedded board).
The public datasets of Sec. III-A are not available here; these scenes stand
in for them.

Conventions shared by all consumers:
  * means, scales: (N, 3); quats: (N, 4) as (w, x, y, z), not necessarily
    unit length; opacity: (N,) in (0, 1); color: (N, 3) degree-0 RGB.
  * scales and opacities are activated values (metres, probability).
  * a camera maps world points to camera coordinates as p_C = R_cw p_W + t_cw,
    with x right, y down, z forward; pixel (u, v) covers [u, u+1) x [v, v+1).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

F32 = np.float32


@dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    R_cw: np.ndarray  # (3, 3) float32, world -> camera rotation
    t_cw: np.ndarray  # (3,) float32

    def __post_init__(self):
        self.fx = float(np.float32(self.fx))
        self.fy = float(np.float32(self.fy))
        self.cx = float(np.float32(self.cx))
        self.cy = float(np.float32(self.cy))
        self.width = int(self.width)
        self.height = int(self.height)
        self.R_cw = np.ascontiguousarray(self.R_cw, dtype=F32).reshape(3, 3)
        self.t_cw = np.ascontiguousarray(self.t_cw, dtype=F32).reshape(3)

    @property
    def npix(self) -> int:
        return self.width * self.height


@dataclass
class Scene:
    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    color: np.ndarray
    cams: List[Camera] = field(default_factory=list)
    name: str = ""
    sh: Optional[np.ndarray] = None  # (N, K, 3) higher-order SH coefficients, K = (degree + 1)^2 - 1

    def __post_init__(self):
        self.mean = np.ascontiguousarray(self.mean, dtype=F32)
        self.scale = np.ascontiguousarray(self.scale, dtype=F32)
        self.quat = np.ascontiguousarray(self.quat, dtype=F32)
        self.opacity = np.ascontiguousarray(self.opacity, dtype=F32).reshape(-1)
        self.color = np.ascontiguousarray(self.color, dtype=F32)
        n = self.mean.shape[0]
        assert self.mean.shape == (n, 3) and self.scale.shape == (n, 3)
        assert self.quat.shape == (n, 4) and self.opacity.shape == (n,)
        assert self.color.shape == (n, 3)
        if self.sh is not None:
            self.sh = np.ascontiguousarray(self.sh, dtype=F32)
            assert self.sh.ndim == 3 and self.sh.shape[0] == n and self.sh.shape[2] == 3
            assert self.sh.shape[1] in (3, 8, 15)

    @property
    def sh_degree(self) -> int:
        return 0 if self.sh is None else {3: 1, 8: 2, 15: 3}[self.sh.shape[1]]

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return replace(self, mean=self.mean[idx], scale=self.scale[idx], quat=self.quat[idx],
                       opacity=self.opacity[idx], color=self.color[idx],
                       sh=None if self.sh is None else self.sh[idx])

    def permuted(self, perm) -> "Scene":
        return self.subset(perm)

    def digest(self) -> str:
        import hashlib
        h = hashlib.sha1()
        for a in (self.mean, self.scale, self.quat, self.opacity, self.color):
            h.update(np.ascontiguousarray(a).tobytes())
        if self.sh is not None:
            h.update(self.sh.tobytes())
        for c in self.cams:
            h.update(np.array([c.fx, c.fy, c.cx, c.cy, c.width, c.height], np.float64).tobytes())
            h.update(c.R_cw.tobytes())
            h.update(c.t_cw.tobytes())
        return h.hexdigest()[:16]


# ----------------------------------------------------------------------------
# small rotation helpers used only to build inputs
# ----------------------------------------------------------------------------

def so3_exp(w) -> np.ndarray:
    """Rotation matrix of the axis-angle vector w (Rodrigues' formula)."""
    w = np.asarray(w, np.float64)
    th = float(np.linalg.norm(w))
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / th**2 * (K @ K)


def _quat_from_matrix(R: np.ndarray) -> np.ndarray:
    """(w, x, y, z) unit quaternions of a stack of rotation matrices (Shepperd)."""
    R = np.asarray(R, np.float64).reshape(-1, 3, 3)
    q = np.empty((R.shape[0], 4))
    tr = R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2]
    d = np.stack([tr, R[:, 0, 0], R[:, 1, 1], R[:, 2, 2]], 1)
    k = np.argmax(d, 1)
    for case in range(4):
        m = k == case
        if not np.any(m):
            continue
        Rm = R[m]
        if case == 0:
            s = np.sqrt(1.0 + tr[m]) * 2
            q[m] = np.stack([0.25 * s, (Rm[:, 2, 1] - Rm[:, 1, 2]) / s,
                             (Rm[:, 0, 2] - Rm[:, 2, 0]) / s, (Rm[:, 1, 0] - Rm[:, 0, 1]) / s], 1)
        elif case == 1:
            s = np.sqrt(1.0 + Rm[:, 0, 0] - Rm[:, 1, 1] - Rm[:, 2, 2]) * 2
            q[m] = np.stack([(Rm[:, 2, 1] - Rm[:, 1, 2]) / s, 0.25 * s,
                             (Rm[:, 0, 1] + Rm[:, 1, 0]) / s, (Rm[:, 0, 2] + Rm[:, 2, 0]) / s], 1)
        elif case == 2:
            s = np.sqrt(1.0 + Rm[:, 1, 1] - Rm[:, 0, 0] - Rm[:, 2, 2]) * 2
            q[m] = np.stack([(Rm[:, 0, 2] - Rm[:, 2, 0]) / s, (Rm[:, 0, 1] + Rm[:, 1, 0]) / s,
                             0.25 * s, (Rm[:, 1, 2] + Rm[:, 2, 1]) / s], 1)
        else:
            s = np.sqrt(1.0 + Rm[:, 2, 2] - Rm[:, 0, 0] - Rm[:, 1, 1]) * 2
            q[m] = np.stack([(Rm[:, 1, 0] - Rm[:, 0, 1]) / s, (Rm[:, 0, 2] + Rm[:, 2, 0]) / s,
                             (Rm[:, 1, 2] + Rm[:, 2, 1]) / s, 0.25 * s], 1)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def camera_from_pose(R_wc, center, width, height, f=None, fx=None, fy=None, cx=None, cy=None) -> Camera:
    """Camera from a camera-to-world rotation and the camera centre in world coordinates."""
    R_wc = np.asarray(R_wc, np.float64)
    center = np.asarray(center, np.float64)
    fx = f if fx is None else fx
    fy = f if fy is None else fy
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    R_cw = R_wc.T
    return Camera(fx, fy, cx, cy, width, height, R_cw, -R_cw @ center)


def look_camera(width, height, f, center=(0, 0, 0), yaw=0.0, pitch=0.0, roll=0.0) -> Camera:
    """Camera at `center`, rotated by yaw (about y), then pitch (about x), then roll (about z)."""
    R_wc = so3_exp([0, yaw, 0]) @ so3_exp([pitch, 0, 0]) @ so3_exp([0, 0, roll])
    return camera_from_pose(R_wc, center, width, height, f)


def perturb_camera(cam: Camera, dphi, dt) -> Camera:
    """Left-perturbed copy: R_cw <- Exp(dphi) R_cw, t_cw <- Exp(dphi) t_cw + dt."""
    E = so3_exp(dphi)
    R = E @ cam.R_cw.astype(np.float64)
    t = E @ cam.t_cw.astype(np.float64) + np.asarray(dt, np.float64)
    return Camera(cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, R, t)


# ----------------------------------------------------------------------------
# Gaussian distributions
# ----------------------------------------------------------------------------

def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _uniform_quats(rng, n):
    q = rng.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def random_scene(n, cam: Camera, seed, zmin=1.0, zmax=5.0, smin=0.01, smax=0.1, name="random",
                 unnormalised_quats=False) -> Scene:
    """Means uniform in the volume of `cam`'s frustum between depths zmin and zmax.

    Scales are log-uniform per axis in [smin, smax] metres, rotations uniform
    on SO(3), opacity sigmoid(N(0, 1)), colour uniform in [0, 1]^3.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    # depth with density proportional to z^2 (uniform in the frustum volume)
    u = rng.uniform(size=n)
    z = (zmin**3 + u * (zmax**3 - zmin**3)) ** (1.0 / 3.0)
    px = rng.uniform(0, cam.width, n)
    py = rng.uniform(0, cam.height, n)
    x = (px - cam.cx) / cam.fx * z
    y = (py - cam.cy) / cam.fy * z
    pc = np.stack([x, y, z], 1)
    R = cam.R_cw.astype(np.float64)
    pw = (pc - cam.t_cw.astype(np.float64)) @ R  # R^T (p_C - t)
    scale = _log_uniform(rng, smin, smax, (n, 3))
    quat = _uniform_quats(rng, n)
    if unnormalised_quats:
        quat = quat * rng.uniform(0.5, 2.0, (n, 1))
    opacity = _sigmoid(rng.normal(size=n))
    color = rng.uniform(0, 1, (n, 3))
    return Scene(pw, scale, quat, opacity, color, [cam], name)


def _plane_frame(normal):
    """Orthonormal (a, b, n) with the first column built from e_x x n (e_y when e_x is parallel to n)."""
    n = normal / np.linalg.norm(normal)
    ex = np.array([1.0, 0.0, 0.0])
    a = np.cross(ex, n)
    if np.linalg.norm(a) < 1e-6:
        a = np.cross(np.array([0.0, 1.0, 0.0]), n)
    a = a / np.linalg.norm(a)
    b = np.cross(n, a)
    return a, b, n


def surface_scene(n_planes, per_plane, seed, centers, patch=4.0, normal_sigma=0.01,
                  smin=0.01, smax=0.1, s_delta=1e-3, name="surface") -> Scene:
    """Surfel Gaussians on random planar patches, as a LiDAR-initialised map would hold.

    `centers` is an (n_planes, 3) array of patch centres.  Each patch is a
    square of side `patch` metres with a normal uniform on the sphere; points
    are uniform on the square with N(0, normal_sigma) offsets along the normal.
    Each Gaussian's rotation has the surface normal as its third column and
    the first column from e_x x n (Sec. II-B), twisted by a random in-plane
    angle; the normal axis gets the small scale s_delta and the two in-plane
    axes log-uniform scales in [smin, smax].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centers = np.asarray(centers, np.float64).reshape(n_planes, 3)
    N = n_planes * per_plane
    mean = np.empty((N, 3))
    Rs = np.empty((N, 3, 3))
    for p in range(n_planes):
        nrm = rng.normal(size=3)
        a, b, nv = _plane_frame(nrm)
        uv = rng.uniform(-patch / 2, patch / 2, (per_plane, 2))
        off = rng.normal(0.0, normal_sigma, per_plane)
        sl = slice(p * per_plane, (p + 1) * per_plane)
        mean[sl] = centers[p] + uv[:, :1] * a + uv[:, 1:] * b + off[:, None] * nv
        th = rng.uniform(0, 2 * np.pi, per_plane)
        c, s = np.cos(th)[:, None], np.sin(th)[:, None]
        a2 = c * a + s * b
        b2 = -s * a + c * b
        Rs[sl, :, 0] = a2
        Rs[sl, :, 1] = b2
        Rs[sl, :, 2] = nv
    quat = _quat_from_matrix(Rs)
    scale = np.empty((N, 3))
    scale[:, :2] = _log_uniform(rng, smin, smax, (N, 2))
    scale[:, 2] = s_delta
    opacity = _sigmoid(rng.normal(size=N))
    color = rng.uniform(0, 1, (N, 3))
    return Scene(mean, scale, quat, opacity, color, [], name)


def frustum_points(rng, cam: Camera, n, zmin, zmax):
    """n world points uniform in pixel coordinates and uniform in depth inside cam's view."""
    z = rng.uniform(zmin, zmax, n)
    px = rng.uniform(0, cam.width, n)
    py = rng.uniform(0, cam.height, n)
    pc = np.stack([(px - cam.cx) / cam.fx * z, (py - cam.cy) / cam.fy * z, z], 1)
    return (pc - cam.t_cw.astype(np.float64)) @ cam.R_cw.astype(np.float64)


def jitter_means(scene: Scene, sigma, seed) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    m = scene.mean.astype(np.float64) + rng.normal(0.0, sigma, scene.mean.shape)
    return replace(scene, mean=m.astype(F32), name=scene.name + "+jitter")


def trajectory_cameras(n, width, height, f, seed, step=0.3, turn_deg=5.0):
    """n keyframes on a smooth random path: consecutive centres `step` metres and
    consecutive orientations `turn_deg` degrees apart, the heading drifting smoothly.
    The world frame is the middle keyframe's camera frame."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Rwc = [np.eye(3)]
    C = [np.zeros(3)]
    head = rng.uniform(0, 2 * np.pi)
    d = np.array([np.cos(head), 0.0, np.sin(head)])
    axis = np.array([0.0, 1.0, 0.0])
    turn = np.deg2rad(turn_deg)
    for _ in range(n - 1):
        d = d + 0.25 * rng.normal(size=3) * np.array([1.0, 0.3, 1.0])
        d /= np.linalg.norm(d)
        axis = axis + 0.2 * rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        C.append(C[-1] + step * (Rwc[-1] @ d))
        Rwc.append(Rwc[-1] @ so3_exp(turn * axis))
    mid = n // 2
    R0, C0 = Rwc[mid], C[mid]
    cams = []
    for R, c in zip(Rwc, C):
        cams.append(camera_from_pose(R0.T @ R, R0.T @ (c - C0), width, height, f))
    return cams


def with_sh(scene: Scene, degree: int, seed, sigma=0.15) -> Scene:
    """The scene with view-dependent colour: higher-order SH coefficients of
    degrees 1..degree drawn N(0, sigma / l) per channel (degree l), the
    degree-0 coefficient being the scene's colour."""
    if degree == 0:
        return replace(scene, sh=None)
    rng = np.random.Generator(np.random.PCG64(seed))
    K = (degree + 1) ** 2 - 1
    lvl = np.array([l for l in range(1, degree + 1) for _ in range(2 * l + 1)], np.float64)
    sh = rng.normal(size=(scene.n, K, 3)) * (sigma / lvl)[None, :, None]
    return replace(scene, sh=sh.astype(F32), name=scene.name + f"+sh{degree}")


def lidar_stream(seed, frames, points_per_frame, n_window, extent=80.0, n_planes=600, patch=6.0,
                 range_m=20.0, step=1.0, nan_frac=0.01, mean_sigma=0.05):
    """A synthetic LiDAR stream for the sliding-window update (Sec. II-C).

    The world is a corridor of planar patches (centres uniform in
    [0, extent] x [-8, 8] x [-3, 3] m, normals uniform on the sphere, side
    `patch` m), densely sampled once.  The sensor moves along +x by `step`
    metres per frame starting at x = range_m; frame k holds points_per_frame
    samples (with replacement) of the surface points within range_m of the
    sensor, a `nan_frac` share of them replaced by NaN returns.  The initial
    window is n_window Gaussian means: samples of frame 0's points with
    N(0, mean_sigma) offsets.  Returns (list of (P, 3) float32 arrays,
    (n_window, 3) float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per = 8000
    cloud = np.empty((n_planes * per, 3))
    for p in range(n_planes):
        c = np.array([rng.uniform(0, extent), rng.uniform(-8, 8), rng.uniform(-3, 3)])
        a, b, _ = _plane_frame(rng.normal(size=3))
        uv = rng.uniform(-patch / 2, patch / 2, (per, 2))
        cloud[p * per:(p + 1) * per] = c + uv[:, :1] * a + uv[:, 1:] * b
    out = []
    for k in range(frames):
        sensor = np.array([range_m + k * step, 0.0, 0.0])
        near = cloud[np.sum((cloud - sensor) ** 2, 1) <= range_m ** 2]
        pts = near[rng.integers(0, len(near), points_per_frame)]
        bad = rng.random(points_per_frame) < nan_frac
        pts[bad] = np.nan
        out.append(pts.astype(F32))
    first = out[0][np.all(np.isfinite(out[0]), 1)].astype(np.float64)
    means = first[rng.integers(0, len(first), n_window)] + rng.normal(0.0, mean_sigma, (n_window, 3))
    return out, means.astype(F32)


# ----------------------------------------------------------------------------
# the five benchmark workloads
# ----------------------------------------------------------------------------

CONFIG_NAMES = {
    1: "plain fwd: 1k Gaussians, 128x96, 16x16 tiles",
    2: "fwd+bwd L1: 100k Gaussians, 640x512",
    3: "batched window: 500k surfel Gaussians on 50 planes, 8 keyframes 1280x1024",
    4: "pose gradient: 200k surfel Gaussians, 640x512, 32 perturbed poses",
    5: "uneven batch: 2M surfel Gaussians, 16 cameras 320x256..1920x1080",
}


def config1(seed=1) -> Scene:
    cam = Camera(100.0, 100.0, 64.0, 48.0, 128, 96, np.eye(3), np.zeros(3))
    return random_scene(1000, cam, seed, name="config1")


def config2(seed=2, n=100_000):
    """Returns (scene, target_scene): the target is a copy with means jittered by N(0, 0.02 m)."""
    cam = Camera(500.0, 500.0, 320.0, 256.0, 640, 512, np.eye(3), np.zeros(3))
    sc = random_scene(n, cam, seed, name="config2")
    return sc, jitter_means(sc, 0.02, seed + 100)


def config3(seed=3, n_planes=50, per_plane=10_000, n_cams=8, width=1280, height=1024, f=1000.0):
    """Returns (scene, target_scene); scene.cams holds the keyframes."""
    cams = trajectory_cameras(n_cams, width, height, f, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    ref = Camera(f, f, width / 2, height / 2, width, height, np.eye(3), np.zeros(3))
    centers = frustum_points(rng, ref, n_planes, 1.5, 5.0)
    sc = surface_scene(n_planes, per_plane, seed, centers, name="config3")
    sc.cams = cams
    tgt = jitter_means(sc, 0.02, seed + 100)
    tgt.cams = cams
    return sc, tgt


def config4(seed=4, n_planes=20, per_plane=10_000, n_poses=32, width=640, height=512, f=500.0,
            t_sigma=0.05, rot_sigma_deg=1.0):
    """Returns (scene, true_camera, perturbed_cameras, twists) with twists[k] = (dphi, dt)."""
    true_cam = Camera(f, f, width / 2, height / 2, width, height, np.eye(3), np.zeros(3))
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    centers = frustum_points(rng, true_cam, n_planes, 1.5, 5.0)
    sc = surface_scene(n_planes, per_plane, seed, centers, name="config4")
    prng = np.random.Generator(np.random.PCG64(seed + 2000))
    cams, tw = [], []
    for _ in range(n_poses):
        dphi = prng.normal(0.0, np.deg2rad(rot_sigma_deg), 3)
        dt = prng.normal(0.0, t_sigma, 3)
        cams.append(perturb_camera(true_cam, dphi, dt))
        tw.append(np.concatenate([dphi, dt]))
    sc.cams = cams
    return sc, true_cam, cams, np.array(tw)


def _count_in_view(cam: Camera, pts):
    pc = pts @ cam.R_cw.T.astype(np.float64) + cam.t_cw.astype(np.float64)
    z = pc[:, 2]
    ok = z > 0.2
    zs = np.where(ok, z, 1.0)
    u = cam.fx * pc[:, 0] / zs + cam.cx
    v = cam.fy * pc[:, 1] / zs + cam.cy
    return int(np.count_nonzero(ok & (u >= 0) & (u < cam.width) & (v >= 0) & (v < cam.height)))


def config5(seed=5, n_planes=200, per_plane=10_000, n_cams=16, vis_lo=50_000, vis_hi=600_000):
    """Returns (scene, target_scene) with 16 cameras of mixed resolution."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    # patch centres in a 24 x 6 x 24 m hall; cameras inside it
    centers = np.stack([rng.uniform(-12, 12, n_planes), rng.uniform(-3, 3, n_planes),
                        rng.uniform(-12, 12, n_planes)], 1)
    sc = surface_scene(n_planes, per_plane, seed, centers, name="config5")
    pts = sc.mean.astype(np.float64)
    sizes = [(320, 256), (1920, 1080)]
    while len(sizes) < n_cams:
        w = int(rng.integers(320, 1921)) // 8 * 8
        h = int(round(w * rng.uniform(0.5625, 0.8))) // 8 * 8
        sizes.append((w, max(256, min(h, 1080))))
    order = rng.permutation(n_cams)
    sizes = [sizes[i] for i in order]
    cams = []
    for (w, h) in sizes:
        f = 0.78125 * w
        for _ in range(10_000):
            center = np.array([rng.uniform(-10, 10), rng.uniform(-1, 1), rng.uniform(-10, 10)])
            yaw = rng.uniform(0, 2 * np.pi)
            pitch = rng.normal(0, 0.15)
            cam = look_camera(w, h, f, center, yaw, pitch, rng.normal(0, 0.05))
            if vis_lo <= _count_in_view(cam, pts) <= vis_hi:
                break
        else:
            raise RuntimeError("no camera pose found with the requested visible count")
        cams.append(cam)
    sc.cams = cams
    tgt = jitter_means(sc, 0.02, seed + 100)
    tgt.cams = cams
    return sc, tgt
