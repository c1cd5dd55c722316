"""Python access to the FP64 CPU oracle (``gsl_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this module; the product path never imports it.  It
imports nothing from the GPU package, and the GPU package imports nothing
from it; the two meet only through the seeded inputs of ``scenegen``.

Functions take a ``scenegen.Scene`` (float32 arrays, widened here to float64)
and ``scenegen.Camera`` objects and return float64 numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsl_oracle.c")
_LIB = os.path.join(_HERE, "libgsl_oracle.so")

AMB_VALUE = 1   # an alpha-threshold or cull decision: the pixel may differ by a whole contribution
AMB_GRAD = 2    # the alpha clamp switches at a contributor: its alpha gradient may differ
AMB_TCUT = 4    # a small-step cutoff decision: the pixel may differ by at most 2.01 T_min (max c + bg)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cam(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("R", C.c_double * 9), ("t", C.c_double * 3)]


class _Opts(C.Structure):
    _fields_ = [("near_z", C.c_double), ("eps2d", C.c_double), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("T_min", C.c_double), ("bg", C.c_double * 3),
                ("guard", C.c_double), ("amb_rel", C.c_double), ("amb_ignore", C.c_double)]


@dataclass
class Opts:
    """Rendering constants (the paper's alpha clamp and transmittance cutoff;
    the remaining values are this build's readings of what the paper leaves open)."""
    near_z: float = 0.2
    eps2d: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    bg: tuple = (0.0, 0.0, 0.0)
    guard: float = 0.15
    amb_rel: float = 4.0  # safety factor on the FP32 error bound of the ambiguity flags
    amb_ignore: float = 5e-5  # deviation budget (half the image tolerance) for alpha-threshold flips left unflagged

    def c(self) -> _Opts:
        o = _Opts()
        o.near_z, o.eps2d, o.alpha_min, o.alpha_max, o.T_min = (
            self.near_z, self.eps2d, self.alpha_min, self.alpha_max, self.T_min)
        for k in range(3):
            o.bg[k] = float(self.bg[k])
        o.guard, o.amb_rel, o.amb_ignore = self.guard, self.amb_rel, self.amb_ignore
        return o


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_project.argtypes = [C.c_int64, P, P, P, C.POINTER(_Cam), C.POINTER(_Opts), P, P, P, P, P]
        L.orc_render_fwd.argtypes = [C.c_int64, P, P, P, P, P, C.POINTER(_Cam), C.POINTER(_Opts),
                                     C.c_int64, P, P, P, P, P, P]
        L.orc_render_bwd.argtypes = [C.c_int64, P, P, P, P, P, C.POINTER(_Cam), C.POINTER(_Opts),
                                     C.c_int64, P, P, P, P, P, P, P, P, P]
        L.orc_pixel_trace.argtypes = [C.c_int64, P, P, P, P, P, C.POINTER(_Cam), C.POINTER(_Opts),
                                      C.c_int32, C.c_int32, C.c_int32, P, P, P]
        L.orc_pixel_trace.restype = C.c_int32
        L.orc_render_jvp.argtypes = [C.c_int64, P, P, P, P, P, P, C.POINTER(_Cam), C.POINTER(_Opts),
                                     C.c_int64, P, P, P]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _cam(cam) -> _Cam:
    c = _Cam()
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    R = np.asarray(cam.R_cw, np.float64).reshape(9)
    t = np.asarray(cam.t_cw, np.float64).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    return c


def _d(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _params(scene, cam=None):
    """Parameters as float64 arrays; with SH coefficients the colour is the
    one seen from `cam`."""
    colour = _d(scene.color) if getattr(scene, "sh", None) is None else _d(sh_colour(scene, cam))
    return (_d(scene.mean), _d(scene.scale), _d(scene.quat), _d(scene.opacity), colour)


# ---------------------------------------------------------------- view-dependent colour (spherical harmonics)

_Y00 = 0.5 / np.sqrt(np.pi)


def sh_basis(u, degree):
    """Real orthonormal spherical harmonics Y_lm of degrees l = 1..degree at
    the points u (..., 3) (unit vectors), each divided by Y_00 = 1/(2 sqrt(pi)),
    so that a colour is c(u) = k_0 + sum_k k_k B_k(u) and the degree-0
    coefficient k_0 is the colour itself (the map's SH coefficients, Sec. II-B).
    Order: l = 1..degree, m = -l..l.  Written as the usual Cartesian
    polynomials of the real basis (no Condon-Shortley sign):
      l = 1: c1 (y, z, x),                         c1 = sqrt(3 / (4 pi))
      l = 2: c2 xy, c2 yz, c20 (3z^2 - 1), c2 xz, c2/2 (x^2 - y^2),
             c2 = sqrt(15 / pi) / 2, c20 = sqrt(5 / pi) / 4
      l = 3: a y(3x^2 - y^2), b xyz, c y(5z^2 - 1), e (5z^3 - 3z),
             c x(5z^2 - 1), b/2 (x^2 - y^2) z, a x(x^2 - 3y^2),
             a = sqrt(35 / (2 pi)) / 4, b = sqrt(105 / pi) / 2,
             c = sqrt(21 / (2 pi)) / 4, e = sqrt(7 / pi) / 4.
    Returns (..., K), K = (degree + 1)^2 - 1."""
    u = np.asarray(u, np.float64)
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    out = []
    if degree >= 1:
        c1 = np.sqrt(3.0 / (4.0 * np.pi))
        out += [c1 * y, c1 * z, c1 * x]
    if degree >= 2:
        c2, c20 = np.sqrt(15.0 / np.pi) / 2.0, np.sqrt(5.0 / np.pi) / 4.0
        out += [c2 * x * y, c2 * y * z, c20 * (3.0 * z * z - 1.0), c2 * x * z, 0.5 * c2 * (x * x - y * y)]
    if degree >= 3:
        a, b = np.sqrt(35.0 / (2.0 * np.pi)) / 4.0, np.sqrt(105.0 / np.pi) / 2.0
        c, e = np.sqrt(21.0 / (2.0 * np.pi)) / 4.0, np.sqrt(7.0 / np.pi) / 4.0
        out += [a * y * (3.0 * x * x - y * y), b * x * y * z, c * y * (5.0 * z * z - 1.0),
                e * (5.0 * z ** 3 - 3.0 * z), c * x * (5.0 * z * z - 1.0), 0.5 * b * (x * x - y * y) * z,
                a * x * (x * x - 3.0 * y * y)]
    if not out:
        return np.zeros(u.shape[:-1] + (0,))
    return np.stack(out, -1) / _Y00


def sh_basis_grad(u, degree):
    """Partial derivatives of the polynomials of sh_basis with respect to
    (x, y, z): (..., K, 3)."""
    u = np.asarray(u, np.float64)
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    o, l = np.zeros_like(x), np.ones_like(x)
    rows = []
    if degree >= 1:
        c1 = np.sqrt(3.0 / (4.0 * np.pi))
        rows += [(o, c1 * l, o), (o, o, c1 * l), (c1 * l, o, o)]
    if degree >= 2:
        c2, c20 = np.sqrt(15.0 / np.pi) / 2.0, np.sqrt(5.0 / np.pi) / 4.0
        rows += [(c2 * y, c2 * x, o), (o, c2 * z, c2 * y), (o, o, 6.0 * c20 * z), (c2 * z, o, c2 * x),
                 (c2 * x, -c2 * y, o)]
    if degree >= 3:
        a, b = np.sqrt(35.0 / (2.0 * np.pi)) / 4.0, np.sqrt(105.0 / np.pi) / 2.0
        c, e = np.sqrt(21.0 / (2.0 * np.pi)) / 4.0, np.sqrt(7.0 / np.pi) / 4.0
        rows += [(6.0 * a * x * y, a * (3.0 * x * x - 3.0 * y * y), o),
                 (b * y * z, b * x * z, b * x * y),
                 (o, c * (5.0 * z * z - 1.0), 10.0 * c * y * z),
                 (o, o, e * (15.0 * z * z - 3.0)),
                 (c * (5.0 * z * z - 1.0), o, 10.0 * c * x * z),
                 (b * x * z, -b * y * z, 0.5 * b * (x * x - y * y)),
                 (a * (3.0 * x * x - 3.0 * y * y), -6.0 * a * x * y, o)]
    if not rows:
        return np.zeros(u.shape[:-1] + (0, 3))
    return np.stack([np.stack(r, -1) for r in rows], -2) / _Y00


def sh_colour_twist_tangent(scene, cam):
    """Derivative of each Gaussian's colour with respect to the left twist
    (dphi, dt) of T_CW: (N, 3, 6).  A rotation leaves the camera centre in
    place (zero); dt moves the view vector d = mu - o by R^T dt, so
    dc/ddt = dc/du (I - u u^T) / r R^T."""
    u, r = _view_dirs(scene, cam)
    sh = np.asarray(scene.sh, np.float64)
    dB = sh_basis_grad(u, scene.sh_degree)
    dc_du = np.einsum("nkc,nkj->ncj", sh, dB)
    proj = np.eye(3)[None] - u[:, :, None] * u[:, None, :]
    dc_dd = np.einsum("ncj,njl->ncl", dc_du, proj) / r[:, None, None]
    R = np.asarray(cam.R_cw, np.float64).reshape(3, 3)
    out = np.zeros((scene.n, 3, 6))
    out[:, :, 3:] = dc_dd @ R.T
    return out


def bilinear_colour(means, cam, image, near_z=0.2):
    """Initial colour of new Gaussians (Sec. II-B, eq. c(mu_I)): the mean is
    projected into the camera, mu_I = (fx x/z + cx, fy y/z + cy), and the
    colour is the bilinear interpolation of the image there: pixel (i, j) has
    its centre at (i + 1/2, j + 1/2); with s = mu_I - 1/2 clamped to the
    centres' range [0, W-1] x [0, H-1], the four surrounding pixels are
    weighted by the areas of the opposite sub-rectangles, c = sum_j c_j A_j.
    A mean with z <= near_z or outside [0, W) x [0, H) gets no colour.
    means (n, 3); image planar (3, H, W).  Returns colour (n, 3) (zero where
    invalid) and valid (n,) bool.  All in float64."""
    means = np.asarray(means, np.float64).reshape(-1, 3)
    img = np.asarray(image, np.float64)
    H, W = img.shape[1], img.shape[2]
    R = np.asarray(cam.R_cw, np.float64).reshape(3, 3)
    t = np.asarray(cam.t_cw, np.float64).reshape(3)
    out = np.zeros((len(means), 3))
    valid = np.zeros(len(means), bool)
    for n in range(len(means)):
        pc = R @ means[n] + t
        if not pc[2] > near_z:
            continue
        u = cam.fx * pc[0] / pc[2] + cam.cx
        v = cam.fy * pc[1] / pc[2] + cam.cy
        if not (0.0 <= u < W and 0.0 <= v < H):
            continue
        sx = min(max(u - 0.5, 0.0), W - 1.0)
        sy = min(max(v - 0.5, 0.0), H - 1.0)
        i0, j0 = min(int(np.floor(sx)), max(W - 2, 0)), min(int(np.floor(sy)), max(H - 2, 0))
        a, b = sx - i0, sy - j0
        i1, j1 = min(i0 + 1, W - 1), min(j0 + 1, H - 1)
        out[n] = ((1 - a) * (1 - b) * img[:, j0, i0] + a * (1 - b) * img[:, j0, i1]
                  + (1 - a) * b * img[:, j1, i0] + a * b * img[:, j1, i1])
        valid[n] = True
    return out, valid


def camera_centre(cam):
    """World position of the camera: o = -R_cw^T t_cw."""
    R = np.asarray(cam.R_cw, np.float64).reshape(3, 3)
    return -R.T @ np.asarray(cam.t_cw, np.float64).reshape(3)


def _view_dirs(scene, cam):
    d = np.asarray(scene.mean, np.float64) - camera_centre(cam)
    r = np.linalg.norm(d, axis=1)
    return d / r[:, None], r


def sh_colour(scene, cam):
    """Colour of every Gaussian seen from `cam`: c = k_0 + sum_k k_k B_k(u)
    with u the unit direction from the camera centre to the mean, in world
    coordinates.  No clamp (the degree-0 colour is used directly, as without
    SH).  (N, 3) float64."""
    col = np.asarray(scene.color, np.float64)
    if getattr(scene, "sh", None) is None:
        return col
    u, _ = _view_dirs(scene, cam)
    B = sh_basis(u, scene.sh_degree)
    return col + np.einsum("nk,nkc->nc", B, np.asarray(scene.sh, np.float64))


def sh_colour_vjp(scene, cam, g_c):
    """Adjoint of sh_colour for a cotangent g_c (N, 3): returns g_color (N,3),
    g_sh (N,K,3), g_mean (N,3) and g_dt (3,), the gradient with respect to the
    translation of the left twist of T_CW (the camera centre moves by
    -R_cw^T dt; a rotation of the twist leaves it in place)."""
    g_c = np.asarray(g_c, np.float64)
    u, r = _view_dirs(scene, cam)
    sh = np.asarray(scene.sh, np.float64)
    B = sh_basis(u, scene.sh_degree)
    dB = sh_basis_grad(u, scene.sh_degree)
    g_sh = B[:, :, None] * g_c[:, None, :]
    g_u = np.einsum("nc,nkc,nkj->nj", g_c, sh, dB)
    g_d = (g_u - u * np.sum(u * g_u, 1, keepdims=True)) / r[:, None]
    R = np.asarray(cam.R_cw, np.float64).reshape(3, 3)
    return g_c.copy(), g_sh, g_d, R @ g_d.sum(0)


def all_pixels(cam) -> np.ndarray:
    v, u = np.mgrid[0:cam.height, 0:cam.width]
    return np.ascontiguousarray(np.stack([u.ravel(), v.ravel()], 1).astype(np.int32))


def project(scene, cam, opts: Opts = Opts()):
    """Per-Gaussian projection into `cam`: p_cam (N,3), mean2d (N,2),
    cov2d (N,3: xx, xy, yy incl. dilation), conic (N,3: A, B, C), status (N,)."""
    N = scene.n
    m, s, q, _, _ = _params(scene, cam)
    out = {k: np.zeros((N, w)) for k, w in (("p_cam", 3), ("mean2d", 2), ("cov2d", 3), ("conic", 3))}
    out["status"] = np.zeros(N, np.int32)
    co, oo = _cam(cam), opts.c()
    lib().orc_project(N, _p(m), _p(s), _p(q), C.byref(co), C.byref(oo), _p(out["p_cam"]), _p(out["mean2d"]),
                      _p(out["cov2d"]), _p(out["conic"]), _p(out["status"]))
    return out


def render(scene, cam, opts: Opts = Opts(), pixels=None):
    """Composite the listed pixels ((P,2) int32 of (u, v); all pixels when None).

    Returns rgb (P,3), T (P,), n (P,) contributor counts, last (P,) index of the
    last contributor (-1 if none) and flags (P,) ambiguity bits."""
    pix = all_pixels(cam) if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
    P = pix.shape[0]
    m, s, q, o, c = _params(scene, cam)
    rgb = np.zeros((P, 3))
    T = np.zeros(P)
    n = np.zeros(P, np.int32)
    last = np.zeros(P, np.int64)
    flags = np.zeros(P, np.int32)
    co, oo = _cam(cam), opts.c()
    lib().orc_render_fwd(scene.n, _p(m), _p(s), _p(q), _p(o), _p(c), C.byref(co), C.byref(oo), P, _p(pix),
                         _p(rgb), _p(T), _p(n), _p(last), _p(flags))
    return {"rgb": rgb, "T": T, "n": n, "last": last, "flags": flags, "pixels": pix}


def render_image(scene, cam, opts: Opts = Opts()):
    """Full image as planar (3, H, W) plus T (H, W), n, last and flags (H, W)."""
    r = render(scene, cam, opts)
    H, W = cam.height, cam.width
    return {"image": r["rgb"].T.reshape(3, H, W), "T": r["T"].reshape(H, W), "n": r["n"].reshape(H, W),
            "last": r["last"].reshape(H, W), "flags": r["flags"].reshape(H, W)}


def render_bwd(scene, cams, vs, opts: Opts = Opts(), pixels=None, want_g2d=False):
    """Gradient of L = sum_c sum_p <v_c[p], I_c[p]>.

    `vs[c]` is (P_c, 3) for the pixel list `pixels[c]` (all pixels when None),
    or a planar (3, H, W) cotangent image.  Returns dict with mean (N,3),
    scale (N,3), quat (N,4), opacity (N,), color (N,3), pose (C,6) as
    (dphi, dt) of a left perturbation of each T_CW, and g2d (C,N,9) if asked."""
    N = scene.n
    has_sh = getattr(scene, "sh", None) is not None
    g = {"mean": np.zeros((N, 3)), "scale": np.zeros((N, 3)), "quat": np.zeros((N, 4)),
         "opacity": np.zeros(N), "color": np.zeros((N, 3)), "pose": np.zeros((len(cams), 6))}
    if has_sh:
        g["sh"] = np.zeros(scene.sh.shape)
    if want_g2d:
        g["g2d"] = np.zeros((len(cams), N, 9))
    oo = opts.c()
    for ci, cam in enumerate(cams):
        v = np.asarray(vs[ci], np.float64)
        if pixels is None or pixels[ci] is None:
            pix = all_pixels(cam)
            if v.ndim == 3:
                v = v.reshape(3, -1).T
        else:
            pix = np.ascontiguousarray(pixels[ci], dtype=np.int32).reshape(-1, 2)
        v = _d(v, (-1, 3))
        assert v.shape[0] == pix.shape[0]
        pose = np.zeros(6)
        g2 = np.zeros((N, 9)) if want_g2d else None
        co = _cam(cam)
        m, s, q, o, c = _params(scene, cam)
        gcol = np.zeros((N, 3)) if has_sh else g["color"]
        lib().orc_render_bwd(N, _p(m), _p(s), _p(q), _p(o), _p(c), C.byref(co), C.byref(oo), pix.shape[0],
                             _p(pix), _p(v), _p(g["mean"]), _p(g["scale"]), _p(g["quat"]), _p(g["opacity"]),
                             _p(gcol), _p(pose), _p(g2))
        if has_sh:  # chain the per-camera colour gradient through the SH colour
            gc0, gsh, gm, gdt = sh_colour_vjp(scene, cam, gcol)
            g["color"] += gc0
            g["sh"] += gsh
            g["mean"] += gm
            pose[3:] += gdt
        g["pose"][ci] = pose
        if want_g2d:
            g["g2d"][ci] = g2
    return g


def pixel_trace(scene, cam, u, v, opts: Opts = Opts(), cap=100000):
    m, s, q, o, c = _params(scene, cam)
    ids = np.zeros(cap, np.int64)
    al = np.zeros(cap)
    Ts = np.zeros(cap)
    co, oo = _cam(cam), opts.c()
    n = lib().orc_pixel_trace(scene.n, _p(m), _p(s), _p(q), _p(o), _p(c), C.byref(co), C.byref(oo),
                              int(u), int(v), cap, _p(ids), _p(al), _p(Ts))
    return ids[:n].copy(), al[:n].copy(), Ts[:n].copy()


# ---------------------------------------------------------------- pose Jacobians and the IESKF update

def render_jvp(scene, cam, opts: Opts = Opts(), pixels=None):
    """Per-pixel Jacobian of the rendered colour with respect to the camera
    twist xi = (dphi, dt) of the left perturbation T_CW <- Exp(xi) T_CW
    (contributor sets held fixed).  Returns rgb (P,3), jac (P,3,6), pixels."""
    pix = all_pixels(cam) if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
    P = pix.shape[0]
    m, s, q, o, c = _params(scene, cam)
    dcol = None if getattr(scene, "sh", None) is None else _d(sh_colour_twist_tangent(scene, cam))
    rgb = np.zeros((P, 3))
    jac = np.zeros((P, 3, 6))
    co, oo = _cam(cam), opts.c()
    lib().orc_render_jvp(scene.n, _p(m), _p(s), _p(q), _p(o), _p(c), _p(dcol), C.byref(co), C.byref(oo), P,
                         _p(pix), _p(rgb), _p(jac))
    return {"rgb": rgb, "jac": jac, "pixels": pix}


def normal_equations(jac, residual, weight=None):
    """H^T R^-1 H (6,6) and H^T R^-1 z (6,) of the stacked measurement model
    z_p + H_p xi (Appendix A, IESKF update): one row per pixel and channel,
    H_p = jac[p] (3,6), z_p = residual[p] (3,), R^-1 = diag(weight[p]) per
    pixel (1 when None).  Also returns z^T R^-1 z."""
    jac = np.asarray(jac, np.float64).reshape(-1, 3, 6)
    z = np.asarray(residual, np.float64).reshape(-1, 3)
    w = np.ones(len(z)) if weight is None else np.asarray(weight, np.float64).reshape(-1)
    H = jac.reshape(-1, 6)
    zz = z.reshape(-1)
    ww = np.repeat(w, 3)
    return H.T @ (ww[:, None] * H), H.T @ (ww * zz), float(zz @ (ww * zz))


def skew(v):
    v = np.asarray(v, np.float64)
    return np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])


def imu_to_camera_twist(R_CI, t_CI, R_CW):
    """A (6,6) with xi_cam = A xi_imu, to first order, from the perturbation
    model (Appendix A): (T(xi_c) T_CW)^-1 T_CI = T_WI [+] T(xi_i), where the
    IMU pose is perturbed as (R_WI Exp(dphi_i), t_WI + dt_i).  Rotation:
    dphi_c = -R_CI dphi_i.  Translation: R_WC (t_CI^ dphi_c - dt_c) = dt_i."""
    R_CI = np.asarray(R_CI, np.float64).reshape(3, 3)
    R_CW = np.asarray(R_CW, np.float64).reshape(3, 3)
    A = np.zeros((6, 6))
    A[:3, :3] = -R_CI
    A[3:, :3] = skew(t_CI) @ A[:3, :3]
    A[3:, 3:] = -R_CW
    return A


def ieskf_pose_update(HtRH, HtRz, P_prior, x_minus_prior=None):
    """One IESKF update of a pose state from the normal equations (Appendix A):
    K = (H^T R^-1 H + P^-1)^-1 H^T R^-1,
    delta = -K z - (I - K H) (x_hat [-] x_bar),  Sigma = (I - K H) P,
    with the Jacobian of [-] taken as the identity.  K z and K H are formed
    from H^T R^-1 z and H^T R^-1 H."""
    HtRH = np.asarray(HtRH, np.float64)
    HtRz = np.asarray(HtRz, np.float64)
    P = np.asarray(P_prior, np.float64)
    n = P.shape[0]
    Ainv = np.linalg.inv(HtRH + np.linalg.inv(P))
    KH = Ainv @ HtRH
    Kz = Ainv @ HtRz
    dx = np.zeros(n) if x_minus_prior is None else np.asarray(x_minus_prior, np.float64)
    delta = -Kz - (np.eye(n) - KH) @ dx
    return delta, (np.eye(n) - KH) @ P


def ieskf_visual_update(HtH_cam, Htz_cam, A, P_prior, x_minus_prior=None, noise_var=1.0):
    """The visual update of the IMU pose from one camera's photometric normal
    equations (Sec. II-D, Appendix A): the measurement Jacobian in the IMU
    twist is H_imu = H_cam A (A of imu_to_camera_twist) and the noise R =
    noise_var I, so H_imu^T R^-1 H_imu = A^T (H_cam^T H_cam) A / noise_var and
    H_imu^T R^-1 z = A^T (H_cam^T z) / noise_var enter ieskf_pose_update."""
    A = np.asarray(A, np.float64)
    HtRH = A.T @ np.asarray(HtH_cam, np.float64) @ A / noise_var
    HtRz = A.T @ np.asarray(Htz_cam, np.float64) / noise_var
    return ieskf_pose_update(HtRH, HtRz, P_prior, x_minus_prior)


# ---------------------------------------------------------------- Adam over the map parameters

# Raw (optimised) parameters, 14 rows per Gaussian: mean (3), log-scale (3),
# quaternion (4), opacity logit (1), colour (3).  The renderer takes the
# activated values: scale = exp(log-scale), opacity = sigmoid(logit); mean,
# quaternion and colour pass unchanged.
RAW_ROWS = {"mean": (0, 3), "scale": (3, 6), "quat": (6, 10), "opacity": (10, 11), "color": (11, 14)}


def activate(raw):
    """raw (14 + 3K, N) -> dict of activated parameters, each (k, N); the
    rows after the colour are SH coefficients, used as they are ("sh")."""
    raw = np.asarray(raw, np.float64)
    out = {"mean": raw[0:3], "scale": np.exp(raw[3:6]), "quat": raw[6:10],
           "opacity": 1.0 / (1.0 + np.exp(-raw[10:11])), "color": raw[11:14]}
    if raw.shape[0] > 14:
        out["sh"] = raw[14:]
    return out


def deactivate(act):
    """Inverse of `activate`: the raw rows (14 + 3K, N) of activated
    parameters (dict of (k, N) arrays as `activate` returns): log-scale =
    ln(scale), opacity logit = ln(o / (1 - o)); mean, quaternion, colour and
    SH rows as they are.  The starting point of the optimisation of the map
    parameters (Sec. II-B)."""
    rows = [act["mean"], np.log(act["scale"]), act["quat"],
            np.log(np.asarray(act["opacity"], np.float64) / (1.0 - np.asarray(act["opacity"], np.float64))),
            act["color"]]
    if "sh" in act:
        rows.append(act["sh"])
    n = np.asarray(act["mean"]).shape[-1]
    return np.concatenate([np.asarray(r, np.float64).reshape(-1, n) for r in rows], 0)


def raw_gradient(raw, g_act):
    """Chain rule from the activated parameters' gradients (dict of (k, N)) to
    the raw rows: d exp(u)/du = exp(u), d sigmoid(u)/du = s (1 - s)."""
    a = activate(raw)
    g = np.zeros_like(np.asarray(raw, np.float64))
    g[0:3] = g_act["mean"]
    g[3:6] = g_act["scale"] * a["scale"]
    g[6:10] = g_act["quat"]
    s = a["opacity"]
    g[10:11] = g_act["opacity"] * s * (1.0 - s)
    g[11:14] = g_act["color"]
    if g.shape[0] > 14:
        g[14:] = g_act["sh"]
    return g


def adam_step(raw, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (Kingma and Ba) at step number t >= 1 with a learning
    rate per row (lr: (14,) or scalar):
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    x <- x - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
    Returns (raw, m, v), new arrays."""
    raw, m, v, grad = (np.asarray(a, np.float64) for a in (raw, m, v, grad))
    lr = np.asarray(lr, np.float64).reshape(-1, 1) if np.ndim(lr) else float(lr)
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return raw - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- sliding-window maintenance

KEY_BITS = 21            # bits per axis of a packed voxel key
KEY_BIAS = 1 << 20       # axis index i is stored as i + 2^20, so i in [-2^20, 2^20)


def voxel_key(points, voxel_size):
    """Root-voxel hash key of each point (Sec. II-A, eq. HashKey): the integer
    voxel index floor(p / v_s) per axis, computed in fp64 (p widened from
    float32, v_s from float32).  The three indices are packed into one uint64
    as ((ix + 2^20) << 42) | ((iy + 2^20) << 21) | (iz + 2^20).  A point with
    an index outside [-2^20, 2^20) on any axis, or a non-finite coordinate,
    has no key.  Returns (keys uint64 [P], valid bool [P]); invalid keys are 0."""
    p = np.asarray(points, np.float32).astype(np.float64).reshape(-1, 3)
    vs = float(np.float32(voxel_size))
    keys = np.zeros(len(p), np.uint64)
    valid = np.zeros(len(p), bool)
    for j in range(len(p)):
        if not np.all(np.isfinite(p[j])):
            continue
        idx = [int(np.floor(p[j, a] / vs)) for a in range(3)]
        if any(i < -KEY_BIAS or i >= KEY_BIAS for i in idx):
            continue
        keys[j] = ((idx[0] + KEY_BIAS) << (2 * KEY_BITS)) | ((idx[1] + KEY_BIAS) << KEY_BITS) | (idx[2] + KEY_BIAS)
        valid[j] = True
    return keys, valid


def window_classify(win_keys, point_keys, point_valid):
    """Steps 1 and 3 of the incremental window update (Sec. II-C): the field
    of view is the set of keys of the current LiDAR frame's points.  A window
    Gaussian whose voxel key is not in it is DELETE; a key of the frame that no
    window Gaussian carries is ADD.  Returns (delete bool [n], add_keys uint64)
    with the ADD keys listed once each, in the order of their first point."""
    win_keys = [int(k) for k in np.asarray(win_keys)]
    fov = set(int(k) for k, ok in zip(np.asarray(point_keys), np.asarray(point_valid)) if ok)
    delete = np.array([k not in fov for k in win_keys], bool)
    in_window = set(win_keys)
    add, seen = [], set()
    for k, ok in zip(np.asarray(point_keys), np.asarray(point_valid)):
        k = int(k)
        if ok and k not in in_window and k not in seen:
            seen.add(k)
            add.append(k)
    return delete, np.array(add, np.uint64)


def window_maintain(keys, rows, fov_keys, add_keys, add_rows):
    """Incremental update of the Gaussian window (Sec. II-C, steps 1, 2, 4),
    written element by element.

    keys (n,) voxel keys of the window; rows (R, n) its parameters;
    fov_keys: the voxel keys of the current field of view.
    Step 1: a Gaussian whose key is not in fov_keys is DELETE; its key and
    parameters go to the evicted lists, in window order.
    Step 2: with D deletions, each DELETE slot before n - D is filled by the
    next kept Gaussian from [n - D, n), in order (swap with the rear); the
    window is then [0, n - D).
    Step 4: add_keys / add_rows are appended.
    Returns keys_out, rows_out, evicted_keys, evicted_rows."""
    keys = np.asarray(keys)
    rows = np.asarray(rows)
    fov = set(int(k) for k in np.asarray(fov_keys))
    n = len(keys)
    delete = [int(k) not in fov for k in keys]
    D = sum(delete)
    ev = [i for i in range(n) if delete[i]]
    holes = [i for i in range(n - D) if delete[i]]
    rear = [i for i in range(n - D, n) if not delete[i]]
    assert len(holes) == len(rear)
    out_keys = keys[: n - D].copy()
    out_rows = rows[:, : n - D].copy()
    for h, r in zip(holes, rear):
        out_keys[h] = keys[r]
        out_rows[:, h] = rows[:, r]
    out_keys = np.concatenate([out_keys, np.asarray(add_keys, keys.dtype)])
    out_rows = np.concatenate([out_rows, np.asarray(add_rows, rows.dtype).reshape(rows.shape[0], -1)], 1)
    return out_keys, out_rows, keys[ev], rows[:, ev]
