"""ctypes view of the C ABI in include/gslivo.h (libgslivo.so).

Only marshalling lives here: struct layouts mirroring the header, the loaded
library, and conversion of return codes into exceptions.  Loading fails with
an error when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgslivo.so")

GSL_OK = 0
GSL_EINVAL = -1
GSL_ENOTSUP = -2
GSL_ECAPACITY = -3
GSL_EHIP = -4
GSL_ESTATE = -5
GSL_D2H = 0
GSL_H2D = 1
GSL_LOSS_L1 = 1
GSL_LOSS_L2 = 2

_NAMES = {GSL_EINVAL: "EINVAL", GSL_ENOTSUP: "ENOTSUP", GSL_ECAPACITY: "ECAPACITY", GSL_EHIP: "EHIP",
          GSL_ESTATE: "ESTATE"}

EXPORTS = ["gsl_create", "gsl_destroy", "gsl_last_error", "gsl_default_opts", "gsl_layout", "gsl_workspace_size",
           "gsl_project", "gsl_bin_sort", "gsl_render_fwd", "gsl_render_bwd", "gsl_render_bwd_noalloc", "gsl_render_stats", "gsl_window_step",
           "gsl_window_tune", "gsl_window_variant", "gsl_graph_count", "gsl_profile", "gsl_profile_read",
           "gsl_pose_jacobian_workspace_size", "gsl_pose_jacobian", "gsl_imu_to_camera_twist",
           "gsl_ieskf_pose_update", "gsl_ieskf_visual_update", "gsl_adam_init", "gsl_adam_activate", "gsl_adam_step", "gsl_window_optimize",
           "gsl_voxel_keys", "gsl_window_workspace_size", "gsl_window_classify", "gsl_window_compact",
           "gsl_window_transfer",
           "gsl_color_init", "gsl_valu_probe", "gsl_window_render"]


class GslError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gslivo {_NAMES.get(code, code)}: {msg}")
        self.code = code


class Camera(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("R_cw", C.c_float * 9), ("t_cw", C.c_float * 3)]


class Opts(C.Structure):
    _fields_ = [("near_z", C.c_float), ("eps2d", C.c_float), ("alpha_min", C.c_float), ("alpha_max", C.c_float),
                ("T_min", C.c_float), ("bg", C.c_float * 3), ("guard", C.c_float), ("tile", C.c_int32),
                ("chunk", C.c_int32)]


class Gaussians(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p), ("opacity", C.c_void_p),
                ("color", C.c_void_p), ("N", C.c_int32), ("sh_degree", C.c_int32), ("sh", C.c_void_p)]


class Proj(C.Structure):
    _fields_ = [("splats", C.c_void_p), ("tiles_touched", C.c_void_p), ("binrecs", C.c_void_p),
                ("depth_keys", C.c_void_p)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_float * 5), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("lr_sh", C.c_float)]


class AdamState(C.Structure):
    _fields_ = [("raw", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p), ("d_step", C.c_void_p),
                ("N", C.c_int32), ("ld", C.c_int32), ("sh_degree", C.c_int32)]


class Bins(C.Structure):
    _fields_ = [("tile_ids", C.c_void_p), ("gauss_ids", C.c_void_p), ("ranges", C.c_void_p), ("d_K", C.c_void_p),
                ("d_status", C.c_void_p), ("capacity_K", C.c_int64)]


class Grads(C.Structure):
    _fields_ = [("g_mean", C.c_void_p), ("g_scale", C.c_void_p), ("g_quat", C.c_void_p), ("g_opacity", C.c_void_p),
                ("g_color", C.c_void_p), ("g_pose", C.c_void_p), ("g_sh", C.c_void_p)]


SPLAT_BYTES = 48

_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2501_08672_amd.build` "
                           "(hipcc, gfx950); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    pc, po, pg = C.POINTER(Camera), C.POINTER(Opts), C.POINTER(Gaussians)
    pp, pb, pgr = C.POINTER(Proj), C.POINTER(Bins), C.POINTER(Grads)
    L.gsl_last_error.restype = C.c_char_p
    L.gsl_last_error.argtypes = []
    L.gsl_create.argtypes = [C.POINTER(P), C.c_int]
    L.gsl_destroy.argtypes = [P]
    L.gsl_default_opts.argtypes = [po]
    L.gsl_default_opts.restype = None
    L.gsl_layout.argtypes = [pc, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.gsl_workspace_size.argtypes = [P, pc, C.c_int32, C.c_int32, po, C.c_int64, C.POINTER(C.c_size_t)]
    L.gsl_project.argtypes = [P, pg, pc, C.c_int32, po, pp, P, C.c_size_t, P]
    L.gsl_bin_sort.argtypes = [P, pc, C.c_int32, C.c_int32, po, pp, pb, P, C.c_size_t, P]
    L.gsl_render_fwd.argtypes = [P, pc, C.c_int32, C.c_int32, po, pp, pb, P, P, P, P, C.c_size_t, P]
    L.gsl_render_bwd.argtypes = [P, pg, pc, C.c_int32, po, pp, pb, P, P, P, C.c_int, pgr, P, C.c_size_t, P]
    L.gsl_render_bwd_noalloc.argtypes = [P, pg, pc, C.c_int32, po, pp, pb, P, P, P, C.c_int, pgr, P]
    L.gsl_render_stats.argtypes = [P, pc, C.c_int32, C.c_int32, po, pp, pb, P, P, C.c_size_t, P]
    L.gsl_window_variant.argtypes = [P, pc, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.gsl_graph_count.argtypes = [P, C.POINTER(C.c_int64)]
    L.gsl_valu_probe.argtypes = [P, C.c_int32, P, C.POINTER(C.c_double)]
    L.gsl_profile.argtypes = [P, C.c_int]
    L.gsl_profile_read.argtypes = [P, C.POINTER(C.c_float), C.c_int32]
    L.gsl_window_step.argtypes = [P, pg, pc, C.c_int32, po, P, C.c_int, pp, pb, P, P, pgr, P, C.c_size_t, C.c_int, P]
    L.gsl_window_render.argtypes = [P, pg, pc, C.c_int32, po, pp, pb, P, P, P, P, C.c_size_t, C.c_int, P]
    L.gsl_window_tune.argtypes = [P, pg, pc, C.c_int32, po, P, C.c_int, pp, pb, P, pgr, P, C.c_size_t,
                                  C.POINTER(C.c_float), C.c_int32, P]
    L.gsl_pose_jacobian_workspace_size.argtypes = [P, pc, C.c_int32, C.c_int32, po, C.c_int64,
                                                   C.POINTER(C.c_size_t)]
    L.gsl_pose_jacobian.argtypes = [P, pg, pc, C.c_int32, po, pp, pb, P, P, P, P, P, P, P, P, C.c_size_t, P]
    L.gsl_imu_to_camera_twist.argtypes = [P, P, P, P]
    L.gsl_ieskf_pose_update.argtypes = [P, P, P, P, P, P]
    L.gsl_ieskf_visual_update.argtypes = [P, P, P, C.c_double, P, P, P, P]
    pa, ps = C.POINTER(Adam), C.POINTER(AdamState)
    L.gsl_adam_init.argtypes = [P, pg, ps, P]
    L.gsl_adam_activate.argtypes = [P, ps, pg, P]
    L.gsl_adam_step.argtypes = [P, ps, pa, pgr, pg, P]
    L.gsl_window_optimize.argtypes = [P, ps, pa, pg, pc, C.c_int32, po, P, C.c_int, pp, pb, P, pgr, C.c_int32, P,
                                      C.c_size_t, C.c_int, P]
    L.gsl_color_init.argtypes = [P, P, C.c_int64, C.c_int32, pc, P, po, P, C.c_int64, P, P]
    L.gsl_voxel_keys.argtypes = [P, P, C.c_int32, C.c_int64, C.c_int64, C.c_float, P, P]
    L.gsl_window_workspace_size.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
    L.gsl_window_classify.argtypes = [P, P, C.c_int32, C.c_float, P, C.c_int32, P, P, P, C.c_size_t, P]
    L.gsl_window_transfer.argtypes = [P, C.c_int, P, P, C.c_int64, P, P, C.c_int64, C.c_int32, C.c_int32, P]
    L.gsl_window_compact.argtypes = [P, P, P, C.c_int32, C.c_int64, C.c_int32, C.c_int32, P, P, C.c_int32, P, P, P,
                                     C.c_size_t, P, P]
    for name in EXPORTS:
        if name not in ("gsl_last_error", "gsl_default_opts"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc: int):
    if rc != GSL_OK:
        raise GslError(rc, lib().gsl_last_error().decode())


def default_opts(tile: int = 16, **kw) -> Opts:
    o = Opts()
    lib().gsl_default_opts(C.byref(o))
    o.tile = tile
    for k, v in kw.items():
        if k == "bg":
            for j in range(3):
                o.bg[j] = float(v[j])
        else:
            setattr(o, k, v)
    return o


def camera_array(cams) -> "C.Array":
    """ctypes array of gsl_camera from objects with fx, fy, cx, cy, width,
    height, R_cw (3x3) and t_cw (3) attributes."""
    arr = (Camera * len(cams))()
    for k, c in enumerate(cams):
        a = arr[k]
        a.fx, a.fy, a.cx, a.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        a.width, a.height = int(c.width), int(c.height)
        R = [float(x) for x in np.asarray(c.R_cw, dtype=np.float32).reshape(9)]
        t = [float(x) for x in np.asarray(c.t_cw, dtype=np.float32).reshape(3)]
        for j in range(9):
            a.R_cw[j] = R[j]
        for j in range(3):
            a.t_cw[j] = t[j]
    return arr
