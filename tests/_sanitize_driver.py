"""Child process of tests/test_sanitizers.py: exercises either the host side
of the C ABI library or the oracle library at a given path and prints what
it computed as one JSON line, so that a build under AddressSanitizer and
UndefinedBehaviorSanitizer can be run (with its runtime preloaded) and its
results compared with the plain build's.

    python _sanitize_driver.py abi <libgslivo.so>
    python _sanitize_driver.py oracle <libgsl_oracle.so>

Only host code runs: the ABI calls are the host helpers, the size queries
and the argument checks that fail before any launch (no GPU is needed)."""
import ctypes as C
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _d(a):
    return np.ascontiguousarray(a, np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def run_abi(path):
    from paper_2501_08672_amd import _abi as A
    A.LIB_PATH = path
    L = A.lib()
    import scenegen as S
    from scipy.spatial.transform import Rotation
    out = {}
    o = A.default_opts(16)
    out["opts"] = [o.near_z, o.eps2d, o.alpha_min, o.alpha_max, o.T_min, o.guard, o.tile]
    # layouts and workspace sizes of the workloads, at every tile size
    sc3, _ = S.config3()
    sc5, _ = S.config5()
    for name, cams, N in (("c1", S.config1().cams, 1000), ("c3", sc3.cams, 500_000), ("c5", sc5.cams, 2_000_000)):
        arr = A.camera_array(cams)
        for tile in (8, 16, 32):
            T, P, nb, nj = C.c_int64(), C.c_int64(), C.c_size_t(), C.c_size_t()
            ot = A.default_opts(tile)
            rc = [L.gsl_layout(arr, len(cams), tile, C.byref(T), C.byref(P)),
                  L.gsl_workspace_size(None, arr, len(cams), N, C.byref(ot), 10_000_000, C.byref(nb)),
                  L.gsl_pose_jacobian_workspace_size(None, arr, len(cams), N, C.byref(ot), 10_000_000, C.byref(nj))]
            out[f"layout_{name}_{tile}"] = rc + [T.value, P.value, nb.value, nj.value]
    # rejected shapes: the message of each failure is formatted on the host
    bad = A.camera_array(S.config1().cams)
    bad[0].width = 0
    T, P = C.c_int64(), C.c_int64()
    out["bad_layout"] = [L.gsl_layout(bad, 1, 16, C.byref(T), C.byref(P)), L.gsl_last_error().decode()]
    out["bad_tile"] = [L.gsl_layout(A.camera_array(S.config1().cams), 1, 12, C.byref(T), C.byref(P)),
                       L.gsl_last_error().decode()]
    for n, p in ((1000, 2000), (500_000, 100_000), (0, 0), (-1, 5)):
        b = C.c_size_t()
        out[f"win_ws_{n}_{p}"] = [L.gsl_window_workspace_size(n, p, C.byref(b)), b.value]
    # host helpers of the visual update
    rng = np.random.default_rng(3)
    R_CI = _d(Rotation.from_rotvec(rng.normal(size=3)).as_matrix())
    t_CI = _d(rng.normal(0, 0.3, 3))
    R_CW = _d(Rotation.from_rotvec(rng.normal(size=3)).as_matrix())
    Am = np.zeros(36)
    out["twist_rc"] = L.gsl_imu_to_camera_twist(_ptr(R_CI), _ptr(t_CI), _ptr(R_CW), _ptr(Am))
    out["twist"] = Am.tolist()
    H = rng.normal(size=(60, 6))
    z = rng.normal(size=60)
    Lm = rng.normal(size=(6, 6))
    Pm = _d(Lm @ Lm.T + 0.1 * np.eye(6))
    HtH, Htz, dx = _d(H.T @ H), _d(H.T @ z), _d(rng.normal(0, 0.05, 6))
    delta, Pn = np.zeros(6), np.zeros(36)
    out["upd_rc"] = L.gsl_ieskf_pose_update(_ptr(HtH), _ptr(Htz), _ptr(Pm), _ptr(dx), _ptr(delta), _ptr(Pn))
    out["upd"] = delta.tolist() + Pn.tolist()
    out["vis_rc"] = L.gsl_ieskf_visual_update(_ptr(HtH), _ptr(Htz), _ptr(Am), 0.25, _ptr(Pm), None, _ptr(delta),
                                              _ptr(Pn))
    out["vis"] = delta.tolist() + Pn.tolist()
    out["vis_bad"] = L.gsl_ieskf_visual_update(_ptr(HtH), _ptr(Htz), _ptr(Am), -1.0, _ptr(Pm), None, _ptr(delta),
                                               _ptr(Pn))
    sing = np.zeros(36)
    out["upd_singular"] = [L.gsl_ieskf_pose_update(_ptr(HtH), _ptr(Htz), _ptr(sing), None, _ptr(delta), _ptr(Pn)),
                           L.gsl_last_error().decode()]
    # every device entry point rejects NULL arguments on the host
    nulls = {"gsl_project": 9, "gsl_bin_sort": 10, "gsl_render_fwd": 13, "gsl_render_bwd": 15,
             "gsl_render_bwd_noalloc": 13, "gsl_render_stats": 11, "gsl_window_step": 16, "gsl_window_tune": 16,
             "gsl_pose_jacobian": 17, "gsl_adam_init": 4, "gsl_adam_activate": 4, "gsl_adam_step": 6,
             "gsl_window_optimize": 18, "gsl_voxel_keys": 8, "gsl_window_classify": 11, "gsl_window_compact": 16,
             "gsl_color_init": 11, "gsl_window_variant": 7, "gsl_graph_count": 2,
             "gsl_window_transfer": 11, "gsl_valu_probe": 4,
             "gsl_window_render": 14}
    for name, nargs in nulls.items():
        fn = getattr(L, name)
        args = [None if t is C.c_void_p or issubclass(t, C._Pointer) else t(0) for t in fn.argtypes]
        assert len(args) == nargs, name
        out[f"null_{name}"] = [fn(*args), L.gsl_last_error().decode()]
    # context creation: fails cleanly without a GPU
    ctx = C.c_void_p()
    rc = L.gsl_create(C.byref(ctx), 0)
    out["create_rc_ok_or_ehip"] = rc in (A.GSL_OK, A.GSL_EHIP, A.GSL_EINVAL)
    if rc == A.GSL_OK:
        L.gsl_destroy(ctx)
    out["create_bad_device"] = L.gsl_create(C.byref(ctx), -1)
    return out


def run_oracle(path):
    from oracle import oracle as O
    O._LIB = path
    import scenegen as S
    out = {}
    sc = S.config1()
    cam = sc.cams[0]
    r = O.render_image(sc, cam, O.Opts(bg=(0.1, 0.2, 0.3)))
    out["image_sum"] = float(r["image"].sum())
    out["image_sq"] = float((r["image"] ** 2).sum())
    out["flags"] = int(r["flags"].sum())
    p = O.project(sc, cam)
    out["proj"] = [float(np.nansum(p[k])) for k in ("p_cam", "mean2d", "cov2d", "conic")] + [int(p["status"].sum())]
    rng = np.random.default_rng(4)
    v = rng.normal(size=(3, cam.height, cam.width))
    g = O.render_bwd(sc, [cam], [v], O.Opts(bg=(0.1, 0.2, 0.3)))
    out["grads"] = {k: float(np.abs(a).sum()) for k, a in g.items()}
    shs = S.with_sh(sc, 3, 5)
    pix = np.stack([rng.integers(0, cam.width, 200), rng.integers(0, cam.height, 200)], 1).astype(np.int32)
    j = O.render_jvp(shs, cam, pixels=pix)
    out["jvp"] = [float(np.abs(j["jac"]).sum()), float(j["rgb"].sum())]
    ids, al, Ts = O.pixel_trace(sc, cam, 64, 48)
    out["trace"] = [int(ids.size), float(al.sum()), float(Ts.sum())]
    return out


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    res = run_abi(path) if mode == "abi" else run_oracle(path)
    print("RESULT " + json.dumps(res, sort_keys=True))
