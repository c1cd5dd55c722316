"""PyTorch-facing binding of the C ABI (argument marshalling only).

Tensors provide device memory and the current HIP stream; every step of the
path runs in libgslivo's kernels.  Names follow the ABI: project, bin_sort,
render_fwd, render_bwd, window_step, window_tune.

Layouts (all CUDA/HIP tensors, contiguous):
  Gaussian parameters, SoA: mean (3, N), scale (3, N), quat (4, N) as
  (w, x, y, z), opacity (N,), color (3, N); float32.
  Images of a camera set are packed: camera c's planar (3, H, W) block starts
  at float 3 * P_c with P_c the pixel count of the cameras before it
  (CameraSet.unpack / CameraSet.pack convert).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import _abi as A

LOSS = {"l1": A.GSL_LOSS_L1, "l2": A.GSL_LOSS_L2}


def _p(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def opts(tile: int = 16, **kw) -> A.Opts:
    """Default rendering constants (alpha clamp 0.99, cutoff 1e-4, skip 1/255,
    near 0.2 m, dilation 0.3 px^2, guard band 0.15, background 0)."""
    return A.default_opts(tile, **kw)


def _opts_copy(o: A.Opts, **kw) -> A.Opts:
    n = A.Opts()
    C.memmove(C.byref(n), C.byref(o), C.sizeof(A.Opts))
    for k, v in kw.items():
        setattr(n, k, v)
    return n


TUNE_TILES = (8, 16, 32)
TUNE_CHUNKS = (64, 128, 256)
TUNE_VARIANTS = 5
TUNE_TIMES = len(TUNE_TILES) * len(TUNE_CHUNKS) * TUNE_VARIANTS


class Context:
    """A gsl_ctx bound to one device, plus a growable scratch workspace."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the gslivo path runs only on the GPU")
        torch.cuda.set_device(device)
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        A.check(A.lib().gsl_create(C.byref(h), int(device)))
        self.h = h
        self._ws = None
        self.capacity = {}

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def close(self):
        if self.h:
            A.lib().gsl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def graph_count(ctx: "Context") -> int:
    """HIP graphs the context holds (gsl_graph_count)."""
    n = C.c_int64()
    A.check(A.lib().gsl_graph_count(ctx.h, C.byref(n)))
    return int(n.value)


VALU_PROBE_MODES = {"fma": 0, "mul_exp2": 1, "umin_add": 2, "add": 3, "mul": 4}


def valu_probe(ctx: "Context", mode: str) -> float:
    """Wave64 VALU instructions the chip issues per CU per 2.4-GHz cycle for
    one instruction kind (gsl_valu_probe; a measurement aid for the
    compositing kernels' roofline): "fma", "mul_exp2" or "umin_add"."""
    import torch
    sink = torch.zeros(1, dtype=torch.float32, device=ctx.device)
    r = C.c_double()
    A.check(A.lib().gsl_valu_probe(ctx.h, VALU_PROBE_MODES[mode], C.c_void_p(sink.data_ptr()), C.byref(r)))
    return float(r.value)


class CameraSet:
    """Host description of the C cameras of a window."""

    def __init__(self, cams):
        self.cams = list(cams)
        self.C = len(self.cams)
        self.arr = A.camera_array(self.cams)
        self.sizes = [(int(c.height), int(c.width)) for c in self.cams]
        self.pix_offsets = np.concatenate([[0], np.cumsum([h * w for h, w in self.sizes])]).astype(np.int64)
        self.P_total = int(self.pix_offsets[-1])

    def tiles(self, tile: int) -> int:
        T = C.c_int64()
        P = C.c_int64()
        A.check(A.lib().gsl_layout(self.arr, self.C, int(tile), C.byref(T), C.byref(P)))
        return int(T.value)

    def unpack(self, packed: torch.Tensor, channels: int = 3) -> List[torch.Tensor]:
        out = []
        for c, (h, w) in enumerate(self.sizes):
            o = int(self.pix_offsets[c]) * channels
            out.append(packed[o:o + channels * h * w].view(channels, h, w) if channels > 1
                       else packed[o:o + h * w].view(h, w))
        return out

    def pack(self, images, channels: int = 3) -> torch.Tensor:
        return torch.cat([im.reshape(-1) for im in images]).contiguous()


def sh_count(degree: int) -> int:
    """Higher-order SH coefficients per channel: (degree + 1)^2 - 1."""
    return (degree + 1) ** 2 - 1


def sh_degree_of(rows: int) -> int:
    """SH degree of 3K coefficient rows."""
    for d in range(4):
        if 3 * sh_count(d) == rows:
            return d
    raise ValueError(f"{rows} SH rows is not 3 ((D + 1)^2 - 1) for D in 0..3")


@dataclass
class Gaussians:
    """The window's Gaussians, component-major (gsl_gaussians); `sh` holds the
    higher-order SH coefficients as (3K, N) rows, row k * 3 + ch, or None."""
    mean: torch.Tensor
    scale: torch.Tensor
    quat: torch.Tensor
    opacity: torch.Tensor
    color: torch.Tensor
    sh: Optional[torch.Tensor] = None

    @property
    def N(self) -> int:
        return int(self.opacity.shape[0])

    @property
    def sh_degree(self) -> int:
        return 0 if self.sh is None else sh_degree_of(int(self.sh.shape[0]))

    @staticmethod
    def from_scene(scene, device="cuda") -> "Gaussians":
        def soa(a):
            return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32).T)).to(device)
        sh = None
        if getattr(scene, "sh", None) is not None:
            a = np.asarray(scene.sh, np.float32)  # (N, K, 3) -> rows k * 3 + ch
            sh = torch.from_numpy(np.ascontiguousarray(a.transpose(1, 2, 0).reshape(-1, a.shape[0]))).to(device)
        return Gaussians(soa(scene.mean), soa(scene.scale), soa(scene.quat),
                         torch.from_numpy(np.ascontiguousarray(scene.opacity, np.float32)).to(device),
                         soa(scene.color), sh)

    def tensors(self):
        return [t for t in (self.mean, self.scale, self.quat, self.opacity, self.color, self.sh) if t is not None]

    def struct(self) -> A.Gaussians:
        for t in self.tensors():
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("Gaussian parameters must be contiguous float32 device tensors")
        g = A.Gaussians()
        g.mean, g.scale, g.quat = self.mean.data_ptr(), self.scale.data_ptr(), self.quat.data_ptr()
        g.opacity, g.color = self.opacity.data_ptr(), self.color.data_ptr()
        g.N = self.N
        g.sh_degree = self.sh_degree
        g.sh = self.sh.data_ptr() if self.sh is not None else None
        return g

    def zeros_like(self) -> "Gaussians":
        return Gaussians(*(torch.zeros_like(t) for t in (self.mean, self.scale, self.quat, self.opacity, self.color)),
                         None if self.sh is None else torch.zeros_like(self.sh))


class Proj:
    """gsl_project output: splats (C, N, 48 B), tiles_touched (C, N), the
    binning records (C, N, 32 B; torch allocations are 256-byte aligned) and
    the depth-sort keys (C, N)."""

    def __init__(self, C_: int, N: int, device):
        self.splats = torch.empty((C_, N, A.SPLAT_BYTES), dtype=torch.uint8, device=device)
        self.tiles_touched = torch.empty((C_, N), dtype=torch.int32, device=device)
        self.binrecs = torch.empty((C_, N, 32), dtype=torch.uint8, device=device)
        self.depth_keys = torch.empty((C_, N), dtype=torch.int32, device=device)

    def struct(self) -> A.Proj:
        p = A.Proj()
        p.splats, p.tiles_touched = self.splats.data_ptr(), self.tiles_touched.data_ptr()
        p.binrecs, p.depth_keys = self.binrecs.data_ptr(), self.depth_keys.data_ptr()
        return p

    def fields(self):
        """Host copy of the splats as named numpy arrays (for tests)."""
        raw = self.splats.cpu().numpy()
        f = raw.view(np.float32).reshape(raw.shape[0], raw.shape[1], 12)
        b = raw.view(np.int16).reshape(raw.shape[0], raw.shape[1], 24)
        names = ["mx", "my", "l11", "l12", "l22", "opacity", "r", "g", "b", "depth"]
        out = {n: f[..., k].copy() for k, n in enumerate(names)}
        out["bbox"] = b[..., 20:24].copy()
        out["tiles_touched"] = self.tiles_touched.cpu().numpy()
        return out


class Bins:
    def __init__(self, capacity: int, T_total: int, device):
        self.capacity = int(capacity)
        self.tile_ids = torch.empty(max(1, self.capacity), dtype=torch.int32, device=device)
        self.gauss_ids = torch.empty(max(1, self.capacity), dtype=torch.int32, device=device)
        self.ranges = torch.empty((max(1, T_total), 2), dtype=torch.int32, device=device)
        self.d_K = torch.zeros(1, dtype=torch.int64, device=device)
        self.d_status = torch.zeros(1, dtype=torch.int32, device=device)
        self.T_total = T_total

    def struct(self) -> A.Bins:
        b = A.Bins()
        b.tile_ids, b.gauss_ids, b.ranges = self.tile_ids.data_ptr(), self.gauss_ids.data_ptr(), self.ranges.data_ptr()
        b.d_K, b.d_status = self.d_K.data_ptr(), self.d_status.data_ptr()
        b.capacity_K = self.capacity
        return b

    @property
    def K(self) -> int:
        return int(self.d_K.item())


class Grads:
    def __init__(self, N: int, C_: int, device, sh_degree: int = 0):
        self.mean = torch.empty((3, N), dtype=torch.float32, device=device)
        self.scale = torch.empty((3, N), dtype=torch.float32, device=device)
        self.quat = torch.empty((4, N), dtype=torch.float32, device=device)
        self.opacity = torch.empty((N,), dtype=torch.float32, device=device)
        self.color = torch.empty((3, N), dtype=torch.float32, device=device)
        self.pose = torch.empty((C_, 6), dtype=torch.float64, device=device)
        self.sh = (torch.empty((3 * sh_count(sh_degree), N), dtype=torch.float32, device=device)
                   if sh_degree > 0 else None)

    def struct(self) -> A.Grads:
        g = A.Grads()
        g.g_mean, g.g_scale, g.g_quat = self.mean.data_ptr(), self.scale.data_ptr(), self.quat.data_ptr()
        g.g_opacity, g.g_color, g.g_pose = self.opacity.data_ptr(), self.color.data_ptr(), self.pose.data_ptr()
        g.g_sh = self.sh.data_ptr() if self.sh is not None else None
        return g


def workspace_size(ctx: Context, cams: CameraSet, N: int, o: A.Opts, capacity: int) -> int:
    n = C.c_size_t()
    A.check(A.lib().gsl_workspace_size(ctx.h, cams.arr, cams.C, int(N), C.byref(o), int(capacity), C.byref(n)))
    return int(n.value)


# ---------------------------------------------------------------- the steps

def project(ctx: Context, g: Gaussians, cams: CameraSet, o: A.Opts, out: Optional[Proj] = None) -> Proj:
    out = out or Proj(cams.C, g.N, ctx.device)
    nb = workspace_size(ctx, cams, g.N, o, 0)
    ws = ctx.workspace(nb)
    gs, ps = g.struct(), out.struct()
    A.check(A.lib().gsl_project(ctx.h, C.byref(gs), cams.arr, cams.C, C.byref(o), C.byref(ps), _p(ws),
                                ws.numel(), _stream()))
    return out


def bin_sort(ctx: Context, cams: CameraSet, N: int, o: A.Opts, proj: Proj, capacity: Optional[int] = None,
             bins: Optional[Bins] = None, grow: bool = True) -> Bins:
    """Eager binning.  With grow=True the call synchronises to read K and
    repeats with a larger capacity when K exceeds it."""
    T_total = cams.tiles(o.tile)
    key = (cams.C, N, int(o.tile), tuple(cams.sizes))
    cap = capacity if capacity is not None else ctx.capacity.get(key, max(1 << 16, 4 * cams.C * N))
    for _ in range(3):
        if bins is None or bins.capacity < cap or bins.T_total != T_total:
            bins = Bins(cap, T_total, ctx.device)
        nb = workspace_size(ctx, cams, N, o, bins.capacity)
        ws = ctx.workspace(nb)
        ps, bs = proj.struct(), bins.struct()
        A.check(A.lib().gsl_bin_sort(ctx.h, cams.arr, cams.C, int(N), C.byref(o), C.byref(ps), C.byref(bs),
                                     _p(ws), ws.numel(), _stream()))
        if not grow:
            return bins
        status = int(bins.d_status.item())
        if status == A.GSL_OK:
            return bins
        cap = int(bins.K * 1.25) + 1024
        ctx.capacity[key] = cap
        bins = None
    raise A.GslError(A.GSL_ECAPACITY, "instance capacity could not be satisfied")


def render_fwd(ctx: Context, cams: CameraSet, N: int, o: A.Opts, proj: Proj, bins: Bins):
    """Returns (packed image (3 P_total,), T_final (P_total,), n_walk (P_total,) int32)."""
    image = torch.empty(3 * cams.P_total, dtype=torch.float32, device=ctx.device)
    T_final = torch.empty(cams.P_total, dtype=torch.float32, device=ctx.device)
    n_walk = torch.empty(cams.P_total, dtype=torch.int32, device=ctx.device)
    nb = workspace_size(ctx, cams, N, o, bins.capacity)
    ws = ctx.workspace(nb)
    ps, bs = proj.struct(), bins.struct()
    A.check(A.lib().gsl_render_fwd(ctx.h, cams.arr, cams.C, int(N), C.byref(o), C.byref(ps), C.byref(bs),
                                   _p(image), _p(T_final), _p(n_walk), _p(ws), ws.numel(), _stream()))
    return image, T_final, n_walk


def render_bwd(ctx: Context, g: Gaussians, cams: CameraSet, o: A.Opts, proj: Proj, bins: Bins, T_final, n_walk,
               dL_dimage: torch.Tensor, accumulate: bool = False, out: Optional[Grads] = None) -> Grads:
    out = out or Grads(g.N, cams.C, ctx.device, g.sh_degree)
    nb = workspace_size(ctx, cams, g.N, o, bins.capacity)
    ws = ctx.workspace(nb)
    gs, ps, bs, gr = g.struct(), proj.struct(), bins.struct(), out.struct()
    dl = dL_dimage.contiguous()
    A.check(A.lib().gsl_render_bwd(ctx.h, C.byref(gs), cams.arr, cams.C, C.byref(o), C.byref(ps), C.byref(bs),
                                   _p(T_final), _p(n_walk), _p(dl), int(bool(accumulate)), C.byref(gr), _p(ws),
                                   ws.numel(), _stream()))
    return out


def render_bwd_noalloc(ctx: Context, g: Gaussians, cams: CameraSet, o: A.Opts, proj: Proj, bins: Bins, T_final,
                       n_walk, dL_dimage: torch.Tensor, accumulate: bool = False, out: Grads = None) -> Grads:
    """gsl_render_bwd_noalloc: the backward pass on the library's static
    scratch array (no workspace; the call allocates nothing when `out` is
    given)."""
    out = out or Grads(g.N, cams.C, ctx.device, g.sh_degree)
    gs, ps, bs, gr = g.struct(), proj.struct(), bins.struct(), out.struct()
    dl = dL_dimage.contiguous()
    A.check(A.lib().gsl_render_bwd_noalloc(ctx.h, C.byref(gs), cams.arr, cams.C, C.byref(o), C.byref(ps),
                                           C.byref(bs), _p(T_final), _p(n_walk), _p(dl), int(bool(accumulate)),
                                           C.byref(gr), _stream()))
    return out


def render_stats(ctx: Context, cams: CameraSet, N: int, o: A.Opts, proj: Proj, bins: Bins):
    """(forward pairs evaluated, contributing pairs, backward pairs evaluated)."""
    counts = torch.zeros(3, dtype=torch.int64, device=ctx.device)
    nb = workspace_size(ctx, cams, N, o, bins.capacity)
    ws = ctx.workspace(nb)
    ps, bs = proj.struct(), bins.struct()
    A.check(A.lib().gsl_render_stats(ctx.h, cams.arr, cams.C, int(N), C.byref(o), C.byref(ps), C.byref(bs),
                                     _p(counts), _p(ws), ws.numel(), _stream()))
    return tuple(int(x) for x in counts.cpu().tolist())


# ---------------------------------------------------------------- Adam over the map parameters

class AdamState:
    """gsl_adam_state: raw parameters (14 + 3K, ld) — mean 3, log-scale 3,
    quaternion 4, opacity logit 1, colour 3, SH 3K — their Adam moments and the
    device step counter.  The first n columns are live (n = ld unless given),
    so a window kept at a fixed capacity can hand in views of its block."""

    def __init__(self, raw: torch.Tensor, m: Optional[torch.Tensor] = None, v: Optional[torch.Tensor] = None,
                 d_step: Optional[torch.Tensor] = None, n: Optional[int] = None):
        if raw.dtype != torch.float32 or raw.dim() != 2 or raw.shape[0] < 14:
            raise ValueError("raw parameters must be a float32 (14 + 3K, ld) tensor")
        self.sh_degree = sh_degree_of(int(raw.shape[0]) - 14)
        self.raw = raw if raw.stride(1) == 1 else raw.contiguous()
        self.m = torch.zeros_like(self.raw) if m is None else m
        self.v = torch.zeros_like(self.raw) if v is None else v
        for t in (self.m, self.v):
            if t.shape != self.raw.shape or t.stride() != self.raw.stride() or t.dtype != torch.float32:
                raise ValueError("moments must have the raw parameters' shape and strides")
        self.d_step = torch.zeros(1, dtype=torch.int32, device=raw.device) if d_step is None else d_step
        self.n = int(self.raw.shape[1]) if n is None else int(n)
        if not 0 <= self.n <= self.raw.shape[1]:
            raise ValueError("live count exceeds the row length")

    @property
    def N(self) -> int:
        return self.n

    @staticmethod
    def from_gaussians(ctx: "Context", g: "Gaussians") -> "AdamState":
        """Raw parameters of activated ones, zero moments and step count
        (gsl_adam_init)."""
        rows = 14 + 3 * (0 if g.sh is None else int(g.sh.shape[0]) // 3)
        st = AdamState(torch.empty(rows, g.N, dtype=torch.float32, device=ctx.device))
        gs, ss = g.struct(), st.struct()
        A.check(A.lib().gsl_adam_init(ctx.h, C.byref(gs), C.byref(ss), _stream()))
        return st

    def struct(self) -> A.AdamState:
        st = A.AdamState()
        st.raw, st.m, st.v, st.d_step = (t.data_ptr() for t in (self.raw, self.m, self.v, self.d_step))
        st.N = self.n
        st.ld = int(self.raw.stride(0))
        st.sh_degree = self.sh_degree
        return st


def adam_hparams(lr=(1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3), beta1=0.9, beta2=0.999, eps=1e-15,
                 lr_sh=1.25e-4) -> A.Adam:
    """Learning rates per group: mean, log-scale, quaternion, opacity logit,
    colour; lr_sh for the higher-order SH coefficients."""
    hp = A.Adam()
    for k in range(5):
        hp.lr[k] = float(lr[k])
    hp.beta1, hp.beta2, hp.eps = float(beta1), float(beta2), float(eps)
    hp.lr_sh = float(lr_sh)
    return hp


def adam_activate(ctx: Context, st: AdamState, g: "Gaussians"):
    """g <- activation(st.raw)."""
    ss, gs = st.struct(), g.struct()
    A.check(A.lib().gsl_adam_activate(ctx.h, C.byref(ss), C.byref(gs), _stream()))


def adam_step(ctx: Context, st: AdamState, hp: A.Adam, grads: "Grads", g: "Gaussians"):
    """One Adam step from the gradients of the activated parameters; writes g."""
    ss, gs, gr = st.struct(), g.struct(), grads.struct()
    A.check(A.lib().gsl_adam_step(ctx.h, C.byref(ss), C.byref(hp), C.byref(gr), C.byref(gs), _stream()))


# ---------------------------------------------------------------- sliding-window maintenance

def color_init(ctx: Context, mean: torch.Tensor, cam, image: torch.Tensor, o: A.Opts,
               color: Optional[torch.Tensor] = None):
    """Bilinear colour of Gaussians (mean (3, n), rows may be strided) from a
    camera image (3, H, W) (gsl_color_init).  Returns (color (3, n), valid
    uint8 (n,)); colour rows of invalid Gaussians are left as they were."""
    n = int(mean.shape[1])
    if mean.stride(1) != 1 or mean.dtype != torch.float32:
        raise ValueError("mean must be float32 (3, n) with unit column stride")
    image = image.contiguous()
    if color is None:
        color = torch.zeros(3, n, dtype=torch.float32, device=mean.device)
    valid = torch.empty(max(n, 1), dtype=torch.uint8, device=mean.device)
    c = A.camera_array([cam])
    A.check(A.lib().gsl_color_init(ctx.h, _p(mean), int(mean.stride(0)), n, c, _p(image), C.byref(o),
                                   _p(color), int(color.stride(0)), _p(valid), _stream()))
    return color, valid[:n]


def voxel_keys(ctx: Context, xyz: torch.Tensor, voxel_size: float, component_major: bool = False) -> torch.Tensor:
    """Voxel keys (int64 tensor holding the uint64 bits; -1 = no key) of
    points given as (P, 3), or (3, P) with component_major (gsl_voxel_keys)."""
    if xyz.dtype != torch.float32 or xyz.dim() != 2 or xyz.shape[0 if component_major else 1] != 3:
        raise ValueError("points must be a float32 (P, 3) tensor, or (3, P) when component-major")
    if component_major:
        P, ps, as_ = xyz.shape[1], xyz.stride(1), xyz.stride(0)
    else:
        P, ps, as_ = xyz.shape[0], xyz.stride(0), xyz.stride(1)
    keys = torch.empty(P, dtype=torch.int64, device=xyz.device)
    A.check(A.lib().gsl_voxel_keys(ctx.h, _p(xyz), P, ps, as_, float(voxel_size), _p(keys), _stream()))
    return keys


def window_workspace(ctx: Context, n: int, P: int) -> torch.Tensor:
    """A workspace of its own for one classify + compact pair (n Gaussians, P points)."""
    nb = C.c_size_t()
    A.check(A.lib().gsl_window_workspace_size(int(n), int(P), C.byref(nb)))
    return torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=ctx.device)


def window_classify(ctx: Context, points: torch.Tensor, voxel_size: float, keys: torch.Tensor, n: int,
                    ws: torch.Tensor):
    """Steps 1 and 3 (gsl_window_classify).  points (P, 3) float32; keys:
    the window's keys (first n used).  Returns (counts int32[2] = (D, A) and
    add_keys int64[P], both on the device; the first A add keys are valid)."""
    points = points.contiguous()
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be a float32 (P, 3) tensor")
    P = points.shape[0]
    counts = torch.zeros(2, dtype=torch.int32, device=points.device)
    add_keys = torch.empty(max(P, 1), dtype=torch.int64, device=points.device)
    A.check(A.lib().gsl_window_classify(ctx.h, _p(points), P, float(voxel_size), _p(keys), int(n), _p(counts),
                                        _p(add_keys), _p(ws), ws.numel(), _stream()))
    return counts, add_keys


def window_compact(ctx: Context, keys: torch.Tensor, rows: Optional[torch.Tensor], n: int, D: int,
                   add_keys: torch.Tensor, add_rows: Optional[torch.Tensor], ws: torch.Tensor, evict: bool = True):
    """Steps 2 and 4 in place (gsl_window_compact).  keys int64 (ld,), rows
    float32 (R, ld) (or None); add_keys (A,), add_rows (R, A).  Returns
    (evicted_keys (D,), evicted_rows (R, D), status int32[1]) on the device."""
    ld = keys.shape[0]
    R = 0 if rows is None else rows.shape[0]
    if rows is not None and (rows.dtype != torch.float32 or rows.shape[1] != ld or rows.stride(1) != 1
                             or rows.stride(0) != ld):
        raise ValueError("rows must be a float32 (R, ld) row-major tensor with the keys' length")
    Aadd = int(add_keys.shape[0])
    add_keys = add_keys.contiguous()
    if R and Aadd:
        add_rows = add_rows.contiguous()
        if add_rows.shape != (R, Aadd) or add_rows.dtype != torch.float32:
            raise ValueError("add_rows must be float32 (R, A)")
    dev = keys.device
    ek = torch.empty(int(D), dtype=torch.int64, device=dev) if evict else None
    er = torch.empty(R, int(D), dtype=torch.float32, device=dev) if evict and R else None
    status = torch.empty(1, dtype=torch.int32, device=dev)  # always written
    A.check(A.lib().gsl_window_compact(ctx.h, _p(keys), _p(rows), R, ld, int(n), int(D), _p(add_keys),
                                       _p(add_rows) if R and Aadd else None, Aadd, _p(ek), _p(er), _p(ws),
                                       ws.numel(), _p(status), _stream()))
    return ek, er, status


def window_transfer(ctx: Context, direction: int, src_keys: Optional[torch.Tensor], src_rows: Optional[torch.Tensor],
                    dst_keys: Optional[torch.Tensor], dst_rows: Optional[torch.Tensor], count: int):
    """gsl_window_transfer: `count` Gaussians' keys (int64 (>= count,)) and
    rows (float32 (R, ld) with unit column stride) between device tensors and
    pinned host tensors, asynchronously on the current stream.  direction:
    A.GSL_D2H or A.GSL_H2D."""
    R = 0
    sld = dld = 0
    if src_rows is not None:
        for t in (src_rows, dst_rows):
            if t is None or t.dtype != torch.float32 or t.dim() != 2 or t.stride(1) != 1:
                raise ValueError("rows must be float32 (R, ld) tensors with unit column stride")
        if src_rows.shape[0] != dst_rows.shape[0]:
            raise ValueError("source and destination row counts differ")
        R, sld, dld = int(src_rows.shape[0]), int(src_rows.stride(0)), int(dst_rows.stride(0))
    A.check(A.lib().gsl_window_transfer(ctx.h, int(direction), _p(src_keys), _p(src_rows), sld, _p(dst_keys),
                                        _p(dst_rows), dld, R, int(count), _stream()))


class _Pinned:
    """A growable pinned host buffer of (rows, columns) (rows = 0: 1-D)."""

    def __init__(self, dtype, rows=0):
        self.dtype, self.rows, self.t = dtype, rows, None

    def get(self, cols: int) -> torch.Tensor:
        cols = max(1, int(cols))
        have = 0 if self.t is None else self.t.shape[-1]
        if have < cols:
            n = max(cols, int(have * 1.5))
            shape = (self.rows, n) if self.rows else (n,)
            self.t = torch.empty(shape, dtype=self.dtype, pin_memory=True)
        return self.t


class SlidingWindow:
    """The window of Gaussians at a fixed capacity on the device (Sec. II-C):
    one float32 block (3R, capacity) — R = 14 + 3K raw parameter rows, then
    the Adam first and second moments — and the voxel keys; the first n
    columns are live.  `update` runs one frame's incremental update."""

    def __init__(self, ctx: Context, capacity: int, voxel_size: float, sh_degree: int = 0):
        self.ctx, self.capacity, self.voxel_size = ctx, int(capacity), float(voxel_size)
        self.params = 14 + 3 * sh_count(sh_degree)
        self.ROWS = 3 * self.params
        dev = ctx.device
        self.block = torch.zeros(self.ROWS, self.capacity, dtype=torch.float32, device=dev)
        self.keys = torch.full((self.capacity,), -1, dtype=torch.int64, device=dev)
        self.d_step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.n = 0
        # pinned staging of the Gaussians that enter (from the host-side map) and leave
        self._in_keys, self._in_rows = _Pinned(torch.int64), _Pinned(torch.float32, self.ROWS)
        self._out_keys, self._out_rows = _Pinned(torch.int64), _Pinned(torch.float32, self.ROWS)

    def adam_state(self) -> AdamState:
        b, R = self.block, self.params
        return AdamState(b[0:R], b[R:2 * R], b[2 * R:3 * R], self.d_step, n=self.n)

    def update(self, points: torch.Tensor, fetch, ws: Optional[torch.Tensor] = None):
        """One frame: classify against the frame's points, then call
        fetch(add_keys int64 (A_vox,) on the host) -> (keys (A,), rows (3R, A))
        on the host, the Gaussians to append (from the global map or newly
        initialised; moments zero).  They are staged in pinned memory and
        copied to the device (gsl_window_transfer), the window is compacted,
        and the evicted Gaussians are copied back to pinned memory.  Returns
        (evicted_keys int64 (D,), evicted_rows float32 (3R, D)) on the host,
        views of the pinned staging valid until the next update, for the
        global map."""
        dev = self.keys.device
        ws = window_workspace(self.ctx, self.n, points.shape[0]) if ws is None else ws
        counts, add_vox = window_classify(self.ctx, points, self.voxel_size, self.keys, self.n, ws)
        D, A_vox = (int(x) for x in counts.cpu())
        akeys, arows = fetch(add_vox[:A_vox].cpu())
        akeys = torch.as_tensor(akeys, dtype=torch.int64).reshape(-1)
        Aadd = int(akeys.shape[0])
        arows = torch.as_tensor(arows, dtype=torch.float32).reshape(self.ROWS, Aadd)
        if self.n - D + Aadd > self.capacity:
            raise ValueError("window capacity exceeded")
        hk, hr = self._in_keys.get(Aadd), self._in_rows.get(Aadd)
        hk[:Aadd].copy_(akeys)
        hr[:, :Aadd].copy_(arows)
        dk = torch.empty(max(1, Aadd), dtype=torch.int64, device=dev)
        dr = torch.empty(self.ROWS, max(1, Aadd), dtype=torch.float32, device=dev)
        window_transfer(self.ctx, A.GSL_H2D, hk, hr, dk, dr, Aadd)
        ek, er, status = window_compact(self.ctx, self.keys, self.block, self.n, D, dk[:Aadd], dr[:, :Aadd], ws)
        ok, orows = self._out_keys.get(D), self._out_rows.get(D)
        if D:
            window_transfer(self.ctx, A.GSL_D2H, ek, er, ok, orows, D)
        torch.cuda.current_stream().synchronize()
        if int(status.item()) != 0:
            raise RuntimeError("window compaction rejected: stale classification")
        self.n = self.n - D + Aadd
        return ok[:D], orows[:, :D]


# ---------------------------------------------------------------- pose Jacobians (IESKF visual update)

@dataclass
class PoseJacobian:
    """Outputs of gsl_pose_jacobian: image (3 P_total), jac (18, P_total) with
    plane 6 ch + j = dI_ch/dxi_j, and per camera HtH (C,6,6), Htz (C,6),
    zz (C,) (None where not requested)."""
    image: Optional[torch.Tensor]
    jac: Optional[torch.Tensor]
    HtH: Optional[torch.Tensor]
    Htz: Optional[torch.Tensor]
    zz: Optional[torch.Tensor]


def pose_jacobian(ctx: Context, g: Gaussians, cams: CameraSet, o: A.Opts, proj: Proj, bins: Bins,
                  target: Optional[torch.Tensor] = None, weight: Optional[torch.Tensor] = None,
                  want_image: bool = False, want_jac: bool = False) -> PoseJacobian:
    """Per-pixel twist Jacobians of the rendered colour and, with a target
    image, the per-camera normal equations of the photometric model."""
    dev = ctx.device
    image = torch.empty(3 * cams.P_total, dtype=torch.float32, device=dev) if want_image else None
    jac = torch.empty(18, cams.P_total, dtype=torch.float32, device=dev) if want_jac else None
    HtH = Htz = zz = None
    if target is not None:
        HtH = torch.empty(cams.C, 6, 6, dtype=torch.float64, device=dev)
        Htz = torch.empty(cams.C, 6, dtype=torch.float64, device=dev)
        zz = torch.empty(cams.C, dtype=torch.float64, device=dev)
        target = target.contiguous()
    if weight is not None:
        weight = weight.contiguous()
    n = C.c_size_t()
    A.check(A.lib().gsl_pose_jacobian_workspace_size(ctx.h, cams.arr, cams.C, g.N, C.byref(o), bins.capacity,
                                                     C.byref(n)))
    ws = ctx.workspace(int(n.value))
    gs, ps, bs = g.struct(), proj.struct(), bins.struct()
    A.check(A.lib().gsl_pose_jacobian(ctx.h, C.byref(gs), cams.arr, cams.C, C.byref(o), C.byref(ps), C.byref(bs),
                                      _p(target), _p(weight), _p(image), _p(jac), _p(HtH), _p(Htz), _p(zz), _p(ws),
                                      ws.numel(), _stream()))
    return PoseJacobian(image, jac, HtH, Htz, zz)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def imu_to_camera_twist(R_CI, t_CI, R_CW) -> np.ndarray:
    """A (6,6) with xi_cam = A xi_imu (gsl_imu_to_camera_twist)."""
    R_CI = np.ascontiguousarray(R_CI, np.float64).reshape(9)
    t_CI = np.ascontiguousarray(t_CI, np.float64).reshape(3)
    R_CW = np.ascontiguousarray(R_CW, np.float64).reshape(9)
    out = np.zeros(36)
    A.check(A.lib().gsl_imu_to_camera_twist(_dptr(R_CI), _dptr(t_CI), _dptr(R_CW), _dptr(out)))
    return out.reshape(6, 6)


def ieskf_pose_update(HtRH, HtRz, P, dx_prior=None):
    """(delta (6,), P_post (6,6)) of one IESKF update (gsl_ieskf_pose_update)."""
    HtRH = np.ascontiguousarray(HtRH, np.float64).reshape(36)
    HtRz = np.ascontiguousarray(HtRz, np.float64).reshape(6)
    P = np.ascontiguousarray(P, np.float64).reshape(36)
    dx = None if dx_prior is None else np.ascontiguousarray(dx_prior, np.float64).reshape(6)
    delta, Pn = np.zeros(6), np.zeros(36)
    A.check(A.lib().gsl_ieskf_pose_update(_dptr(HtRH), _dptr(HtRz), _dptr(P), None if dx is None else _dptr(dx),
                                          _dptr(delta), _dptr(Pn)))
    return delta, Pn.reshape(6, 6)


def ieskf_visual_update(HtH_cam, Htz_cam, A_imu, P, dx_prior=None, noise_var: float = 1.0):
    """IESKF update of the IMU pose from one camera's photometric normal
    equations: H_imu = H_cam A, R = noise_var I (the per-pixel weights, if
    any, already applied)."""
    HtH_cam = np.ascontiguousarray(HtH_cam, np.float64).reshape(36)
    Htz_cam = np.ascontiguousarray(Htz_cam, np.float64).reshape(6)
    A_imu = np.ascontiguousarray(A_imu, np.float64).reshape(36)
    P = np.ascontiguousarray(P, np.float64).reshape(36)
    dx = None if dx_prior is None else np.ascontiguousarray(dx_prior, np.float64).reshape(6)
    delta, Pn = np.zeros(6), np.zeros(36)
    A.check(A.lib().gsl_ieskf_visual_update(_dptr(HtH_cam), _dptr(Htz_cam), _dptr(A_imu), float(noise_var), _dptr(P),
                                            None if dx is None else _dptr(dx), _dptr(delta), _dptr(Pn)))
    return delta, Pn.reshape(6, 6)


# ---------------------------------------------------------------- window

class WindowRender:
    """Forward render of a camera set as one unit (gsl_window_render):
    projection, binning and compositing of every camera, recorded into a HIP
    graph on the first call and replayed afterwards (new poses replay the same
    graph).  The buffers live here, so replays find them at the addresses the
    graph was recorded with.  `capacity` bounds the instance count; by default
    an eager binning at construction sizes it with `headroom`."""

    def __init__(self, ctx: Context, g: Gaussians, cams: CameraSet, o: A.Opts, capacity: Optional[int] = None,
                 headroom: float = 1.25):
        self.ctx, self.g, self.cams, self.opts = ctx, g, cams, _opts_copy(o)
        self.proj = Proj(cams.C, g.N, ctx.device)
        if capacity is None:
            project(ctx, g, cams, self.opts, out=self.proj)
            b = bin_sort(ctx, cams, g.N, self.opts, self.proj)
            capacity = int(b.K * headroom) + 4096
            del b
        self.bins = Bins(capacity, cams.tiles(self.opts.tile), ctx.device)
        self.ws = torch.empty(workspace_size(ctx, cams, g.N, self.opts, capacity), dtype=torch.uint8,
                              device=ctx.device)
        self.image = torch.empty(3 * cams.P_total, dtype=torch.float32, device=ctx.device)
        self.T_final = torch.empty(cams.P_total, dtype=torch.float32, device=ctx.device)
        self.n_walk = torch.empty(cams.P_total, dtype=torch.int32, device=ctx.device)

    def __call__(self, use_graph: bool = True):
        """Enqueues one render; returns (packed image, T_final, n_walk), valid
        once the stream reaches them and status() is 0."""
        gs, ps, bs = self.g.struct(), self.proj.struct(), self.bins.struct()
        A.check(A.lib().gsl_window_render(self.ctx.h, C.byref(gs), self.cams.arr, self.cams.C, C.byref(self.opts),
                                          C.byref(ps), C.byref(bs), _p(self.image), _p(self.T_final),
                                          _p(self.n_walk), _p(self.ws), self.ws.numel(), int(bool(use_graph)),
                                          _stream()))
        return self.image, self.T_final, self.n_walk

    def status(self) -> int:
        return int(self.bins.d_status.item())


class Window:
    """All buffers of one batched-window optimisation pass (gsl_window_step).

    The buffers are owned here so that a captured HIP graph can be replayed:
    after the first graph-mode step, later steps with the same objects only
    launch the graph."""

    def __init__(self, ctx: Context, g: Gaussians, cams: CameraSet, o: A.Opts, target: torch.Tensor,
                 loss: str = "l1", capacity: Optional[int] = None, keep_image: bool = False, headroom=1.15):
        self.ctx, self.g, self.cams, self.opts = ctx, g, cams, _opts_copy(o)
        self.target = target.contiguous()
        self.loss = LOSS[loss]
        self.keep_image = keep_image
        self.headroom = headroom
        self.grads = Grads(g.N, cams.C, ctx.device, g.sh_degree)
        self.d_loss = torch.zeros(1, dtype=torch.float64, device=ctx.device)
        self.image = torch.empty(3 * cams.P_total, dtype=torch.float32, device=ctx.device) if keep_image else None
        self._alloc(capacity)

    def _alloc(self, capacity):
        o = self.opts
        self.proj = Proj(self.cams.C, self.g.N, self.ctx.device)
        if capacity is None:
            project(self.ctx, self.g, self.cams, o, out=self.proj)
            b = bin_sort(self.ctx, self.cams, self.g.N, o, self.proj)
            capacity = int(b.K * self.headroom) + 4096
            del b
        self.bins = Bins(capacity, self.cams.tiles(o.tile), self.ctx.device)
        nb = workspace_size(self.ctx, self.cams, self.g.N, o, capacity)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=self.ctx.device)

    def step(self, use_graph: bool = True):
        gs, ps, bs, gr = self.g.struct(), self.proj.struct(), self.bins.struct(), self.grads.struct()
        A.check(A.lib().gsl_window_step(self.ctx.h, C.byref(gs), self.cams.arr, self.cams.C, C.byref(self.opts),
                                        _p(self.target), self.loss, C.byref(ps), C.byref(bs), _p(self.image),
                                        _p(self.d_loss), C.byref(gr), _p(self.ws), self.ws.numel(),
                                        int(bool(use_graph)), _stream()))

    def optimize(self, st: AdamState, hp: A.Adam, iters: int = 10, use_graph: bool = True) -> torch.Tensor:
        """`iters` window steps each followed by an Adam step (gsl_window_optimize);
        self.g must hold activation(st.raw) (adam_activate) and is updated.
        Returns the per-iteration losses (device float64)."""
        if st.N != self.g.N:
            raise ValueError("optimiser and window hold different Gaussian counts")
        key = (iters, id(st))
        if getattr(self, "_losses_key", None) != key:
            self._losses = torch.zeros(iters, dtype=torch.float64, device=self.ctx.device)
            self._losses_key = key
        gs, ps, bs, gr, ss = (self.g.struct(), self.proj.struct(), self.bins.struct(), self.grads.struct(),
                              st.struct())
        A.check(A.lib().gsl_window_optimize(self.ctx.h, C.byref(ss), C.byref(hp), C.byref(gs), self.cams.arr,
                                            self.cams.C, C.byref(self.opts), _p(self.target), self.loss, C.byref(ps),
                                            C.byref(bs), _p(self._losses), C.byref(gr), int(iters), _p(self.ws),
                                            self.ws.numel(), int(bool(use_graph)), _stream()))
        return self._losses

    def profiled_step(self, graph: bool = False):
        """One step (eager, or a replay of the profiling graph) with HIP events
        between its stages; returns the milliseconds of (project, bin_sort,
        fused render, adjoint, total)."""
        A.check(A.lib().gsl_profile(self.ctx.h, 1))
        try:
            self.step(use_graph=graph)
            ms = (C.c_float * 5)()
            A.check(A.lib().gsl_profile_read(self.ctx.h, ms, 5))
        finally:
            A.lib().gsl_profile(self.ctx.h, 0)
        return [float(x) for x in ms]

    def set_variant(self, variant: int, chunk: int = 0):
        """Pin the fused-kernel variant and LDS chunk depth (0: the tile's
        default) for this window's shapes (see gsl_window_variant)."""
        A.check(A.lib().gsl_window_variant(self.ctx.h, self.cams.arr, self.cams.C, self.g.N, int(self.opts.tile),
                                           int(variant), int(chunk)))

    def status(self) -> int:
        return int(self.bins.d_status.item())

    def tune(self):
        """Autotune tile size, LDS chunk depth and fused variant; re-allocates
        for the chosen tile.  Returns (tile, times) with the 45 times in the
        order tile (8, 16, 32) x chunk (64, 128, 256) x variant (0..4)."""
        o8 = _opts_copy(self.opts, tile=8)
        save = self.opts
        self.opts = o8
        self._alloc(None)  # capacity and ranges for tile 8 bound every tile size
        times = (C.c_float * TUNE_TIMES)()
        gs, ps, bs, gr = self.g.struct(), self.proj.struct(), self.bins.struct(), self.grads.struct()
        ot = _opts_copy(save)
        A.check(A.lib().gsl_window_tune(self.ctx.h, C.byref(gs), self.cams.arr, self.cams.C, C.byref(ot),
                                        _p(self.target), self.loss, C.byref(ps), C.byref(bs), _p(self.d_loss),
                                        C.byref(gr), _p(self.ws), self.ws.numel(), times, TUNE_TIMES, _stream()))
        self.opts = ot
        self._alloc(None)
        return int(ot.tile), [float(t) for t in times]
