"""torch.autograd.Function over the C ABI: forward = project, bin_sort,
render_fwd; backward = render_bwd (hand-written adjoint, recomputing forward
state from T_final and the walk length per pixel)."""
from __future__ import annotations

import torch

from . import ops


class RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, scale, quat, opacity, color, sh, pose, gctx, cams, o):
        g = ops.Gaussians(mean.detach().contiguous(), scale.detach().contiguous(), quat.detach().contiguous(),
                          opacity.detach().contiguous(), color.detach().contiguous(),
                          None if sh is None else sh.detach().contiguous())
        proj = ops.project(gctx, g, cams, o)
        bins = ops.bin_sort(gctx, cams, g.N, o, proj)
        image, T_final, n_walk = ops.render_fwd(gctx, cams, g.N, o, proj, bins)
        ctx.state = (g, gctx, cams, o, proj, bins, T_final, n_walk)
        ctx.mark_non_differentiable(T_final)
        return image, T_final

    @staticmethod
    def backward(ctx, d_image, d_T):
        g, gctx, cams, o, proj, bins, T_final, n_walk = ctx.state
        if d_image is None:
            d_image = torch.zeros(3 * cams.P_total, dtype=torch.float32, device=gctx.device)
        gr = ops.render_bwd(gctx, g, cams, o, proj, bins, T_final, n_walk, d_image.contiguous())
        return gr.mean, gr.scale, gr.quat, gr.opacity, gr.color, gr.sh, gr.pose, None, None, None


def rasterize(mean, scale, quat, opacity, color, cams: "ops.CameraSet", gctx: "ops.Context", o=None, pose=None,
              sh=None):
    """Differentiable render of the packed image of `cams`.

    mean, scale, color: (3, N); quat: (4, N) as (w, x, y, z); opacity: (N,);
    all float32 device tensors (activated values); sh: (3K, N) higher-order
    SH coefficients (row k * 3 + ch) or None.  `pose`, if given, is a
    (C, 6) float64 tensor of twists (dphi, dt) evaluated at zero, i.e. the
    cameras in `cams` are the linearisation point; its gradient is the
    photometric gradient of each camera's pose under a left perturbation of
    T_CW.  Returns (image (3 * P_total,), T_final (P_total,))."""
    o = o if o is not None else ops.opts()
    if pose is None:
        pose = torch.zeros((cams.C, 6), dtype=torch.float64, device=mean.device)
    return RasterizeFn.apply(mean, scale, quat, opacity, color, sh, pose, gctx, cams, o)
