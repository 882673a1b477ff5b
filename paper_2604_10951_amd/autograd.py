"""torch.autograd.Function over the HIP forward and backward renderers.

The forward runs preprocess -> bin -> sort -> render_forward; the backward
runs render_backward (blend, ray-splat intersection, projection) in the HIP
library.  The blend's discrete choices (accepted surfels, stopping points,
the Top-K set, the alpha clamp) are held fixed, so with Top-K only the
selected surfels receive gradient (Sec. 3.4).  Scales and opacity enter
already activated; ``rasterize`` applies exp / sigmoid to raw parameters in
torch, whose autograd chains through them.
"""
from __future__ import annotations

import torch

from .raster import Rasterizer


class RasterizeFeatures(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacity, feats, rast: Rasterizer):
        means, scales, quats, opacity = (t.contiguous() for t in (means, scales, quats, opacity))
        feats = feats.contiguous()
        frame = rast.render(means, scales, quats, opacity, feats, want_last=True)
        ctx.rast = rast
        ctx.frame = frame
        ctx.feat_dtype = feats.dtype
        ctx.save_for_backward(means, scales, quats, opacity, feats)
        ctx.mark_non_differentiable(frame.T, frame.n)
        return frame.feat, frame.T, frame.n

    @staticmethod
    def backward(ctx, grad_feat, grad_T, grad_n):
        means, scales, quats, opacity, feats = ctx.saved_tensors
        if grad_feat is None:
            return None, None, None, None, None, None
        g = ctx.rast.render_backward(means, scales, quats, opacity, feats, ctx.frame, grad_feat)
        return g["means"], g["scales"], g["quats"], g["opacity"], g["feats"].to(ctx.feat_dtype), None


def rasterize(means, log_scales, quats, opacity_logit, feats, rast: Rasterizer):
    """Render (total_pixels, C) features from raw parameters (log-scales and
    opacity logits are activated here); returns (features, T_final, n)."""
    return RasterizeFeatures.apply(means, torch.exp(log_scales), quats, torch.sigmoid(opacity_logit), feats, rast)
