"""torch.autograd wrappers: SSIM and MS-SSIM as differentiable functions of
both planes, and the BT.601 luma front end.  Forward and backward both run in
libssimx; the backward recomputes the window moments instead of saving them.
SSIM and MS-SSIM are symmetric in their two planes (every term of the
Background-section definitions is), so the gradient with respect to the
reference plane is the library's adjoint with the two planes swapped."""
from __future__ import annotations

import torch

from . import ops


class SSIMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, cfg):
        ctx.save_for_backward(x, y)
        ctx.cfg = cfg
        return ops.ssim(x, y, cfg)

    @staticmethod
    def backward(ctx, g):
        x, y = ctx.saved_tensors
        gx = ops.ssim_backward(y, x, g, ctx.cfg).to(x.dtype) if ctx.needs_input_grad[0] else None
        gy = ops.ssim_backward(x, y, g, ctx.cfg).to(y.dtype) if ctx.needs_input_grad[1] else None
        return gx, gy, None


class MSSSIMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, cfg, weights, n_scales, renorm, cs_clamp, aggregation, coarse_separate):
        ctx.args = (cfg, tuple(weights), n_scales, renorm, cs_clamp, aggregation, coarse_separate)
        if coarse_separate:  # the split coarsest term is not in cs: the backward recomputes
            ctx.save_for_backward(x, y)
            return ops.ms_ssim(x, y, cfg, weights=weights, n_scales=n_scales, renorm=renorm, cs_clamp=cs_clamp,
                               aggregation=aggregation, coarse_separate=coarse_separate)
        score, cs = ops.ms_ssim(x, y, cfg, weights=weights, n_scales=n_scales, renorm=renorm, cs_clamp=cs_clamp,
                                aggregation=aggregation, return_cs=True)
        # the forward's values let the backward skip its windowed passes
        ctx.save_for_backward(x, y, score, cs)
        return score

    @staticmethod
    def backward(ctx, g):
        saved = ctx.saved_tensors
        x, y = saved[0], saved[1]
        fwd = (saved[2], saved[3]) if len(saved) == 4 else None
        cfg, weights, n_scales, renorm, cs_clamp, aggregation, coarse_separate = ctx.args
        kw = dict(weights=weights, n_scales=n_scales, renorm=renorm, cs_clamp=cs_clamp, aggregation=aggregation,
                  coarse_separate=coarse_separate, fwd=fwd)
        gx = gy = None
        if ctx.needs_input_grad[0]:  # the forward's values are symmetric too
            gx = ops.ms_ssim_backward(y, x, g, cfg, **kw).to(x.dtype)
        if ctx.needs_input_grad[1]:
            gy = ops.ms_ssim_backward(x, y, g, cfg, **kw).to(y.dtype)
        return gx, gy, None, None, None, None, None, None, None


class LumaFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rgb):
        ctx.in_dtype = rgb.dtype
        return ops.rgb_to_luma(rgb)

    @staticmethod
    def backward(ctx, gy):
        return ops.luma_grad_to_rgb(gy).to(ctx.in_dtype)


def ssim(x, y, cfg: ops.SSIMConfig | None = None, **kw):
    """Differentiable mean SSIM per frame, float32 [B]."""
    return SSIMFunction.apply(x, y, ops._cfg(cfg, kw))


def ms_ssim(x, y, cfg: ops.SSIMConfig | None = None, weights=ops.MS_WEIGHTS, n_scales: int = 5,
            renorm: bool = False, cs_clamp: bool = False, aggregation: str = "product", coarse_separate: bool = False,
            **kw):
    """Differentiable MS-SSIM per frame, float32 [B] (weighted product, or
    aggregation="sum" for the weighted average)."""
    return MSSSIMFunction.apply(x, y, ops._cfg(cfg, kw), tuple(weights), n_scales, renorm, cs_clamp, aggregation,
                                coarse_separate)


def luma(rgb):
    """Differentiable BT.601 luma of (B, 3, H, W) planes."""
    return LumaFunction.apply(rgb)


class MSSSIMLossFunction(torch.autograd.Function):
    """mean_b(1 - MS-SSIM_b) on BT.601 luma.  The forward runs the whole
    library evaluation up to the luma-level gradients (kept in a per-call
    workspace); the backward writes the RGB gradient with the upstream
    folded into the same kernel, so no separate scaling pass is needed."""

    @staticmethod
    def forward(ctx, ref, dis, cfg, n_scales, renorm):
        if ctx.needs_input_grad[1]:
            loss, _, ctx.state = ops.msssim_loss_rgb_deferred(ref, dis, cfg, n_scales=n_scales, renorm=renorm)
        else:
            loss, _, _ = ops.msssim_loss_rgb(ref, dis, cfg, n_scales=n_scales, renorm=renorm, with_grad=False)
            ctx.state = None
        ctx.grad_dtype = dis.dtype
        return loss

    @staticmethod
    def backward(ctx, g):
        if ctx.state is None:
            return None, None, None, None, None
        return None, ops.msssim_loss_rgb_grad(ctx.state, g, ctx.grad_dtype), None, None, None


def ms_ssim_loss_rgb(ref_rgb, dis_rgb, cfg: ops.SSIMConfig | None = None, n_scales: int = 3, renorm: bool = True,
                     **kw):
    """1 - MS-SSIM on BT.601 luma, averaged over the batch (the training loss
    of the differentiable workload).  When only the distorted planes need a
    gradient (the training case) the loss and that gradient come from the
    library's loss calls; otherwise the composed path gives gradients to both
    planes."""
    cfg = ops._cfg(cfg, kw)
    ref4 = ref_rgb.unsqueeze(0) if ref_rgb.dim() == 3 else ref_rgb
    dis4 = dis_rgb.unsqueeze(0) if dis_rgb.dim() == 3 else dis_rgb
    if not ref4.requires_grad and ref4.shape == dis4.shape and ref4.dtype == dis4.dtype and \
            ref4.dtype in (torch.float32, torch.bfloat16) and ref4.stride(3) == 1 and dis4.stride(3) == 1:
        return MSSSIMLossFunction.apply(ref4, dis4, cfg, n_scales, renorm)
    return ms_ssim_loss_rgb_composed(ref_rgb, dis_rgb, cfg, n_scales=n_scales, renorm=renorm)


def ms_ssim_loss_rgb_composed(ref_rgb, dis_rgb, cfg: ops.SSIMConfig | None = None, n_scales: int = 3,
                              renorm: bool = True, **kw):
    """The same loss from the separate differentiable pieces (luma, MS-SSIM,
    mean); gradients flow to both planes."""
    cfg = ops._cfg(cfg, kw)
    yr = luma(ref_rgb)
    yd = luma(dis_rgb)
    return (1.0 - ms_ssim(yr, yd, cfg, n_scales=n_scales, renorm=renorm)).mean()
