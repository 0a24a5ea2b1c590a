"""torch.autograd.Function over the sparse chain: the filter as a trainable
layer (Sec. 6), with the hand-written adjoint of libdisk for its backward."""
from __future__ import annotations

import torch


class DiskChain(torch.autograd.Function):
    """y = F_Theta(x) for an image x [C][H][W] (FP32 or BF16), or the impulse
    response on an H x W canvas when x is None.  Gradients flow to theta and
    x.  A BF16 image is filtered with BF16 input and output (FP32 inside);
    the adjoint reads the input in FP32, so the image is saved widened to FP32
    (exactly: every BF16 value is an FP32 value) and x's gradient is returned
    in x's dtype."""

    @staticmethod
    def forward(ctx, theta, x, taps, boundary, H=None, W=None):
        from . import disk_forward
        out, saved = disk_forward(theta, taps, x, H=H, W=W, boundary=boundary, save=len(taps) > 1)
        ctx.taps = list(taps)
        ctx.boundary = boundary
        ctx.has_x = x is not None
        ctx.x_dtype = x.dtype if x is not None else None
        xs = x.float().contiguous() if x is not None else torch.empty(0, device=theta.device)
        ctx.save_for_backward(theta, xs, saved if saved is not None else torch.empty(0, device=theta.device))
        return out

    @staticmethod
    def backward(ctx, g):
        from . import disk_backward
        theta, x, saved = ctx.saved_tensors
        need_t = ctx.needs_input_grad[0]
        need_x = ctx.has_x and ctx.needs_input_grad[1]
        gt, gx = disk_backward(theta, ctx.taps, x if ctx.has_x else None, saved if saved.numel() else None,
                               g.float().contiguous(), boundary=ctx.boundary, need_theta=need_t, need_input=need_x)
        if gx is not None and gx.dtype != ctx.x_dtype:
            gx = gx.to(ctx.x_dtype)
        return gt, gx, None, None, None, None


def disk_chain(theta, x=None, taps=(8, 8, 8), boundary=1, H=None, W=None):
    return DiskChain.apply(theta, x, list(taps), boundary, H, W)
