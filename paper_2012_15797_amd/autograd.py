"""torch.autograd wrapper: differentiable rendering for forward-model fits.

`render(psf, mix, x, y, flux, r_e, e1, e2, W, amp=None, ...)` returns float32
stamps [n, W, W]; its backward calls the library's adjoint kernels
(gfc_render_stamps_backward) and returns gradients for x, y, flux, r_e, e1,
e2 and, when `amp` is given, the mixture amplitudes [n_tables, 16].
"""

from __future__ import annotations

import torch

from . import api
from ._lib import GFC_KMAX


class RenderStamps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psf, mix, W, flags, cd, mix_id, x, y, flux, r_e, e1, e2, amp):
        gctx = psf.ctx
        a = None
        if amp is not None:  # a per-call table: the mixture's own amplitudes stay as they are
            a = amp.detach().to(gctx.torch_device, torch.float32).contiguous()
            if a.numel() != mix.n_tables * GFC_KMAX:
                raise ValueError("amp must hold n_tables x 16 values")
        out = api.gfc_render_stamps(gctx, psf, mix, x, y, flux, r_e, e1, e2, W, mix_id=mix_id,
                                    flags=flags, cd=cd, mix_amp=a)
        ctx.psf, ctx.mix, ctx.W, ctx.flags, ctx.cd, ctx.mix_id = psf, mix, W, flags, cd, mix_id
        ctx.has_amp = amp is not None
        ctx.amp_keep = a
        ctx.save_for_backward(x, y, flux, r_e, e1, e2)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        x, y, flux, r_e, e1, e2 = ctx.saved_tensors
        gctx = ctx.psf.ctx
        gp, ga = api.gfc_render_stamps_backward(
            gctx, ctx.psf, ctx.mix, x, y, flux, r_e, e1, e2, ctx.W, grad_out.contiguous(),
            mix_id=ctx.mix_id, flags=ctx.flags, cd=ctx.cd, mix_amp=ctx.amp_keep)
        r = r_e.to(gp.device, torch.float32)
        grads = [gp[:, 0], gp[:, 1], gp[:, 2], gp[:, 3] / r, gp[:, 4], gp[:, 5]]
        grads = [g.to(t.device, t.dtype).reshape(t.shape) if t.requires_grad else None
                 for g, t in zip(grads, (x, y, flux, r_e, e1, e2))]
        g_amp = ga if ctx.has_amp else None
        return (None, None, None, None, None, None, *grads, g_amp)


def render(psf, mix, x, y, flux, r_e, e1, e2, W, amp=None, mix_id=None, flags=0, cd=None):
    """Differentiable render.  Galaxy parameters are float32 device tensors
    of length n; amp (optional) is a float32 [n_tables, 16] tensor of mixture
    amplitudes used by this call (and its backward) instead of the table's;
    the mixture itself is not changed, so it may be shared with a server or
    other renders."""
    return RenderStamps.apply(psf, mix, int(W), int(flags), cd, mix_id, x, y, flux, r_e, e1, e2, amp)
