"""torch.autograd binding of the image and its geometry adjoint.

``TDBPImage.apply(tx, rx, c, bufs_template, plan)`` returns the complex64 image
of one swath; its backward calls ``sas_bp_adjoint`` for the gradients of the
transmitter positions, receiver positions and sound speed, and
``sas_bp_reproject`` for the gradient of a complex64 echo (the image is linear
in the echo; 16-bit stored echoes get no gradient). Everything is marshalled
to the HIP library.
"""
from __future__ import annotations

import torch

from .api import SwathBuffers, sas_bp_adjoint, sas_bp_image, sas_bp_reproject


class TDBPImage(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tx: torch.Tensor, rx: torch.Tensor, c: torch.Tensor, echo: torch.Tensor,
                echo_scale, plan, image_out: torch.Tensor):
        buf = SwathBuffers(echo=echo, tx=tx.detach().contiguous(), rx=rx.detach().contiguous(),
                           c=c.detach().contiguous(), image=image_out, echo_scale=echo_scale)
        sas_bp_image(plan, [buf])
        ctx.plan = plan
        ctx.buf = buf
        return image_out.clone()

    @staticmethod
    def backward(ctx, grad_image: torch.Tensor):
        buf = ctx.buf
        plan = ctx.plan
        g = grad_image.contiguous()
        if g.dtype != torch.complex64:
            g = g.to(torch.complex64)
        gtx = grx = gc = gecho = None
        if any(ctx.needs_input_grad[:3]):
            gtx = torch.empty_like(buf.tx)
            grx = torch.empty_like(buf.rx)
            gc = torch.empty_like(buf.c)
            sas_bp_adjoint(plan, [buf], [g], [gtx], [grx], [gc])
        if ctx.needs_input_grad[3] and buf.echo.dtype == torch.complex64:
            gecho = torch.empty_like(buf.echo)
            sas_bp_reproject(plan, [buf], [g], [gecho])
        return gtx, grx, gc, gecho, None, None, None


def tdbp_image(plan, echo: torch.Tensor, tx: torch.Tensor, rx: torch.Tensor, c: torch.Tensor,
               echo_scale=None) -> torch.Tensor:
    """Differentiable image of one swath planned in ``plan`` (complex64 [nz, ny, nx])."""
    d = plan.descs[0]
    out = torch.empty((d.n[2], d.n[1], d.n[0]), dtype=torch.complex64, device=echo.device)
    return TDBPImage.apply(tx, rx, c, echo, echo_scale, plan, out)
