"""E as a torch.autograd.Function, with the hand-written backward.

``encode(rho, b0, kcoef, sens, fields, t, precision)`` returns m = E rho
([G][K] complex64) computed by the HIP library; its backward calls
``nfs_encode_backward`` for the gradients with respect to rho (E^H of the
output gradient), to the B0 map and to the dynamic field coefficients (see
include/nfs.h for the formulas).  sens, fields and t are treated as
constants.  No PyTorch arithmetic is involved beyond argument marshalling.
"""
import torch

from . import nfs


class _Encode(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, b0, kcoef, sens, fields, t, precision):
        prob = nfs.Problem(sens, fields, b0.detach(), kcoef.detach(), t, device=rho.device)
        ctx.prob = prob
        ctx.precision = precision
        ctx.save_for_backward(rho.detach().to(torch.complex64).contiguous())
        return nfs.apply_E(prob, rho.detach(), precision)

    @staticmethod
    def backward(ctx, grad_m):
        (rho,) = ctx.saved_tensors
        need_rho, need_b0, need_k = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        g_rho, g_b0, g_k = nfs.encode_backward(ctx.prob, rho, grad_m.contiguous(), ctx.precision, need_rho, need_b0,
                                               need_k)
        return g_rho, g_b0, g_k, None, None, None, None


def encode(rho, b0, kcoef, sens, fields, t, precision: str = "fp32"):
    """m = E rho, differentiable in rho (complex), b0 and kcoef (real)."""
    return _Encode.apply(rho, b0, kcoef, sens, fields, t, precision)
