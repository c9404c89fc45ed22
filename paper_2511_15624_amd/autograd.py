"""torch.autograd.Function over the C ABI: forward = ibp_bound_boxes,
backward = ibp_bound_backward (the hand-written VJP kernels).

Gradients are taken with respect to the float32 box endpoints; the library
returns them in float64 and they are cast to the endpoints' dtype.
"""
from __future__ import annotations

import torch

from . import ibp as _ibp


class IBPBound(torch.autograd.Function):
    """(f_lo, f_hi) = IBPBound.apply(lo, hi, net) for float32 device boxes [n_box, X]."""

    @staticmethod
    def forward(ctx, lo, hi, net, flags: int = 0):
        f_lo, f_hi = _ibp.ibp_bound_boxes(net, lo.detach(), hi.detach(), flags=flags)
        ctx.save_for_backward(lo.detach(), hi.detach())
        ctx.net = net
        ctx.flags = flags
        return f_lo, f_hi

    @staticmethod
    def backward(ctx, g_lo, g_hi):
        lo, hi = ctx.saved_tensors
        n = lo.shape[0]
        if g_lo is None:
            g_lo = torch.zeros(n, dtype=torch.float64, device=lo.device)
        if g_hi is None:
            g_hi = torch.zeros(n, dtype=torch.float64, device=lo.device)
        d_lo, d_hi = _ibp.ibp_bound_backward(ctx.net, lo, hi, g_lo, g_hi, flags=ctx.flags)
        return d_lo.to(lo.dtype), d_hi.to(hi.dtype), None, None


def ibp_bound(net, lo, hi, flags: int = 0):
    return IBPBound.apply(lo, hi, net, flags)
