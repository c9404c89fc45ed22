"""torch.autograd.Function over the C ABI: forward = ibp_bound_boxes,
backward = ibp_bound_backward (the hand-written VJP kernels).

Gradients are taken with respect to the float32 box endpoints; the library
returns them in float64 and they are cast to the endpoints' dtype.  The
forward keeps its intermediates (box preparation, base flows, line and outage
constants) in a workspace held by the autograd graph, and the backward reuses
them instead of recomputing them (IBP_F_KEEP_PREP / IBP_F_REUSE_PREP); the
workspace has the backward's size and lives until the graph is freed.  When
only one bound reaches the loss, the backward is the one-sided call (the
gradient of f_hi alone takes the screened sweep).
"""
from __future__ import annotations

import torch

from . import ibp as _ibp


class IBPBound(torch.autograd.Function):
    """(f_lo, f_hi) = IBPBound.apply(lo, hi, net) for float32 device boxes [n_box, X]."""

    @staticmethod
    def forward(ctx, lo, hi, net, flags: int = 0):
        lo_d, hi_d = lo.detach().contiguous(), hi.detach().contiguous()
        ws = _ibp.Workspace(net)
        f_lo, f_hi = _ibp.ibp_bound_boxes(net, lo_d, hi_d, flags=flags | _ibp.IBP_F_KEEP_PREP, ws=ws)
        ctx.save_for_backward(lo_d, hi_d)
        # an output that does not reach the loss gets None, not zeros, so
        # that the backward can take the one-sided call
        ctx.set_materialize_grads(False)
        ctx.net = net
        ctx.flags = flags
        ctx.ws = ws
        return f_lo, f_hi

    @staticmethod
    def backward(ctx, g_lo, g_hi):
        lo, hi = ctx.saved_tensors
        if g_lo is None and g_hi is None:
            ctx.ws = None
            return torch.zeros_like(lo), torch.zeros_like(hi), None, None
        flags = ctx.flags & _ibp.IBP_F_PLAIN
        if g_lo is None:
            flags |= _ibp.IBP_F_UPPER_ONLY  # the weight of f_lo is not read
        elif g_hi is None:
            flags |= _ibp.IBP_F_LOWER_ONLY
        try:
            d_lo, d_hi = _ibp.ibp_bound_backward(ctx.net, lo, hi, g_lo, g_hi, flags=flags | _ibp.IBP_F_REUSE_PREP,
                                                 ws=ctx.ws)
        except _ibp.IBPError as e:
            # the intermediates are gone (the tiles changed since the forward,
            # or the call was split into chunks): recompute them
            if e.name != "IBP_E_INVALID_ARG":
                raise
            d_lo, d_hi = _ibp.ibp_bound_backward(ctx.net, lo, hi, g_lo, g_hi, flags=flags, ws=ctx.ws)
        ctx.ws = None
        return d_lo.to(lo.dtype), d_hi.to(hi.dtype), None, None


def ibp_bound(net, lo, hi, flags: int = 0):
    return IBPBound.apply(lo, hi, net, flags)
