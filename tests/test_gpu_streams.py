"""Calls queued on a side stream: the binding allocates the outputs and a
temporary workspace on the stream the kernels run on, so memory the default
stream allocates and overwrites right after the call returns cannot be the
memory those kernels still use.  Forward, backward and a branch-and-bound
round on a side stream must equal the same calls on the default stream."""
import numpy as np
import pytest

from paper_2511_15624_amd import ibp, synth
from paper_2511_15624_amd.split import BoxSplitter
from tests.test_gpu_forward import setup

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _scribble(torch, nbytes):
    """Allocates and overwrites about nbytes on the current stream."""
    junk = [torch.full((nbytes // 8 // 4,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4)]
    return junk


def test_side_stream_calls_equal_default_stream_calls():
    torch = _torch()
    net, fac, n = setup("c2000")
    blo, bhi = synth.sub_boxes(net, 512, seed=91)
    lo, hi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    g1 = torch.ones(512, dtype=torch.float64, device="cuda")
    r_lo, r_hi = ibp.ibp_bound_boxes(n, lo, hi)
    d_ref = ibp.ibp_bound_backward(n, lo, hi, None, g1, flags=ibp.IBP_F_UPPER_ONLY)
    torch.cuda.synchronize()
    ws_bytes = n.workspace_bytes(512, ibp.IBP_F_BACKWARD)
    s = torch.cuda.Stream()
    for _ in range(3):
        f_lo, f_hi = ibp.ibp_bound_boxes(n, lo, hi, stream=s)        # temporary workspace freed on return
        junk = _scribble(torch, ws_bytes)
        d_lo, d_hi = ibp.ibp_bound_backward(n, lo, hi, None, g1, flags=ibp.IBP_F_UPPER_ONLY, stream=s)
        junk += _scribble(torch, ws_bytes)
        s.synchronize()
        torch.cuda.synchronize()
        assert torch.equal(f_lo, r_lo) and torch.equal(f_hi, r_hi)
        assert torch.equal(d_lo, d_ref[0]) and torch.equal(d_hi, d_ref[1])
        del junk, f_lo, f_hi, d_lo, d_hi


def test_splitting_round_on_a_side_stream():
    torch = _torch()
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 64, seed=92)
    lo, hi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    a = BoxSplitter(n, lo, hi, rounds=3)
    b = BoxSplitter(n, lo, hi, rounds=3)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for _ in range(3):
        a.step()
        b.step(stream=s)
        junk = _scribble(torch, 1 << 24)
        s.synchronize()
        torch.cuda.synchronize()
        del junk
    assert torch.equal(a.root_ub, b.root_ub) and torch.equal(a.root_lb, b.root_lb)
    assert torch.equal(a.leaf_lo, b.leaf_lo) and torch.equal(a.leaf_hi, b.leaf_hi)
