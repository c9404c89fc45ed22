"""The compute calls under HIP graph capture: a call captured on a stream
(torch.cuda.CUDAGraph) and replayed gives, on every replay, bitwise the
eager call's outputs.  The calls allocate nothing, queue no memset and never
synchronise the host, so capture records their kernels only.  Each graph is
replayed three times with eager calls of the library and host synchronisations
in between, and every replay is checked."""
import ctypes

import numpy as np
import pytest

from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_forward import _torch

pytestmark = pytest.mark.gpu

vp = ctypes.c_void_p


def _p(t):
    return vp(t.data_ptr()) if t is not None else vp()


def _replays_match(call, outs, torch):
    """Eager reference, capture, then three replays with eager work between."""
    cur = torch.cuda.current_stream()
    assert call(cur) == 0
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    side = torch.cuda.Stream()
    side.wait_stream(cur)
    with torch.cuda.stream(side):
        assert call(side) == 0
    cur.wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        assert call(torch.cuda.current_stream()) == 0
    for _ in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r)
        assert call(cur) == 0            # the library's own eager work between replays
        torch.cuda.synchronize()
    del g


@pytest.mark.parametrize("name,n_box", [("tiny", 1), ("c500", 37)])
def test_forward_under_capture(name, n_box):
    torch = _torch()
    lib = ibp.load_library()
    net = synth.make_config(name)
    n = ibp.Network(net, device=0)
    blo, bhi = synth.sub_boxes(net, n_box, seed=21)
    lo, hi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    ws = ibp.Workspace(n)
    buf, _ = ws.get(n_box)
    f_lo = torch.empty(n_box, dtype=torch.float64, device="cuda")
    f_hi = torch.empty(n_box, dtype=torch.float64, device="cuda")
    terms = torch.empty(n_box * 8, dtype=torch.float64, device="cuda")

    def call(s):
        return lib.ibp_bound_boxes(n.handle, n_box, _p(lo), _p(hi), _p(f_lo), _p(f_hi), _p(terms), _p(buf),
                                   buf.numel(), vp(s.cuda_stream), 0)
    _replays_match(call, [f_lo, f_hi, terms], torch)
    n.close()


def test_backward_and_lower_bound_under_capture():
    torch = _torch()
    lib = ibp.load_library()
    net = synth.make_config("c500")
    n = ibp.Network(net, device=0)
    blo, bhi = synth.sub_boxes(net, 6, seed=22)
    lo, hi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    ws = ibp.Workspace(n)
    X = n.n_input
    gl = torch.full((6,), 0.5, dtype=torch.float64, device="cuda")
    gh = torch.ones(6, dtype=torch.float64, device="cuda")
    d_lo = torch.empty(6 * X, dtype=torch.float64, device="cuda")
    d_hi = torch.empty(6 * X, dtype=torch.float64, device="cuda")
    buf_b, _ = ws.get(6, ibp.IBP_F_BACKWARD)

    def bwd(s):
        return lib.ibp_bound_backward(n.handle, 6, _p(lo), _p(hi), _p(gl), _p(gh), _p(d_lo), _p(d_hi), _p(buf_b),
                                      buf_b.numel(), vp(s.cuda_stream), 0)
    _replays_match(bwd, [d_lo, d_hi], torch)
    ws2 = ibp.Workspace(n)
    buf_c, _ = ws2.get(6, ibp.IBP_F_CROWN)
    f_lo = torch.empty(6, dtype=torch.float64, device="cuda")
    f_hi = torch.empty(6, dtype=torch.float64, device="cuda")
    c_lo = torch.empty(6, dtype=torch.float64, device="cuda")

    def lower(s):
        return lib.ibp_crown_lower_boxes(n.handle, 6, _p(lo), _p(hi), _p(f_lo), _p(f_hi), _p(c_lo), vp(),
                                         _p(buf_c), buf_c.numel(), vp(s.cuda_stream), 0)
    _replays_match(lower, [f_lo, f_hi, c_lo], torch)
    assert np.all(np.isfinite(c_lo.cpu().numpy()))
    n.close()
