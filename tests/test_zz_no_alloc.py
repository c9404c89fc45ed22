"""The no-allocation forward entry point (ibp_bound_boxes_noalloc) against
ibp_bound_boxes, through the C ABI: the same kernels on the library's own
scratch array must give the same bounds bit for bit, on two calls in a row
(the second with fewer boxes, so the scratch still holds the first call's
contents), at the largest box count the scratch takes, and one box beyond it
must be refused before anything is launched."""
import numpy as np
import pytest

from paper_2511_15624_amd import ibp, synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _noalloc(n, lo, hi, flags=0, terms=False):
    torch = _torch()
    nb = lo.shape[0]
    f_lo = torch.full((nb,), -7.0, dtype=torch.float64, device=lo.device)
    f_hi = torch.full((nb,), -7.0, dtype=torch.float64, device=lo.device)
    t = torch.full((nb, 8), -7.0, dtype=torch.float64, device=lo.device) if terms else None
    ibp.ibp_bound_boxes_noalloc(n, lo, hi, f_lo, f_hi, t, flags=flags)
    torch.cuda.synchronize()
    return f_lo, f_hi, t


def _max_boxes(n, flags=0):
    """Largest box count whose workspace fits the library's scratch array."""
    lo, hi = 1, 1
    while n.workspace_bytes(hi * 2, flags) <= ibp.IBP_NOALLOC_SCRATCH_BYTES:
        hi *= 2
    hi *= 2
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if n.workspace_bytes(mid, flags) <= ibp.IBP_NOALLOC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("name,first,flags", [("tiny", 23, 0), ("c500", 37, 0), ("c500", 9, ibp.IBP_F_PLAIN),
                                              ("c2000", 6, ibp.IBP_F_UPPER_ONLY)])
def test_noalloc_equals_workspace_call_twice(name, first, flags):
    torch = _torch()
    net = synth.make_config(name)
    n = ibp.Network(net, device=0)
    blo, bhi = synth.sub_boxes(net, first, seed=707)
    lo = torch.from_numpy(blo).cuda()
    hi = torch.from_numpy(bhi).cuda()
    for nb in (first, max(1, first // 3)):          # second call smaller: stale scratch contents
        print(f"[noalloc] {name} flags={flags} boxes={nb}", flush=True)
        a_lo, a_hi, a_t = _noalloc(n, lo[:nb], hi[:nb], flags=flags, terms=True)
        r_lo, r_hi, r_t = ibp.ibp_bound_boxes(n, lo[:nb], hi[:nb], terms=True, flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(a_lo, r_lo) and torch.equal(a_hi, r_hi) and torch.equal(a_t, r_t), nb
        assert torch.all(torch.isfinite(a_hi))


def test_noalloc_at_the_scratch_limit_and_beyond():
    """8316 buses: the largest batch the scratch holds, then one box (the
    headline whole box), and a call one box too large is refused."""
    torch = _torch()
    net = synth.make_config("c8316")
    n = ibp.Network(net, device=0)
    nmax = _max_boxes(n)
    assert nmax >= 1
    print(f"[noalloc] c8316 largest batch in the scratch: {nmax} boxes", flush=True)
    blo, bhi = synth.sub_boxes(net, nmax, seed=808)
    lo = torch.from_numpy(blo).cuda()
    hi = torch.from_numpy(bhi).cuda()
    a_lo, a_hi, _ = _noalloc(n, lo, hi)
    r_lo, r_hi = ibp.ibp_bound_boxes(n, lo, hi)
    torch.cuda.synchronize()
    assert torch.equal(a_lo, r_lo) and torch.equal(a_hi, r_hi)
    wlo, whi = synth.full_box(net)
    wlo = torch.from_numpy(wlo[None]).cuda()
    whi = torch.from_numpy(whi[None]).cuda()
    a_lo, a_hi, _ = _noalloc(n, wlo, whi)
    r_lo, r_hi = ibp.ibp_bound_boxes(n, wlo, whi)
    torch.cuda.synchronize()
    assert torch.equal(a_lo, r_lo) and torch.equal(a_hi, r_hi)
    big_lo = torch.cat([lo, lo[:1]])
    big_hi = torch.cat([hi, hi[:1]])
    f = torch.empty(nmax + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(ibp.IBPError) as e:
        ibp.ibp_bound_boxes_noalloc(n, big_lo, big_hi, f, f.clone())
    assert e.value.name == "IBP_E_WORKSPACE"
