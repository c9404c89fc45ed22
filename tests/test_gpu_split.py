"""GPU tests of the box-splitting rounds (gradient-ranked bisection)."""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_forward import setup
from tests.test_oracle_pins import _lp_max

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def test_splitting_tightens_and_stays_certified(tmp_path):
    torch = _torch()
    from paper_2511_15624_amd.split import BoxSplitter
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 6, seed=17)
    lo = torch.from_numpy(blo).cuda()
    hi = torch.from_numpy(bhi).cuda()
    sp = BoxSplitter(n, lo, hi, rounds=6)
    ub_prev = sp.root_ub.cpu().numpy().copy()
    lb_prev = sp.root_lb.cpu().numpy().copy()
    for r in range(6):
        if r == 3:  # checkpoint and resume through a fresh splitter
            path = tmp_path / "split.pt"
            torch.save(sp.state_dict(), path)
            sp2 = BoxSplitter(n, lo, hi, rounds=6)
            sp2.load_state_dict(torch.load(path, weights_only=True))
            sp = sp2
        sp.step()
        torch.cuda.synchronize()
        ub = sp.root_ub.cpu().numpy()
        lb = sp.root_lb.cpu().numpy()
        assert np.all(ub <= ub_prev) and np.all(lb >= lb_prev)
        ub_prev, lb_prev = ub.copy(), lb.copy()
    # certified: LB <= max f over the root (Problem 1 LP) <= UB
    for b in range(6):
        lp = _lp_max(net, blo[b].astype(float), bhi[b].astype(float), fac)
        assert lb_prev[b] <= lp + 1e-6 * max(1.0, abs(lp))
        assert ub_prev[b] >= lp - 1e-6 * max(1.0, abs(lp))
    # leaves partition each root: inside it, and widths multiply to the root volume
    L_lo, L_hi, root = (t.cpu().numpy() for t in sp.leaves())
    assert L_lo.shape[0] == 6 * 7
    for b in range(6):
        m = root == b
        assert np.all(L_lo[m] >= blo[b]) and np.all(L_hi[m] <= bhi[b])
        w = (L_hi[m].astype(float) - L_lo[m]).clip(min=0)
        vol = np.prod(w / (bhi[b].astype(float) - blo[b]).clip(min=1e-300), axis=1).sum()
        assert vol == pytest.approx(1.0, rel=1e-9)
    # every leaf's f_hi is a valid bound for its own box
    f_lo, f_hi = ibp.ibp_bound_boxes(n, torch.from_numpy(L_lo).cuda(), torch.from_numpy(L_hi).cuda())
    fh = f_hi.cpu().numpy()
    for i in range(0, L_lo.shape[0], 7):
        r = oracle.ibp(net, L_lo[i], L_hi[i], fac)
        assert fh[i] >= r["f_hi"]


def test_split_coordinate_follows_the_gradient():
    torch = _torch()
    from paper_2511_15624_amd.split import BoxSplitter
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 5, seed=3)
    lo = torch.from_numpy(blo).cuda()
    hi = torch.from_numpy(bhi).cuda()
    sp = BoxSplitter(n, lo, hi, rounds=2)
    sp.step()
    torch.cuda.synchronize()
    k_lo = sp.kid_lo.cpu().numpy()
    k_hi = sp.kid_hi.cpu().numpy()
    d_lo, d_hi = ibp.ibp_bound_backward(n, lo, hi, torch.zeros(5, dtype=torch.float64, device="cuda"),
                                        torch.ones(5, dtype=torch.float64, device="cuda"))
    d_lo, d_hi = d_lo.cpu().numpy(), d_hi.cpu().numpy()
    for b in range(5):
        w = 0.5 * (bhi[b].astype(float) - blo[b])
        score = np.where(w > 0, (d_hi[b] - d_lo[b]) * w, -np.inf)
        j = int(np.argmax(score))
        changed = np.flatnonzero(k_hi[2 * b] != bhi[b])
        assert list(changed) == [j]
        assert k_lo[2 * b + 1, j] == k_hi[2 * b, j]
