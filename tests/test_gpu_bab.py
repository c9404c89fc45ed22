"""GPU tests of branch and bound with screening over many root boxes.

No run of the method exists to compare against, so the tests check what the
mathematics fixes: every root's bounds bracket max f over the root (the LP of
Problem 1 on the 14-bus network), a certified status agrees with the sign of
that maximum, the recorded point attains the lower bound (direct power flow),
bounds only tighten, the open list is exactly the undecided roots, and a run
resumed from a checkpoint ends bitwise identical to an uninterrupted one.
"""
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


def _mixed_roots(net, n=24, seed=7):
    """Boxes of 30-90% of each range at seeded positions: some have max f < 0."""
    lo, hi = synth.full_box(net)
    span = hi.astype(float) - lo
    rng = np.random.default_rng(seed)
    A, B = [], []
    for _ in range(n):
        w = rng.uniform(0.3, 0.9)
        a = lo + rng.random(lo.size) * span * (1 - w)
        A.append(synth.round_down_f32(a))
        B.append(synth.round_up_f32(a + w * span))
    return np.asarray(A, np.float32), np.asarray(B, np.float32)


def test_statuses_agree_with_the_lp_and_bounds_bracket_it(tmp_path):
    torch = _torch()
    from paper_2511_15624_amd.split import BranchAndBound, CLOSED, NONNEGATIVE, OPEN, WELFARE_NEGATIVE
    net, fac, n = setup("tiny")
    A, B = _mixed_roots(net)
    lp = np.array([_lp_max(net, a.astype(float), b.astype(float), fac) for a, b in zip(A, B)])
    lo, hi = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    bb = BranchAndBound(n, lo, hi, rounds=60, relax=True, rel_tol=1e-6)
    st0 = bb.status.cpu().numpy()
    ub0 = bb.root_ub.cpu().numpy()
    assert st0[11] == WELFARE_NEGATIVE                  # IBP alone certifies this one
    ub_prev, lb_prev = bb.root_ub.cpu().numpy(), bb.root_lb.cpu().numpy()
    n_prev = bb.n_open
    for r in range(60):
        if r == 5:   # checkpoint and resume through a fresh instance
            path = tmp_path / "bab.pt"
            torch.save(bb.state_dict(), path)
            bb2 = BranchAndBound(n, lo, hi, rounds=60, relax=True, rel_tol=1e-6)
            bb2.load_state_dict(torch.load(path, weights_only=True))
            bb = bb2
        if not bb.step():
            break
        torch.cuda.synchronize()
        ub, lb = bb.root_ub.cpu().numpy(), bb.root_lb.cpu().numpy()
        assert np.all(ub <= ub_prev) and np.all(lb >= lb_prev)
        assert bb.n_open <= n_prev
        ub_prev, lb_prev, n_prev = ub, lb, bb.n_open
        st = bb.status.cpu().numpy()
        opened = bb.open_roots[:bb.n_open].cpu().numpy()
        assert list(opened) == list(np.flatnonzero(st == OPEN))
    st = bb.status.cpu().numpy()
    ub, lb = bb.root_ub.cpu().numpy(), bb.root_lb.cpu().numpy()
    tol = 1e-6 * np.maximum(1.0, np.abs(lp))
    assert np.all(ub >= lp - tol) and np.all(lb <= lp + tol)
    assert np.all(lp[st == WELFARE_NEGATIVE] < 0)
    assert np.all(lp[st == NONNEGATIVE] >= -tol[st == NONNEGATIVE])
    assert np.all(ub[st == CLOSED] - lb[st == CLOSED] <= 1e-6 * np.maximum(1.0, np.abs(ub[st == CLOSED])))
    # most roots have max f >= 0: points found while branching certify it
    assert np.sum(st == NONNEGATIVE) >= 21, st
    # root 18 has max f < 0 while IBP's root bound is positive: branching lowers it
    assert st0[18] == OPEN and ub[18] < 0.7 * ub0[18]
    print("statuses", st.tolist(), "root 18 bounds", ub[18], lb[18], "lp", lp[18], flush=True)
    # the recorded points are inside their roots and attain the lower bounds
    X = bb.root_x.cpu().numpy().astype(float)
    assert np.all(X >= A) and np.all(X <= B)
    fx = oracle.point_eval_many(net, X, fac["ctg"])
    assert np.all(fx >= lb - 1e-9 * np.maximum(1.0, np.abs(lb)))
    assert np.all(fx <= ub + 1e-9 * np.maximum(1.0, np.abs(ub)))


def test_resumed_run_is_bitwise_identical():
    torch = _torch()
    from paper_2511_15624_amd.split import BranchAndBound
    net, fac, n = setup("tiny")
    A, B = _mixed_roots(net, n=12, seed=3)
    lo, hi = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    a = BranchAndBound(n, lo, hi, rounds=8)
    for _ in range(8):
        a.step()
    b = BranchAndBound(n, lo, hi, rounds=8)
    for _ in range(3):
        b.step()
    c = BranchAndBound(n, lo, hi, rounds=8)
    c.load_state_dict({k: (v.clone() if hasattr(v, "clone") else v) for k, v in b.state_dict().items()})
    for _ in range(5):
        c.step()
    torch.cuda.synchronize()
    for k in ("root_ub", "root_lb", "root_x", "status", "n_leaf", "leaf_lo", "leaf_hi"):
        assert torch.equal(getattr(a, k), getattr(c, k)), k
    # unused slots hold NaN
    assert torch.allclose(a.leaf_fhi, c.leaf_fhi, rtol=0, atol=0, equal_nan=True)


def test_c500_relaxation_closes_more_than_ibp_alone():
    torch = _torch()
    from paper_2511_15624_amd.split import BranchAndBound
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 16, seed=23)
    lo, hi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    gaps = {}
    for relax in (False, True):
        bb = BranchAndBound(n, lo, hi, rounds=4, relax=relax, screen=False)
        bb.run(4)
        gaps[relax] = bb.gap().cpu().numpy()
        X = bb.root_x.cpu().numpy().astype(float)
        lb = bb.root_lb.cpu().numpy()
        fx = oracle.point_eval_many(net, X[:4], fac["ctg"])
        assert np.all(fx >= lb[:4] - 1e-9 * np.maximum(1.0, np.abs(lb[:4])))
        ub = bb.root_ub.cpu().numpy()
        for b in range(2):
            c = oracle.crown_upper(net, blo[b], bhi[b], fac)["f_hi"]
            # the root bound is no looser than the oracle's own root relaxation (slack for float32)
            assert ub[b] <= max(c, oracle.ibp(net, blo[b], bhi[b], fac)["f_hi"]) + 1e-5 * abs(c)
    assert np.sum(gaps[True]) < np.sum(gaps[False])
