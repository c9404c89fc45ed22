"""Gradient-ranked bisection of input boxes: tightening IBP bounds by
branching on the box (the paper names branch and bound over the inputs as the
way to tighten IBP bounds, Sec. I and Sec. V).

Each root box keeps up to ``rounds + 1`` leaves that partition it.  One round
(for every root at once, all on the device):

1. ``ibp_split_select``: the leaf with the largest upper bound f_hi;
2. ``ibp_bound_backward`` on those leaves with (g_lo, g_hi) = (0, 1): the
   gradient of f_hi with respect to the leaf endpoints;
3. ``ibp_split_bisect``: split at the float32 midpoint of the coordinate with
   the largest (d f_hi/d hi_j - d f_hi/d lo_j) * r_j;
4. ``ibp_bound_boxes`` on the two children, and on their centre points as
   zero-width boxes (f_lo there is a certified value of f at a feasible point);
5. ``ibp_split_update``: root upper bound = the smaller of its previous value
   and the largest leaf f_hi, root lower bound on max f = largest certified
   centre value.

The gap UB - LB of every root can only shrink.  The state (leaves, bounds,
round counter) can be saved with ``state_dict`` and restored with
``load_state_dict`` to resume a run.
"""
from __future__ import annotations

import ctypes
import time

import torch

from . import ibp as _ibp


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


class BoxSplitter:
    def __init__(self, net: _ibp.Network, lo: torch.Tensor, hi: torch.Tensor, rounds: int = 10):
        lo, hi = _ibp._check_boxes(net, lo, hi)
        self.net = net
        self.R, self.X = lo.shape
        self.S = rounds + 1
        self.n_used = 1
        self.round = 0
        dev = lo.device
        R, S, X = self.R, self.S, self.X
        self.leaf_lo = torch.zeros((R * S, X), dtype=torch.float32, device=dev)
        self.leaf_hi = torch.zeros((R * S, X), dtype=torch.float32, device=dev)
        self.leaf_lo.view(R, S, X)[:, 0] = lo
        self.leaf_hi.view(R, S, X)[:, 0] = hi
        self.leaf_fhi = torch.full((R * S,), float("nan"), dtype=torch.float64, device=dev)
        self.sel = torch.zeros(R, dtype=torch.int64, device=dev)
        self.sel_lo = torch.empty((R, X), dtype=torch.float32, device=dev)
        self.sel_hi = torch.empty((R, X), dtype=torch.float32, device=dev)
        self.kid_lo = torch.empty((2 * R, X), dtype=torch.float32, device=dev)
        self.kid_hi = torch.empty((2 * R, X), dtype=torch.float32, device=dev)
        self.cen = torch.empty((2 * R, X), dtype=torch.float32, device=dev)
        self.g_lo = torch.zeros(R, dtype=torch.float64, device=dev)
        self.g_hi = torch.ones(R, dtype=torch.float64, device=dev)
        self.ws_f = _ibp.Workspace(net)
        self.ws_b = _ibp.Workspace(net)
        self.ws_c = _ibp.Workspace(net)
        f_lo, f_hi = _ibp.ibp_bound_boxes(net, lo, hi, ws=self.ws_f)
        self.leaf_fhi.view(R, S)[:, 0] = f_hi
        self.root_ub = f_hi.clone()
        mid = 0.5 * lo + 0.5 * hi
        c_lo, _ = _ibp.ibp_bound_boxes(net, mid, mid, ws=self.ws_c)
        self.root_lb = c_lo.clone()
        self.ub0 = self.root_ub.clone()
        self.lb0 = self.root_lb.clone()

    def step(self, stream=None):
        if self.n_used >= self.S:
            raise RuntimeError("no free leaf slot left; create the splitter with more rounds")
        lib = _ibp.load_library()
        s = _ibp._stream_ptr(stream)
        R, S, X = self.R, self.S, self.X
        _ibp._check(lib.ibp_split_select(R, S, self.n_used, X, _p(self.leaf_lo), _p(self.leaf_hi),
                                         _p(self.leaf_fhi), _p(self.sel), _p(self.sel_lo), _p(self.sel_hi), s))
        d_lo, d_hi = _ibp.ibp_bound_backward(self.net, self.sel_lo, self.sel_hi, self.g_lo, self.g_hi,
                                             ws=self.ws_b, stream=stream)
        _ibp._check(lib.ibp_split_bisect(R, S, self.n_used, X, _p(self.leaf_lo), _p(self.leaf_hi), _p(self.sel),
                                         _p(self.sel_lo), _p(self.sel_hi), _p(d_lo), _p(d_hi), _p(self.kid_lo),
                                         _p(self.kid_hi), _p(self.cen), s))
        _, kid_fhi = _ibp.ibp_bound_boxes(self.net, self.kid_lo, self.kid_hi, ws=self.ws_f, stream=stream)
        cen_flo, _ = _ibp.ibp_bound_boxes(self.net, self.cen, self.cen, ws=self.ws_c, stream=stream)
        self.n_used += 1
        _ibp._check(lib.ibp_split_update(R, S, self.n_used, _p(self.sel), _p(kid_fhi), _p(cen_flo),
                                         _p(self.leaf_fhi), _p(self.root_ub), _p(self.root_lb), s))
        self.round += 1

    def gap(self):
        return self.root_ub - self.root_lb

    def run(self, rounds: int):
        """Runs `rounds` rounds; returns per-round total gap and wall seconds."""
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(rounds):
            self.step()
            torch.cuda.synchronize()
            hist.append((float(self.gap().sum()), time.perf_counter() - t0))
        return hist

    def leaves(self):
        """(lo, hi, root index) of the used leaves."""
        R, S = self.R, self.S
        idx = torch.arange(R * S, device=self.leaf_lo.device).view(R, S)[:, : self.n_used].reshape(-1)
        return self.leaf_lo[idx], self.leaf_hi[idx], idx // S

    def state_dict(self):
        return {k: getattr(self, k) for k in ("leaf_lo", "leaf_hi", "leaf_fhi", "root_ub", "root_lb", "ub0",
                                              "lb0")} | {"n_used": self.n_used, "round": self.round,
                                                         "S": self.S, "R": self.R, "X": self.X}

    def load_state_dict(self, st):
        if (st["S"], st["R"], st["X"]) != (self.S, self.R, self.X):
            raise ValueError("state does not match this splitter's shape")
        for k in ("leaf_lo", "leaf_hi", "leaf_fhi", "root_ub", "root_lb", "ub0", "lb0"):
            getattr(self, k).copy_(st[k])
        self.n_used = int(st["n_used"])
        self.round = int(st["round"])
