"""Branch and bound over input boxes: tightening IBP bounds by branching on the
box (the paper names branch and bound over the inputs as the way to tighten
IBP bounds, Sec. I and Sec. V) and screening instances for max f < 0
(welfare-negative or infeasible, Sec. III-D eq. (inf-or-wn)).

Each root box keeps up to ``rounds + 1`` leaves that partition it.  One round,
for every open root at once, all on the device:

1. ``ibp_split_select``: the leaf with the largest upper bound f_hi;
2. ``ibp_bound_backward`` on those leaves, one-sided with g_hi = 1: the
   gradient of f_hi with respect to the leaf endpoints;
3. ``ibp_split_bisect``: split at the float32 midpoint of the coordinate with
   the largest (d f_hi/d hi_j - d f_hi/d lo_j) * r_j;
4. bound the two children from above (IBP, or IBP tightened by the linear
   relaxation; one-sided calls, as only f_hi is used), and evaluate points
   inside them as zero-width boxes (f_lo there is a certified value of f;
   lower-bound-only calls): their centres, and with the relaxation the vertex
   that maximises its linear part;
5. ``ibp_split_update``: root upper bound = the smaller of its previous value
   and the largest leaf f_hi, root lower bound on max f = the best certified
   point value (the point is kept in ``root_x``);
6. ``ibp_split_screen`` (``BranchAndBound`` only): roots with a certified sign
   of max f or a closed gap leave the open list.

The gap UB - LB of every root can only shrink.  The state can be saved with
``state_dict`` and restored with ``load_state_dict`` to resume a run.
"""
from __future__ import annotations

import ctypes
import time

import torch

from . import ibp as _ibp

OPEN, WELFARE_NEGATIVE, NONNEGATIVE, CLOSED, INVALID = 0, 1, 2, 3, 4


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()


class BranchAndBound:
    """Best-first branch and bound over R root boxes [R, X] (float32, device).

    relax:   bound children with the linear relaxation (tighter upper bounds,
             and its maximising vertex as a second point per child).
    ref_iters: further relaxations per bound with slopes taken at reference
             points (see ``ibp_crown_bound_boxes``).
    screen:  drop roots from the open list once their status is decided
             (max f < 0 or >= 0 certified) or their gap is below rel_tol.
    """

    _STATE = ("leaf_lo", "leaf_hi", "leaf_fhi", "n_leaf", "root_ub", "root_lb", "root_x", "ub0", "lb0",
              "status", "open_roots")

    def __init__(self, net: _ibp.Network, lo: torch.Tensor, hi: torch.Tensor, rounds: int = 10,
                 relax: bool = True, screen: bool = True, rel_tol: float = 1e-6, ref_iters: int = 0):
        lo, hi = _ibp._check_boxes(net, lo, hi)
        self.net = net
        self.R, self.X = lo.shape
        self.S = rounds + 1
        self.relax = bool(relax)
        self.screen_on = bool(screen)
        self.rel_tol = float(rel_tol)
        self.ref_iters = int(ref_iters) if relax else 0
        self.round = 0
        dev = lo.device
        R, S, X = self.R, self.S, self.X
        self.P = 4 if self.relax else 2  # points per root and round
        self.leaf_lo = torch.zeros((R * S, X), dtype=torch.float32, device=dev)
        self.leaf_hi = torch.zeros((R * S, X), dtype=torch.float32, device=dev)
        self.leaf_lo.view(R, S, X)[:, 0] = lo
        self.leaf_hi.view(R, S, X)[:, 0] = hi
        self.leaf_fhi = torch.full((R * S,), float("nan"), dtype=torch.float64, device=dev)
        self.n_leaf = torch.ones(R, dtype=torch.int32, device=dev)
        self.sel = torch.zeros(R, dtype=torch.int64, device=dev)
        self.sel_lo = torch.empty((R, X), dtype=torch.float32, device=dev)
        self.sel_hi = torch.empty((R, X), dtype=torch.float32, device=dev)
        self.kid_lo = torch.empty((2 * R, X), dtype=torch.float32, device=dev)
        self.kid_hi = torch.empty((2 * R, X), dtype=torch.float32, device=dev)
        self.cen = torch.empty((2 * R, X), dtype=torch.float32, device=dev)
        self.vtx = torch.empty((2 * R, X), dtype=torch.float32, device=dev) if self.relax else None
        self.g_hi = torch.ones(R, dtype=torch.float64, device=dev)
        self.status = torch.zeros(R, dtype=torch.int32, device=dev)
        self.open_roots = torch.arange(R, dtype=torch.int64, device=dev)
        self.n_open_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.n_open = R
        self.ws_f = _ibp.Workspace(net)
        self.ws_b = _ibp.Workspace(net)
        self.ws_c = _ibp.Workspace(net)
        # root bounds and first points: the root centre (and the relaxation's vertex)
        f_hi, vt = self._bound(lo, hi, R)
        self.leaf_fhi.view(R, S)[:, 0] = f_hi
        self.root_ub = f_hi.clone()
        mid = 0.5 * lo + 0.5 * hi
        pts = torch.stack([mid, vt], 1) if self.relax else mid[:, None]
        p_lo, _ = _ibp.ibp_bound_boxes(net, pts.reshape(-1, X), pts.reshape(-1, X), ws=self.ws_c,
                                       flags=_ibp.IBP_F_LOWER_ONLY | _ibp.IBP_F_SCREEN_UPPER)
        p_lo = p_lo.view(R, -1)
        best = torch.nan_to_num(p_lo, nan=-float("inf")).argmax(1)
        self.root_lb = p_lo.gather(1, best[:, None])[:, 0].clone()
        self.root_x = pts[torch.arange(R, device=dev), best].contiguous()
        self.ub0 = self.root_ub.clone()
        self.lb0 = self.root_lb.clone()
        if self.screen_on:
            self.screen()

    def _bound(self, lo, hi, n, stream=None):
        if self.relax:
            vt = self.vtx[:n] if n <= self.vtx.shape[0] else torch.empty_like(lo)
            _, f_hi = _ibp.ibp_crown_bound_boxes(self.net, lo, hi, ws=self.ws_f, stream=stream, vertex=vt,
                                                 ref_iters=self.ref_iters, flags=_ibp.IBP_F_UPPER_ONLY)
            return f_hi, vt
        _, f_hi = _ibp.ibp_bound_boxes(self.net, lo, hi, ws=self.ws_f, stream=stream, flags=_ibp.IBP_F_UPPER_ONLY)
        return f_hi, None

    def screen(self, stream=None):
        """Classifies every root and compacts the open list; returns the open count."""
        lib = _ibp.load_library()
        with _ibp._on(stream):
            _ibp._check(lib.ibp_split_screen(self.R, _p(self.root_ub), _p(self.root_lb), self.rel_tol,
                                             _p(self.status), _p(self.open_roots), _p(self.n_open_dev),
                                             _ibp._stream_ptr(stream)))
            self.n_open = int(self.n_open_dev.item())      # waits for this stream
        return self.n_open

    def step(self, stream=None):
        """One round over the open roots, queued on `stream` (default: the
        current stream); returns False when none is open."""
        with _ibp._on(stream):
            return self._step(stream)

    def _step(self, stream):
        n = self.n_open if self.screen_on else self.R
        if n == 0:
            return False
        if self.round >= self.S - 1:
            raise RuntimeError("no free leaf slot left; create the splitter with more rounds")
        lib = _ibp.load_library()
        s = _ibp._stream_ptr(stream)
        S, X = self.S, self.X
        roots = self.open_roots[:n] if self.screen_on else None
        _ibp._check(lib.ibp_split_select(n, _p(roots), S, _p(self.n_leaf), X, _p(self.leaf_lo), _p(self.leaf_hi),
                                         _p(self.leaf_fhi), _p(self.sel), _p(self.sel_lo), _p(self.sel_hi), s))
        d_lo, d_hi = _ibp.ibp_bound_backward(self.net, self.sel_lo[:n], self.sel_hi[:n], None, self.g_hi[:n],
                                             ws=self.ws_b, stream=stream, flags=_ibp.IBP_F_UPPER_ONLY)
        _ibp._check(lib.ibp_split_bisect(n, _p(roots), S, _p(self.n_leaf), X, _p(self.leaf_lo), _p(self.leaf_hi),
                                         _p(self.sel), _p(self.sel_lo), _p(self.sel_hi), _p(d_lo), _p(d_hi),
                                         _p(self.kid_lo), _p(self.kid_hi), _p(self.cen), s))
        kid_fhi, vt = self._bound(self.kid_lo[:2 * n], self.kid_hi[:2 * n], 2 * n, stream)
        if self.relax:
            pts = torch.cat([self.cen[:2 * n].view(n, 2, X), vt.view(n, 2, X)], 1).contiguous()
        else:
            pts = self.cen[:2 * n]
        flat = pts.view(-1, X)
        p_lo, _ = _ibp.ibp_bound_boxes(self.net, flat, flat, ws=self.ws_c, stream=stream,
                                       flags=_ibp.IBP_F_LOWER_ONLY | _ibp.IBP_F_SCREEN_UPPER)
        _ibp._check(lib.ibp_split_update(n, _p(roots), S, _p(self.n_leaf), _p(self.sel), _p(kid_fhi), self.P,
                                         _p(p_lo), _p(flat), X, _p(self.leaf_fhi), _p(self.root_ub),
                                         _p(self.root_lb), _p(self.root_x), s))
        self.round += 1
        if self.screen_on:
            self.screen(stream)
        return True

    def gap(self):
        return self.root_ub - self.root_lb

    def counts(self):
        st = self.status.cpu()
        return {name: int((st == v).sum()) for name, v in
                (("open", OPEN), ("welfare_negative", WELFARE_NEGATIVE), ("nonnegative", NONNEGATIVE),
                 ("closed", CLOSED), ("invalid", INVALID))}

    def run(self, rounds: int):
        """Runs up to `rounds` rounds; returns per-round (total gap, seconds, open roots)."""
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(rounds):
            if not self.step():
                break
            torch.cuda.synchronize()
            hist.append((float(self.gap().sum()), time.perf_counter() - t0, self.n_open))
        return hist

    def leaves(self):
        """(lo, hi, root index) of the used leaves."""
        R, S = self.R, self.S
        used = torch.arange(S, device=self.leaf_lo.device)[None, :] < self.n_leaf[:, None].long()
        idx = torch.arange(R * S, device=self.leaf_lo.device).view(R, S)[used]
        return self.leaf_lo[idx], self.leaf_hi[idx], idx // S

    def state_dict(self):
        return {k: getattr(self, k) for k in self._STATE} | {"round": self.round, "S": self.S, "R": self.R,
                                                              "X": self.X, "n_open": self.n_open}

    def load_state_dict(self, st):
        if (st["S"], st["R"], st["X"]) != (self.S, self.R, self.X):
            raise ValueError("state does not match this splitter's shape")
        for k in self._STATE:
            getattr(self, k).copy_(st[k])
        self.round = int(st["round"])
        self.n_open = int(st["n_open"])


class BoxSplitter(BranchAndBound):
    """Every root is split in every round, children bounded by IBP, centre points
    as the certified lower bounds (no screening)."""

    def __init__(self, net: _ibp.Network, lo: torch.Tensor, hi: torch.Tensor, rounds: int = 10):
        super().__init__(net, lo, hi, rounds=rounds, relax=False, screen=False)
