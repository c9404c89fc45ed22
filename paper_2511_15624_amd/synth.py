"""Seeded synthetic SC-DCOPF instances and input boxes.

This module is the only code shared by the oracle side and the GPU side: it
draws networks, device data and boxes from ``numpy.random.default_rng`` and
holds none of the bounding arithmetic (no PTDF, LODF, interval or penalty
math).  Everything is returned as plain numpy arrays in a dict.

Instance recipe (stand-in for the GO3 cases of Table I, which are not
available): a uniform random labelled spanning tree decoded from a random
Pruefer sequence, plus uniformly random extra edges (no self loops, no
duplicates) up to ``n_line`` lines; line order shuffled and each line given a
random orientation.  Susceptance ``b ~ U[5, 50]`` p.u., flow limit
``fmax ~ U[0.5, 2.0]`` p.u. (the same limit is used for base case and
contingencies).  Generators sit on uniform buses with ``pmin = 0``,
``pmax ~ U[0.5, 3]`` and linear cost ``~ U[10, 50]``; flexible loads sit on
uniform buses with ``peak ~ U[0.2, 1.0]``, ``[dmin, dmax] = [0.6, 1.0] * peak``
and value ``~ U[60, 120]``.  Slack bus 0, penalty weights 1e3 (imbalance) and
5e2 (flow overload), as in the soft-constraint objective of Sec. II-D.

Piecewise-linear cost and value curves (``with_pwl_costs``; the curve form of
Sec. III-B): every device gets 1 to ``max_seg`` segments that split
``[0, pmax]`` (generators) or ``[0, dmax]`` (loads) at sorted uniform points.
Generator segment prices are sorted ``U[10, 50]`` draws, ascending (a convex
cost); load segment values are sorted ``U[60, 120]`` draws, descending (a
concave value).  Segment i is stored as slope ``a_i``, shift ``b_i`` (its
start) and cap ``U_i`` (the curve's value at its end); the linear weights are
set to zero so the curves carry the whole surplus.

Box endpoints are float32 by design: they are rounded outward to float32 and
those float32 values *are* the box that both the oracle and the kernels bound.
"""
from __future__ import annotations

import heapq
import math

import numpy as np

__all__ = [
    "CONFIGS",
    "make_network",
    "make_config",
    "full_box",
    "sub_boxes",
    "period_scales",
    "period_boxes",
    "find_bridges",
    "round_down_f32",
    "round_up_f32",
    "with_pwl_costs",
]

# name -> (n_bus, n_line, n_gen, n_load, n_ctg or None, network seed)
CONFIGS = {
    # tiny: 14 buses, 20 lines (13 tree + 7 extra), every non-islanding outage
    "tiny": dict(n_bus=14, n_line=20, n_gen=5, n_load=11, n_ctg=None, seed=1),
    # 500 buses, 700 lines, every non-islanding outage, one box
    "c500": dict(n_bus=500, n_line=700, n_gen=90, n_load=300, n_ctg=None, seed=2),
    # batched form: 2000 buses, 3200 lines, 18 periods x 1024 sub-boxes
    "c2000": dict(n_bus=2000, n_line=3200, n_gen=400, n_load=1200, n_ctg=None, seed=3),
    # large form: 8316 buses, 14000 lines, 8000 sampled non-islanding outages
    "c8316": dict(n_bus=8316, n_line=14000, n_gen=1500, n_load=5000, n_ctg=8000, seed=4),
}


def round_down_f32(x):
    """Largest float32 value <= x (elementwise)."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    bad = f.astype(np.float64) > x
    f[bad] = np.nextafter(f[bad], np.float32(-np.inf))
    return f


def round_up_f32(x):
    """Smallest float32 value >= x (elementwise)."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    bad = f.astype(np.float64) < x
    f[bad] = np.nextafter(f[bad], np.float32(np.inf))
    return f


def _pruefer_tree(n: int, rng: np.random.Generator):
    """Edges of the labelled tree encoded by a uniformly random Pruefer sequence."""
    if n == 1:
        return []
    if n == 2:
        return [(0, 1)]
    seq = rng.integers(0, n, size=n - 2)
    degree = np.ones(n, dtype=np.int64)
    for x in seq:
        degree[x] += 1
    leaves = [i for i in range(n) if degree[i] == 1]
    heapq.heapify(leaves)
    edges = []
    for x in seq:
        leaf = heapq.heappop(leaves)
        edges.append((leaf, int(x)))
        degree[x] -= 1
        if degree[x] == 1:
            heapq.heappush(leaves, int(x))
    u = heapq.heappop(leaves)
    v = heapq.heappop(leaves)
    edges.append((u, v))
    return edges


def make_network(n_bus: int, n_line: int, n_gen: int, n_load: int, seed: int,
                 n_ctg: int | None = None) -> dict:
    """Draw one synthetic network (fixed draw order; see the module docstring)."""
    if n_line < n_bus - 1:
        raise ValueError("need at least n_bus - 1 lines for a connected network")
    max_lines = n_bus * (n_bus - 1) // 2
    if n_line > max_lines:
        raise ValueError("too many lines for a simple graph")
    rng = np.random.default_rng(seed)
    edges = _pruefer_tree(n_bus, rng)
    seen = {(min(u, v), max(u, v)) for u, v in edges}
    while len(edges) < n_line:
        u, v = (int(t) for t in rng.integers(0, n_bus, size=2))
        if u == v:
            continue
        key = (min(u, v), max(u, v))
        if key in seen:
            continue
        seen.add(key)
        edges.append((u, v))
    edges = np.asarray(edges, dtype=np.int64)
    edges = edges[rng.permutation(n_line)]
    flip = rng.random(n_line) < 0.5
    line_from = np.where(flip, edges[:, 1], edges[:, 0]).astype(np.int32)
    line_to = np.where(flip, edges[:, 0], edges[:, 1]).astype(np.int32)
    line_b = rng.uniform(5.0, 50.0, n_line)
    fmax = rng.uniform(0.5, 2.0, n_line)
    gen_bus = rng.integers(0, n_bus, n_gen).astype(np.int32)
    gen_pmax = rng.uniform(0.5, 3.0, n_gen)
    gen_cost = rng.uniform(10.0, 50.0, n_gen)
    load_bus = rng.integers(0, n_bus, n_load).astype(np.int32)
    peak = rng.uniform(0.2, 1.0, n_load)
    load_value = rng.uniform(60.0, 120.0, n_load)
    net = dict(
        n_bus=int(n_bus),
        slack_bus=0,
        line_from=line_from,
        line_to=line_to,
        line_b=line_b,
        fmax_base=fmax.copy(),
        fmax_ctg=fmax.copy(),
        gen_bus=gen_bus,
        gen_cost=gen_cost,
        gen_pmin=np.zeros(n_gen),
        gen_pmax=gen_pmax,
        load_bus=load_bus,
        load_value=load_value,
        load_dmin=0.6 * peak,
        load_dmax=1.0 * peak,
        zeta_inj=1.0e3,
        zeta_f=5.0e2,
        ctg_line=None,
    )
    if n_ctg is not None:
        bridge = find_bridges(n_bus, line_from, line_to)
        candidates = np.flatnonzero(~bridge)
        if n_ctg > candidates.size:
            raise ValueError(f"only {candidates.size} non-islanding lines, asked {n_ctg}")
        pick = rng.choice(candidates, size=n_ctg, replace=False)
        net["ctg_line"] = np.sort(pick).astype(np.int32)
    return net


def make_config(name: str) -> dict:
    c = CONFIGS[name]
    return make_network(c["n_bus"], c["n_line"], c["n_gen"], c["n_load"], c["seed"],
                        n_ctg=c["n_ctg"])


def find_bridges(n_bus: int, line_from, line_to) -> np.ndarray:
    """Boolean mask of lines whose removal disconnects the graph.

    Used only to pick a seeded subset of non-islanding outages for the large
    workload; iterative depth-first search with low-link values.
    """
    line_from = np.asarray(line_from)
    line_to = np.asarray(line_to)
    n_line = line_from.size
    adj = [[] for _ in range(n_bus)]
    for l in range(n_line):
        a, b = int(line_from[l]), int(line_to[l])
        adj[a].append((b, l))
        adj[b].append((a, l))
    disc = [-1] * n_bus
    low = [0] * n_bus
    bridge = np.zeros(n_line, dtype=bool)
    t = 0
    for root in range(n_bus):
        if disc[root] >= 0:
            continue
        disc[root] = low[root] = t
        t += 1
        stack = [(root, -1, iter(adj[root]))]
        while stack:
            v, via, it = stack[-1]
            advanced = False
            for w, l in it:
                if l == via:
                    continue
                if disc[w] < 0:
                    disc[w] = low[w] = t
                    t += 1
                    stack.append((w, l, iter(adj[w])))
                    advanced = True
                    break
                low[v] = min(low[v], disc[w])
            if advanced:
                continue
            stack.pop()
            if stack:
                p = stack[-1][0]
                low[p] = min(low[p], low[v])
                if low[v] > disc[p]:
                    bridge[via] = True
    return bridge


def input_range(net: dict, load_scale: float = 1.0):
    """Float64 [lo, hi] of the inputs x = (p_g, p_d): generators first, then loads."""
    lo = np.concatenate([net["gen_pmin"], net["load_dmin"] * load_scale])
    hi = np.concatenate([net["gen_pmax"], net["load_dmax"] * load_scale])
    return lo, hi


def full_box(net: dict, load_scale: float = 1.0):
    """The whole admissible box [pmin, pmax] x [dmin, dmax], rounded outward to float32."""
    lo, hi = input_range(net, load_scale)
    return round_down_f32(lo), round_up_f32(hi)


def sub_boxes(net: dict, n_box: int, seed: int, load_scale: float = 1.0):
    """Sub-boxes of the full box with log-uniform widths in [1%, 100%] of each range.

    For box b and input j: ``w = exp(U[ln 0.01, 0]) * (hi_j - lo_j)`` and
    ``a = lo_j + U[0, 1] * (hi_j - lo_j - w)``; the box is ``[a, a + w]``
    rounded outward to float32 and clamped into the float32 full box.
    Returns float32 arrays of shape (n_box, X).
    """
    rng = np.random.default_rng(seed)
    lo, hi = input_range(net, load_scale)
    flo, fhi = round_down_f32(lo), round_up_f32(hi)
    X = lo.size
    u_w = rng.random((n_box, X))
    u_a = rng.random((n_box, X))
    span = hi - lo
    w = np.exp(math.log(0.01) * (1.0 - u_w)) * span
    a = lo + u_a * (span - w)
    blo = np.maximum(round_down_f32(a), flo)
    bhi = np.minimum(round_up_f32(a + w), fhi)
    blo = np.minimum(blo, bhi)
    return blo.astype(np.float32), bhi.astype(np.float32)


def period_scales(n_period: int, seed: int) -> np.ndarray:
    """Load scale per period: 0.85 + 0.15 sin(2 pi t / n_period + phi), phi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    t = np.arange(n_period)
    return 0.85 + 0.15 * np.sin(2.0 * math.pi * t / n_period + phi)


def period_boxes(net: dict, n_period: int, boxes_per_period: int, seed: int):
    """Batched workload: per period, loads scaled by the period's sinusoid, then sub-boxes.

    Returns (lo, hi, period_index) with lo/hi float32 of shape
    (n_period * boxes_per_period, X).
    """
    scales = period_scales(n_period, seed)
    los, his, idx = [], [], []
    for t, s in enumerate(scales):
        blo, bhi = sub_boxes(net, boxes_per_period, seed * 1000 + 17 + t, load_scale=float(s))
        los.append(blo)
        his.append(bhi)
        idx.append(np.full(boxes_per_period, t, dtype=np.int32))
    return np.concatenate(los), np.concatenate(his), np.concatenate(idx)


def with_pwl_costs(net: dict, seed: int, max_seg: int = 4) -> dict:
    """A copy of ``net`` whose surplus comes from piecewise-linear curves.

    Adds ``seg_ptr`` (int32 [X + 1], segments of input j are
    ``seg_ptr[j]:seg_ptr[j + 1]``), ``seg_a``, ``seg_b``, ``seg_U`` (float64);
    ``gen_cost`` and ``load_value`` become zero.
    """
    rng = np.random.default_rng(seed)
    caps = np.concatenate([net["gen_pmax"], net["load_dmax"]])
    G = np.asarray(net["gen_bus"]).size
    ptr = [0]
    A, B, U = [], [], []
    for j, cap in enumerate(caps):
        n = int(rng.integers(1, max_seg + 1))
        cuts = np.sort(rng.uniform(0.0, cap, n - 1))
        starts = np.concatenate([[0.0], cuts])
        ends = np.concatenate([cuts, [cap]])
        if j < G:
            price = np.sort(rng.uniform(10.0, 50.0, n))
        else:
            price = np.sort(rng.uniform(60.0, 120.0, n))[::-1]
        A.extend(price)
        B.extend(starts)
        U.extend(np.cumsum(price * (ends - starts)))
        ptr.append(ptr[-1] + n)
    out = dict(net)
    out["gen_cost"] = np.zeros(G)
    out["load_value"] = np.zeros(caps.size - G)
    out["seg_ptr"] = np.asarray(ptr, dtype=np.int32)
    out["seg_a"] = np.asarray(A, dtype=np.float64)
    out["seg_b"] = np.asarray(B, dtype=np.float64)
    out["seg_U"] = np.asarray(U, dtype=np.float64)
    return out
