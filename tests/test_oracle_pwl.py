"""Pins of the oracle's piecewise-linear cost and value curves (Sec. III-B,
eqs. (single ReLU) and (combined ReLUs)) against facts other than the oracle:
knot interpolation by numpy, exactness of IBP on a monotone curve, the linear
special case, direct power flow at points, brute force over vertices, the LP
of Problem 1 with epigraph rows, and finite differences.  No GPU."""
import math

import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import synth
from tests.test_oracle_pins import _lp_max


@pytest.fixture(scope="module")
def tiny():
    net = synth.with_pwl_costs(synth.make_config("tiny"), seed=5)
    return net, oracle.factors(net)


@pytest.fixture(scope="module")
def c500():
    net = synth.with_pwl_costs(synth.make_config("c500"), seed=6)
    return net, oracle.factors(net)


def _knots(net, j):
    """Breakpoints and values of curve j: 0 at x = 0, U_i at the end of segment i."""
    p, a, b, U = (np.asarray(net[k]) for k in ("seg_ptr", "seg_a", "seg_b", "seg_U"))
    caps = np.concatenate([net["gen_pmax"], net["load_dmax"]])
    s0, s1 = p[j], p[j + 1]
    xs = np.concatenate([[0.0], b[s0 + 1:s1], [caps[j]]])
    ys = np.concatenate([[0.0], U[s0:s1]])
    return (a[s0:s1], b[s0:s1], U[s0:s1]), xs, ys


def test_curve_is_knot_interpolation(c500):
    """F* of the ReLU chain equals linear interpolation between its knots (np.interp),
    and IBP of the chain over [lo, hi] is exactly [F*(lo), F*(hi)] (a monotone curve)."""
    net, _ = c500
    rng = np.random.default_rng(0)
    for j in range(0, net["seg_ptr"].size - 1, 7):
        (a, b, U), xs, ys = _knots(net, j)
        x = rng.uniform(0.0, xs[-1], 64)
        np.testing.assert_allclose(oracle.curve_value(a, b, U, x), np.interp(x, xs, ys),
                                   rtol=1e-13, atol=1e-12)
        lo, hi = np.sort(rng.uniform(0.0, xs[-1], 2))
        c, r = 0.5 * (lo + hi), 0.5 * (hi - lo)
        F_lo, F_hi = oracle.curve_interval(a, b, U, c, r)
        assert F_lo == pytest.approx(np.interp(c - r, xs, ys), rel=1e-12, abs=1e-12)
        assert F_hi == pytest.approx(np.interp(c + r, xs, ys), rel=1e-12, abs=1e-12)


def test_single_segment_curves_equal_linear_costs():
    """One segment a = price, b = 0, U = inf per device is the linear cost: bounds,
    gradients and point values match the linear-cost oracle."""
    net = synth.make_config("tiny")
    fac = oracle.factors(net)
    G = net["gen_bus"].size
    X = G + net["load_bus"].size
    lin = dict(net, seg_ptr=np.arange(X + 1, dtype=np.int32),
               seg_a=np.concatenate([net["gen_cost"], net["load_value"]]),
               seg_b=np.zeros(X), seg_U=np.full(X, np.inf),
               gen_cost=np.zeros(G), load_value=np.zeros(X - G))
    blo, bhi = synth.sub_boxes(net, 3, seed=4)
    for a, b in zip(blo, bhi):
        r0, r1 = oracle.ibp(net, a, b, fac), oracle.ibp(lin, a, b, fac)
        for k in ("f_lo", "f_hi", "S_lo", "S_hi"):
            assert r1[k] == pytest.approx(r0[k], rel=1e-13), k
        g0 = oracle.grad(net, a, b, 0.4, 0.6, fac)
        g1 = oracle.grad(lin, a, b, 0.4, 0.6, fac)
        np.testing.assert_allclose(g1[0], g0[0], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(g1[1], g0[1], rtol=1e-12, atol=1e-12)
    x = blo[0].astype(float)
    assert oracle.point_eval(lin, x, fac["ctg"]) == pytest.approx(oracle.point_eval(net, x, fac["ctg"]),
                                                                  rel=1e-13)


def test_zero_width_and_sampled_points(tiny, c500):
    """P5 and P7 with curves: zero-width boxes give f(x) from direct power flow, and
    seeded points of a box stay inside its bounds."""
    for (net, fac), n in ((tiny, 4000), (c500, 48)):
        lo, hi = synth.full_box(net)
        rng = np.random.default_rng(2)
        for _ in range(3):
            x = (lo + rng.random(lo.size) * (hi.astype(float) - lo)).astype(np.float32)
            r = oracle.ibp(net, x, x, fac)
            fx = oracle.point_eval(net, x.astype(float), fac["ctg"])
            assert r["f_lo"] == r["f_hi"]
            assert r["f_lo"] == pytest.approx(fx, rel=1e-9, abs=1e-9)
        blo, bhi = synth.sub_boxes(net, 2, seed=3)
        for a, b in [(lo, hi)] + list(zip(blo, bhi)):
            r = oracle.ibp(net, a, b, fac)
            span = b.astype(float) - a
            pts = a[None, :] + rng.random((n, a.size)) * span[None, :]
            verts = a[None, :] + (rng.random((n // 2, a.size)) < 0.5) * span[None, :]
            fv = oracle.point_eval_many(net, np.vstack([pts, verts]), fac["ctg"])
            tol = 1e-9 * max(1.0, abs(r["f_lo"]), abs(r["f_hi"]))
            assert fv.min() >= r["f_lo"] - tol and fv.max() <= r["f_hi"] + tol


def test_bounds_bracket_vertices_and_lp(tiny):
    """P6 with curves: convex costs and concave values keep f concave, so the minimum
    over the box sits at one of its 2^16 vertices and the maximum is the LP of
    Problem 1 with one epigraph row per segment."""
    net, fac = tiny
    X = net["seg_ptr"].size - 1
    bits = ((np.arange(2 ** X)[:, None] >> np.arange(X)[None, :]) & 1).astype(float)
    lo, hi = synth.full_box(net)
    boxes = [(lo, hi)] + list(zip(*synth.sub_boxes(net, 2, seed=9)))
    for a, b in boxes:
        V = a[None, :] + bits * (b.astype(float) - a)[None, :]
        fv = oracle.point_eval_many(net, V, fac["ctg"])
        r = oracle.ibp(net, a, b, fac)
        assert r["f_lo"] <= fv.min() + 1e-9 * abs(fv.min())
        lp = _lp_max(net, a.astype(float), b.astype(float), fac)
        assert lp >= fv.max() - 1e-6 * max(1.0, abs(fv.max()))
        assert r["f_hi"] >= lp - 1e-7 * max(1.0, abs(lp))


def test_gradient_matches_central_differences(tiny):
    """P11 with curves: the analytic VJP equals central differences (h = 1e-4)
    wherever the map is linear on [x - h, x + h]."""
    net, fac = tiny
    blo, bhi = synth.sub_boxes(net, 3, seed=8)
    h = 1e-4
    checked = 0
    for a, b in zip(blo.astype(float), bhi.astype(float)):
        for g_lo, g_hi in ((1.0, 0.0), (0.0, 1.0), (0.3, -0.7)):
            d_lo, d_hi, _ = oracle.grad(net, a, b, g_lo, g_hi, fac)

            def F(lo_, hi_):
                r = oracle.ibp(net, lo_, hi_, fac)
                return g_lo * r["f_lo"] + g_hi * r["f_hi"]

            for side, d in (("lo", d_lo), ("hi", d_hi)):
                for j in range(a.size):
                    lo_p, hi_p, lo_m, hi_m = a.copy(), b.copy(), a.copy(), b.copy()
                    if side == "lo":
                        lo_p[j] += h
                        lo_m[j] -= h
                        if lo_p[j] > b[j]:
                            continue
                    else:
                        hi_p[j] += h
                        hi_m[j] -= h
                        if hi_m[j] < a[j]:
                            continue
                    gp = oracle.grad(net, lo_p, hi_p, g_lo, g_hi, fac)
                    gm = oracle.grad(net, lo_m, hi_m, g_lo, g_hi, fac)
                    gj = (gp[0] if side == "lo" else gp[1])[j]
                    gmj = (gm[0] if side == "lo" else gm[1])[j]
                    if not (math.isclose(gj, d[j], rel_tol=1e-9, abs_tol=1e-9)
                            and math.isclose(gmj, d[j], rel_tol=1e-9, abs_tol=1e-9)):
                        continue
                    fd = (F(lo_p, hi_p) - F(lo_m, hi_m)) / (2 * h)
                    assert fd == pytest.approx(d[j], rel=1e-6, abs=1e-5), (side, j)
                    checked += 1
    assert checked > 100


def test_planted_curve_mistakes_are_caught(tiny, c500, monkeypatch):
    """A dropped cap U_i fails the knot interpolation pin; a generator curve added
    instead of subtracted fails the point-evaluation pin."""
    net, _ = c500
    j = int(np.flatnonzero(np.diff(net["seg_ptr"]) >= 3)[0])
    (a, b, U), xs, ys = _knots(net, j)
    x = np.linspace(0.0, xs[-1], 50)
    no_cap = oracle.curve_value(a, b, np.full_like(U, np.inf), x)
    assert not np.allclose(no_cap, np.interp(x, xs, ys), rtol=1e-9)

    tnet, tfac = tiny
    lo, hi = synth.full_box(tnet)
    xpt = (0.5 * lo + 0.5 * hi).astype(np.float32)
    fx = oracle.point_eval(tnet, xpt.astype(float), tfac["ctg"])
    assert oracle.ibp(tnet, xpt, xpt, tfac)["f_lo"] == pytest.approx(fx, rel=1e-9)
    G = tnet["gen_bus"].size
    real = oracle.ibp_oracle._curve_surplus

    def wrong(net_, mu, sg):
        lo_, hi_ = real(net_, mu, sg)
        # add the generator curves back twice: they are now counted with a + sign
        gl = gh = 0.0
        ptr, A, B, Uc = oracle.ibp_oracle._curves(net_)
        for j in range(G):
            l_, h_ = oracle.curve_interval(A[ptr[j]:ptr[j + 1]], B[ptr[j]:ptr[j + 1]], Uc[ptr[j]:ptr[j + 1]],
                                           mu[j], sg[j])
            gl += 2 * l_
            gh += 2 * h_
        return lo_ + gl, hi_ + gh

    monkeypatch.setattr(oracle.ibp_oracle, "_curve_surplus", wrong)
    assert oracle.ibp(tnet, xpt, xpt, tfac)["f_lo"] != pytest.approx(fx, rel=1e-9)
