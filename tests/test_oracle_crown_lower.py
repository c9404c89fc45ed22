"""Pins of the oracle's linear-relaxation lower bound (chords of the penalties)
against facts other than the oracle: with linear costs f is concave (linear
surplus minus convex penalties), so its minimum over a box sits at a vertex and
brute force over all 2^16 vertices of the 14-bus boxes gives it exactly; on a
box that varies one coordinate, with outage limits out of reach, every IBP
interval is exact and the relaxation equals that minimum, and so it does on
boxes small enough that no interval holds a kink; the linear function
the oracle assembles matches a direct per-element sum of the chord lines over
flows from direct power-flow solves; IBP's f_lo is never tighter; zero-width
boxes give the point value; planted mistakes fail.  No GPU."""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import synth
from tests.test_oracle_crown import _tiny_boxes, _vertices
from tests.test_oracle_pins import _direct_flows


@pytest.fixture(scope="module")
def tiny():
    net = synth.make_config("tiny")
    return net, oracle.factors(net)


@pytest.fixture(scope="module")
def c500():
    net = synth.make_config("c500")
    return net, oracle.factors(net)


def _boxes(net):
    lo, hi = synth.full_box(net)
    return [(lo, hi)] + list(zip(*synth.sub_boxes(net, 6, seed=3))) + _tiny_boxes(net, 3, seed=5, delta=0.05)


def test_below_the_vertex_minimum_and_never_below_ibp(tiny):
    net, fac = tiny
    tighter = 0
    for a, b in _boxes(net):
        fmin = oracle.point_eval_many(net, _vertices(a, b), fac["ctg"]).min()
        c = oracle.crown_lower(net, a, b, fac)["f_lo"]
        i = oracle.ibp(net, a, b, fac)["f_lo"]
        assert c <= fmin + 1e-9 * max(1.0, abs(fmin))
        assert c >= i - 1e-9 * max(1.0, abs(i))
        tighter += c > i + 1e-6 * abs(i)
    assert tighter >= 6


def test_exact_on_one_coordinate_boxes(tiny):
    """Only x_j varies and no outage limit can bind: the base and imbalance
    intervals are the exact images of [lo_j, hi_j], the sum of the chords is the
    chord of f along x_j, and the bound is min(f(lo), f(hi)); IBP is lower."""
    net0, fac = tiny
    net = dict(net0, fmax_ctg=np.full(np.asarray(net0["fmax_ctg"]).size, 1e9))
    lo, hi = synth.full_box(net)
    rng = np.random.default_rng(8)
    strict = 0
    for _ in range(12):
        x = (lo + rng.random(lo.size) * (hi.astype(float) - lo)).astype(np.float32)
        j = int(rng.integers(lo.size))
        a, b = x.copy(), x.copy()
        a[j], b[j] = lo[j], hi[j]
        ends = oracle.point_eval_many(net, np.vstack([a, b]).astype(float), fac["ctg"])
        c = oracle.crown_lower(net, a, b, fac)["f_lo"]
        assert c == pytest.approx(ends.min(), rel=1e-9, abs=1e-7)
        strict += oracle.ibp(net, a, b, fac)["f_lo"] < ends.min() - 1e-6 * abs(ends.min())
    assert strict >= 3


def test_exact_where_f_is_affine_on_the_box(tiny):
    """On boxes of relative half-width 1e-6 where no pre-activation interval
    holds a kink (the upper relaxation reports no decision near switching),
    every penalty is affine on its interval, so every chord is the penalty
    itself, outage elements included: the bound equals the smallest of all
    2^16 vertex values (direct power flow), and IBP's f_lo is strictly lower."""
    net, fac = tiny
    checked = 0
    for a, b in _tiny_boxes(net, 8, seed=11, delta=1e-6):
        if oracle.crown_upper(net, a, b, fac)["near"]:
            continue
        fv = oracle.point_eval_many(net, _vertices(a, b), fac["ctg"])
        c = oracle.crown_lower(net, a, b, fac)
        assert c["f_lo"] == pytest.approx(fv.min(), rel=1e-9, abs=1e-9)
        assert c["n_active"] > 0
        assert oracle.ibp(net, a, b, fac)["f_lo"] < fv.min() - 1e-9 * abs(fv.min())
        checked += 1
    assert checked >= 6


def _imbalance(net, f, p):
    """E^T f - p_inj from the line end points (no PTDF)."""
    z = -p.copy()
    np.add.at(z, np.asarray(net["line_from"]), f)
    np.add.at(z, np.asarray(net["line_to"]), -f)
    return z


def test_assembly_matches_direct_flows(tiny):
    """const + G.x equals the surplus minus the weighted chord lines summed element
    by element, with every pre-activation from direct (outaged) power-flow
    solves; and every line lies above its penalty there."""
    net, fac = tiny
    zi, zf = float(net["zeta_inj"]), float(net["zeta_f"])
    w = np.concatenate([-np.asarray(net["gen_cost"], float), np.asarray(net["load_value"], float)])
    fb = np.asarray(net["fmax_base"], float)
    fc = np.asarray(net["fmax_ctg"], float)
    rng = np.random.default_rng(12)
    for a, b in list(zip(*synth.sub_boxes(net, 2, seed=3)))[:2]:
        r = oracle.crown_lower(net, a, b, fac, keep_slopes=True)
        aI, bI = r["chord_imb"]
        ab, bb = r["chord_base"]
        A, B = r["chord_ctg"]
        for _ in range(4):
            x = a + rng.random(a.size) * (b.astype(float) - a)
            f, p = _direct_flows(net, x)
            zI = _imbalance(net, f, p)
            tot = w @ x - zi * np.sum(aI * zI + bI) - zf * np.sum(ab * f + bb)
            assert np.all(aI * zI + bI >= np.abs(zI) - 1e-9 * (1 + np.abs(zI)))
            assert np.all(ab * f + bb >= np.maximum(np.abs(f) - fb, 0) - 1e-9 * (1 + np.abs(f)))
            for k, c in enumerate(fac["ctg"]):
                z = _direct_flows(net, x, line_out=c)[0]
                assert A[k, c] == 0.0 and B[k, c] == 0.0
                tot -= zf * np.sum(A[k] * z + B[k])
                line = A[k] * z + B[k]
                pen = np.maximum(np.abs(z) - fc, 0)
                pen[c] = 0.0
                assert np.all(line >= pen - 1e-9 * (1 + np.abs(z)))
            assert r["const"] + r["G"] @ x == pytest.approx(tot, rel=1e-10, abs=1e-7)


def test_zero_width_box_is_the_point_value(tiny, c500):
    for net, fac in (tiny, c500):
        lo, hi = synth.full_box(net)
        x = (0.3 * lo + 0.7 * hi).astype(np.float32)
        fx = oracle.point_eval(net, x.astype(float), fac["ctg"])
        assert oracle.crown_lower(net, x, x, fac)["f_lo"] == pytest.approx(fx, rel=1e-9, abs=1e-9)


def test_sampled_points_above_the_bound(c500):
    net, fac = c500
    rng = np.random.default_rng(6)
    blo, bhi = synth.sub_boxes(net, 2, seed=9)
    for a, b in zip(blo, bhi):
        r = oracle.crown_lower(net, a, b, fac)
        span = b.astype(float) - a
        pts = a[None, :] + rng.random((16, a.size)) * span[None, :]
        verts = a[None, :] + (rng.random((8, a.size)) < 0.5) * span[None, :]
        fv = oracle.point_eval_many(net, np.vstack([pts, verts, r["vertex"][None, :]]), fac["ctg"])
        assert fv.min() >= r["f_lo"] - 1e-9 * abs(r["f_lo"])
        assert r["f_lo"] >= oracle.ibp(net, a, b, fac)["f_lo"] - 1e-9 * abs(r["f_lo"])


def test_with_curves_and_distinct_outage_limits(tiny):
    """Curves enter through their interval's lower end; still >= IBP's f_lo and
    <= every sampled point value."""
    from tests.test_oracle_pins import _emergency
    net = _emergency(synth.with_pwl_costs(tiny[0], seed=5), 3)
    fac = tiny[1]
    rng = np.random.default_rng(2)
    for a, b in zip(*synth.sub_boxes(net, 3, seed=7)):
        c = oracle.crown_lower(net, a, b, fac)["f_lo"]
        assert c >= oracle.ibp(net, a, b, fac)["f_lo"] - 1e-9 * abs(c)
        pts = a[None, :] + rng.random((64, a.size)) * (b.astype(float) - a)[None, :]
        assert oracle.point_eval_many(net, pts, fac["ctg"]).min() >= c - 1e-9 * abs(c)


def test_planted_mistakes_are_caught(tiny, monkeypatch):
    """Each of three plausible slips lifts the bound above the vertex minimum on
    some box: slopes of the wrong sign, an intercept that puts the line below
    the chord, and dropped intercepts."""
    net, fac = tiny
    real = oracle.ibp_oracle._chord

    def flipped(c, r, t):
        a, b = real(c, r, t)
        return -a, b

    def wrong_end(c, r, t):
        a, b = real(c, r, t)
        zu = c + r
        pu = np.maximum(np.abs(zu) - t, 0.0)
        return a, pu - a * zu - a * 0.5 * r

    def no_intercept(c, r, t):
        a, _ = real(c, r, t)
        return a, np.zeros_like(a)

    boxes = _boxes(net)
    fmins = {}
    for bad in (flipped, wrong_end, no_intercept):
        monkeypatch.setattr(oracle.ibp_oracle, "_chord", bad)
        broken = False
        for i, (a, b) in enumerate(boxes):
            if i not in fmins:
                fmins[i] = oracle.point_eval_many(net, _vertices(a, b), fac["ctg"]).min()
            c = oracle.crown_lower(net, a, b, fac)["f_lo"]
            if c > fmins[i] + 1e-6 * max(1.0, abs(fmins[i])):
                broken = True
                break
        assert broken, bad.__name__
    monkeypatch.setattr(oracle.ibp_oracle, "_chord", real)
