"""Pins of the oracle's linear-relaxation (CROWN-style) upper bound against
facts other than the oracle: the LP of Problem 1 (a valid bound can never be
below it), brute force over the vertices of boxes on which f is affine (there
the relaxation is exact), direct power flow at points, IBP (never tighter),
sampled points, and planted mistakes.  No GPU."""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import synth
from tests.test_oracle_pins import _lp_max


@pytest.fixture(scope="module")
def tiny():
    net = synth.make_config("tiny")
    return net, oracle.factors(net)


@pytest.fixture(scope="module")
def c500():
    net = synth.make_config("c500")
    return net, oracle.factors(net)


def _vertices(a, b):
    X = a.size
    bits = ((np.arange(2 ** X)[:, None] >> np.arange(X)[None, :]) & 1).astype(float)
    return a[None, :].astype(float) + bits * (b.astype(float) - a)[None, :]


def _tiny_boxes(net, n, seed, delta):
    """Boxes of relative half-width delta around seeded points of the whole box."""
    lo, hi = synth.full_box(net)
    span = hi.astype(float) - lo
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        x = lo + rng.random(lo.size) * span
        a = synth.round_down_f32(np.maximum(lo, x - delta * span))
        b = synth.round_up_f32(np.minimum(hi, x + delta * span))
        out.append((a, b))
    return out


def test_valid_against_the_lp_and_never_above_ibp(tiny):
    """The LP of Problem 1 is max f (Remark 1); every relaxation bound is >= it, and
    the slope rule keeps it <= IBP's f_hi.  On sub-boxes it is strictly tighter."""
    net, fac = tiny
    lo, hi = synth.full_box(net)
    boxes = [(lo, hi)] + list(zip(*synth.sub_boxes(net, 6, seed=3)))
    tighter = 0
    for a, b in boxes:
        lp = _lp_max(net, a.astype(float), b.astype(float), fac)
        c = oracle.crown_upper(net, a, b, fac)["f_hi"]
        i = oracle.ibp(net, a, b, fac)["f_hi"]
        assert c >= lp - 1e-7 * max(1.0, abs(lp))
        assert c <= i + 1e-9 * max(1.0, abs(i))
        tighter += c < i - 1e-6 * abs(i)
    assert tighter >= 4


def test_exact_where_f_is_affine_on_the_box(tiny):
    """On boxes small enough that no element crosses a kink, f is affine on the box,
    and the bound equals the largest vertex value (all 2^16 vertices, direct power
    flow); IBP stays above it."""
    net, fac = tiny
    checked = 0
    for a, b in _tiny_boxes(net, 8, seed=11, delta=1e-6):
        r = oracle.crown_upper(net, a, b, fac)
        if r["near"]:
            continue
        fv = oracle.point_eval_many(net, _vertices(a, b), fac["ctg"])
        assert r["f_hi"] == pytest.approx(fv.max(), rel=1e-9, abs=1e-9)
        assert oracle.ibp(net, a, b, fac)["f_hi"] > fv.max() + 1e-9 * abs(fv.max())
        checked += 1
    assert checked >= 6


def test_zero_width_box_is_the_point_value(tiny, c500):
    for net, fac in (tiny, c500):
        lo, hi = synth.full_box(net)
        x = (0.3 * lo + 0.7 * hi).astype(np.float32)
        fx = oracle.point_eval(net, x.astype(float), fac["ctg"])
        assert oracle.crown_upper(net, x, x, fac)["f_hi"] == pytest.approx(fx, rel=1e-9, abs=1e-9)


def test_sampled_points_below_the_bound(c500):
    net, fac = c500
    rng = np.random.default_rng(4)
    blo, bhi = synth.sub_boxes(net, 3, seed=9)
    for a, b in zip(blo, bhi):
        c = oracle.crown_upper(net, a, b, fac)["f_hi"]
        span = b.astype(float) - a
        pts = a[None, :] + rng.random((48, a.size)) * span[None, :]
        verts = a[None, :] + (rng.random((24, a.size)) < 0.5) * span[None, :]
        fv = oracle.point_eval_many(net, np.vstack([pts, verts]), fac["ctg"])
        assert fv.max() <= c + 1e-9 * abs(c)


def test_with_curves_and_distinct_outage_limits(tiny):
    """Curves (through their interval) and outage limits unlike the base limits:
    still >= the LP with epigraph rows and <= IBP."""
    from tests.test_oracle_pins import _emergency
    net = _emergency(synth.with_pwl_costs(tiny[0], seed=5), 3)
    fac = tiny[1]
    for a, b in zip(*synth.sub_boxes(net, 3, seed=7)):
        lp = _lp_max(net, a.astype(float), b.astype(float), fac)
        c = oracle.crown_upper(net, a, b, fac)["f_hi"]
        assert lp - 1e-7 * max(1.0, abs(lp)) <= c <= oracle.ibp(net, a, b, fac)["f_hi"] + 1e-9 * abs(c)


def test_planted_mistakes_are_caught(tiny, monkeypatch):
    """A wrong slope on the negative side is caught by the affine-box exactness pin;
    a dropped intercept by the LP pin."""
    net, fac = tiny
    a, b = next((a, b) for a, b in _tiny_boxes(net, 8, seed=11, delta=1e-6)
                if oracle.crown_upper(net, a, b, fac)["near"] == 0)
    fmax = oracle.point_eval_many(net, _vertices(a, b), fac["ctg"]).max()
    real = oracle.ibp_oracle._crown_slopes

    def unsigned(c, r, t, near_rel):
        s, k = real(c, r, t, near_rel)
        return np.abs(s), k

    monkeypatch.setattr(oracle.ibp_oracle, "_crown_slopes", unsigned)
    assert oracle.crown_upper(net, a, b, fac)["f_hi"] != pytest.approx(fmax, rel=1e-9)
    monkeypatch.setattr(oracle.ibp_oracle, "_crown_slopes", real)

    below = 0
    for x, y in zip(*synth.sub_boxes(net, 6, seed=3)):
        lp = _lp_max(net, x.astype(float), y.astype(float), fac)
        r = oracle.crown_upper(net, x, y, fac)
        below += r["f_hi"] - r["const"] < lp - 1e-6 * abs(lp)   # intercepts zeta_f sum |s| t dropped
    assert below >= 1


def test_point_gradient_slopes_are_valid_anywhere(tiny):
    """Slopes taken at any reference point, inside the box or not, still give a
    bound >= the LP; at a zero-width box and its own point the bound is f(x)."""
    net, fac = tiny
    rng = np.random.default_rng(21)
    lo, hi = synth.full_box(net)
    span = hi.astype(float) - lo
    for a, b in zip(*synth.sub_boxes(net, 3, seed=3)):
        lp = _lp_max(net, a.astype(float), b.astype(float), fac)
        for _ in range(4):
            ref = lo - 0.2 * span + 1.4 * rng.random(lo.size) * span
            c = oracle.crown_upper(net, a, b, fac, ref=ref)["f_hi"]
            assert c >= lp - 1e-7 * max(1.0, abs(lp))
    x = (0.3 * lo + 0.7 * hi).astype(np.float32)
    fx = oracle.point_eval(net, x.astype(float), fac["ctg"])
    assert oracle.crown_upper(net, x, x, fac, ref=x.astype(float))["f_hi"] == pytest.approx(fx, rel=1e-9)


def test_iterated_point_slopes_reach_the_lp_optimum(tiny):
    """The iterated rule (interval slopes, then point-gradient slopes at points
    moving halfway to each relaxation's maximising vertex) attains the LP optimum
    of Problem 1 on several sub-boxes (an independent solver), is never below
    it, and never above the interval rule alone."""
    net, fac = tiny
    reached = 0
    for a, b in zip(*synth.sub_boxes(net, 6, seed=3)):
        lp = _lp_max(net, a.astype(float), b.astype(float), fac)
        r = oracle.crown_upper_iterated(net, a, b, fac, iters=8)
        assert r["f_hi"] >= lp - 1e-7 * max(1.0, abs(lp))
        assert r["f_hi"] <= r["bounds"][0]
        reached += abs(min(r["bounds"][1:]) - lp) <= 1e-7 * max(1.0, abs(lp))   # point rules alone
    assert reached >= 3


def test_planted_point_slope_mistake_is_caught(tiny, monkeypatch):
    """Point slopes with the wrong sign stay valid but no longer reach the LP."""
    net, fac = tiny
    real = oracle.ibp_oracle._crown_point_slopes
    monkeypatch.setattr(oracle.ibp_oracle, "_crown_point_slopes",
                        lambda z, t, n: (-real(z, t, n)[0], real(z, t, n)[1]))
    reached = 0
    for a, b in zip(*synth.sub_boxes(net, 6, seed=3)):
        lp = _lp_max(net, a.astype(float), b.astype(float), fac)
        r = oracle.crown_upper_iterated(net, a, b, fac, iters=8)
        reached += abs(min(r["bounds"][1:]) - lp) <= 1e-7 * max(1.0, abs(lp))
    assert reached == 0
