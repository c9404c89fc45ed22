"""GPU parity with piecewise-linear cost and value curves (Sec. III-B): forward
bounds enclose the FP64 oracle's within 1e-5 (per-box and box-tiled forms),
the surplus alone is exact to float64 rounding, and the backward matches the
oracle's gradient."""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_backward import gpu_grad, rel_l2
from tests.test_gpu_forward import assert_encloses, assert_terms_enclose, gpu_bounds, orc, register

pytestmark = pytest.mark.gpu

_cache = {}


def setup_pwl(name, seed):
    if name not in _cache:
        net = synth.with_pwl_costs(synth.make_config(name), seed=seed)
        print(f"[setup] {name} with curves", flush=True)
        _cache[name] = (net, oracle.factors(net), ibp.Network(net, device=0))
        register(_cache[name][1], _cache[name][2])
    return _cache[name]


def test_tiny_curves_full_sub_and_point_boxes():
    net, fac, n = setup_pwl("tiny", 5)
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 8, seed=3)
    rng = np.random.default_rng(4)
    pts = (lo + rng.random((3, lo.size)) * (hi.astype(float) - lo)).astype(np.float32)
    LO = np.vstack([lo[None], blo, pts])
    HI = np.vstack([hi[None], bhi, pts])
    for flags in (0, ibp.IBP_F_PLAIN):
        f_lo, f_hi, t = gpu_bounds(n, LO, HI, terms=True, flags=flags)
        for b in range(LO.shape[0]):
            r = orc(net, LO[b], HI[b], fac)
            assert_encloses(f_lo[b], f_hi[b], r, what=f"box {b} flags {flags}")
            assert_terms_enclose(t[b], r)


def test_c500_curves_full_box_and_sub_boxes():
    net, fac, n = setup_pwl("c500", 6)
    lo, hi = synth.full_box(net)
    r = orc(net, lo, hi, fac)
    f_lo, f_hi = gpu_bounds(n, lo, hi)
    assert_encloses(f_lo[0], f_hi[0], r, what="full box", strict_f=True)
    blo, bhi = synth.sub_boxes(net, 6, seed=8)
    f_lo, f_hi = gpu_bounds(n, blo, bhi)
    for b in range(6):
        assert_encloses(f_lo[b], f_hi[b], orc(net, blo[b], bhi[b], fac), what=f"box {b}")


def test_c2000_curves_period_boxes_subset():
    net, fac, n = setup_pwl("c2000", 7)
    lo, hi, _ = synth.period_boxes(net, 2, 4, seed=31)
    f_lo, f_hi = gpu_bounds(n, lo, hi)
    for b in (0, 5):
        assert_encloses(f_lo[b], f_hi[b], orc(net, lo[b], hi[b], fac), what=f"box {b}")


def test_curves_alone_give_the_surplus_interval():
    """With zero penalty weights f is the surplus: [sum F*(lo_d) - sum F*(hi_g),
    sum F*(hi_d) - sum F*(lo_g)] for monotone curves, exact up to float64 rounding."""
    net = dict(synth.with_pwl_costs(synth.make_config("c500"), seed=6), zeta_inj=0.0, zeta_f=0.0)
    n = ibp.Network(net, device=0)
    blo, bhi = synth.sub_boxes(net, 5, seed=1)
    f_lo, f_hi = gpu_bounds(n, blo, bhi)
    fac = oracle.factors(net)
    for b in range(5):
        r = oracle.ibp(net, blo[b], bhi[b], fac)
        assert f_lo[b] <= r["f_lo"] and f_hi[b] >= r["f_hi"]
        assert r["f_lo"] - f_lo[b] <= 1e-12 * abs(r["f_lo"]) + 1e-9
        assert f_hi[b] - r["f_hi"] <= 1e-12 * abs(r["f_hi"]) + 1e-9


@pytest.mark.parametrize("name,seed", [("tiny", 5), ("c500", 6)])
def test_curves_gradient_matches_oracle(name, seed):
    """Whole objective: relative L2 <= 1e-4 as for linear costs.  Surplus alone
    (zero weights): the curve derivatives take the same float64 kink decisions
    as the oracle (the full box puts lo exactly on the first kink of every
    generator curve), so they agree to 1e-12."""
    net, fac, n = setup_pwl(name, seed)
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 5, seed=12)
    LO = np.vstack([lo[None], blo])
    HI = np.vstack([hi[None], bhi])
    gl, gh = np.full(6, 0.3), np.full(6, -0.7)
    for flags in (0, ibp.IBP_F_PLAIN):
        d_lo, d_hi = gpu_grad(n, LO, HI, gl, gh, flags=flags)
        for b in range(6):
            o_lo, o_hi, near = oracle.grad(net, LO[b], HI[b], 0.3, -0.7, fac)
            err = rel_l2(np.concatenate([d_lo[b], d_hi[b]]), np.concatenate([o_lo, o_hi]))
            print(f"[{name}] box {b} flags {flags}: rel L2 {err:.2e}, near-kink elements {near}", flush=True)
            assert err <= 1e-4, (b, flags, err, near)
    z = dict(net, zeta_inj=0.0, zeta_f=0.0)
    nz = ibp.Network(z, device=0)
    d_lo, d_hi = gpu_grad(nz, LO, HI, gl, gh)
    for b in range(6):
        o_lo, o_hi, _ = oracle.grad(z, LO[b], HI[b], 0.3, -0.7, fac)
        np.testing.assert_allclose(d_lo[b], o_lo, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(d_hi[b], o_hi, rtol=1e-12, atol=1e-12)
