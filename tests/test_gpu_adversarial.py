"""Adversarial enclosure cases: where the padding model is most likely to fail.

The penalties max(|z| - t, 0) of Sec. III-A eqs. (slack-sfb), (slack-Sc) have
kinks at |z| = t and at z = 0; the imbalance |sum p_inj| has its kink where the
injections cancel.  Each case runs the single-box, box-tiled and one-sided
forward calls and asserts enclosure of the FP64 oracle with no slack and each
gap within the box's error budget:

* limits placed exactly on a kink: every line's outage limit (or base limit)
  set to one element's |C| - R or |C| + R as the oracle computes it, as the
  float64 value and rounded down and up to float32;
* boxes whose injections cancel exactly (sum of injection centres 0), with
  and without width, and a zero-width box at the cancelling point;
* limits of 1e-6, which make nearly every element active;
* an outage whose 1 - H_cc is near the 1e-6 guard (a strong line with a weak
  parallel path), and one below the guard, which is refused.
"""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_forward import assert_encloses, gpu_bounds, one_sided_close, orc, register

pytestmark = pytest.mark.gpu


def _all_paths(n, net, fac, LO, HI, what):
    """Box-tiled (>= 4 boxes), per-box and both one-sided calls enclose the oracle."""
    refs = [orc(net, LO[b], HI[b], fac) for b in range(LO.shape[0])]
    f_lo, f_hi = gpu_bounds(n, LO, HI)
    p_lo, p_hi = gpu_bounds(n, LO, HI, flags=ibp.IBP_F_PLAIN)
    u_lo, u_hi = gpu_bounds(n, LO, HI, flags=ibp.IBP_F_UPPER_ONLY)
    l_lo, l_hi = gpu_bounds(n, LO, HI, flags=ibp.IBP_F_LOWER_ONLY)
    assert one_sided_close(u_hi, f_hi) and one_sided_close(l_lo, f_lo)
    for b, r in enumerate(refs):
        assert_encloses(f_lo[b], f_hi[b], r, what=f"{what} box-tiled box {b}")
        assert u_hi[b] >= r["f_hi"] and l_lo[b] <= r["f_lo"], f"{what} one-sided box {b}"
        assert_encloses(p_lo[b], p_hi[b], r, what=f"{what} per-box box {b}")
        assert l_hi[b] >= r["f_hi"], f"{what} lower-only call's f_hi {l_hi[b]!r} < oracle {r['f_hi']!r}"
        s_lo, s_hi = gpu_bounds(n, LO[b], HI[b])                       # single box alone
        assert s_lo[0] == p_lo[b] and s_hi[0] == p_hi[b]
    return refs


def _elements(net, fac, lo, hi):
    """The oracle's post-outage centre/radius C, R (K x L), outaged entries NaN."""
    r = oracle.ibp(net, lo, hi, fac, keep_intermediates=True)
    Lam = oracle.lodf(net, fac).T                                     # K x L
    ctg = fac["ctg"]
    c_f, r_f = r["c_f"], r["r_f"]
    C = c_f[None, :] + Lam * c_f[ctg][:, None]
    R = r_f[None, :] + np.abs(Lam) * r_f[ctg][:, None]
    C[np.arange(ctg.size), ctg] = np.nan
    R[np.arange(ctg.size), ctg] = np.nan
    return C, R, c_f, r_f


def _boxes(net, seed):
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 5, seed=seed)
    return np.vstack([lo[None], blo]), np.vstack([hi[None], bhi])


@pytest.mark.parametrize("edge", ["lower", "upper"])
@pytest.mark.parametrize("rounding", ["f64", "down", "up"])
def test_outage_limits_on_a_kink(edge, rounding):
    """Every line's outage limit equals one element's |C| - R (lower penalty's
    kink, f_hi side) or |C| + R (upper penalty's kink, f_lo side) on box 1."""
    base = synth.make_config("c500")
    fac = oracle.factors(base)
    LO, HI = _boxes(base, seed=61)
    C, R, _, _ = _elements(base, fac, LO[1], HI[1])
    t = np.abs(C) - R if edge == "lower" else np.abs(C) + R
    # per line, the element whose value is the median of the positive ones
    fc = np.array(base["fmax_ctg"], float)
    for l in range(t.shape[1]):
        col = t[:, l]
        col = col[np.isfinite(col) & (col > 1e-3)]
        if col.size:
            fc[l] = np.sort(col)[col.size // 2]
    if rounding == "down":
        fc = synth.round_down_f32(fc).astype(np.float64)
    elif rounding == "up":
        fc = synth.round_up_f32(fc).astype(np.float64)
    net = dict(base, fmax_ctg=fc)
    n = ibp.Network(net, device=0)
    register(fac, n)
    refs = _all_paths(n, net, fac, LO, HI, f"ctg limits on {edge} kinks ({rounding})")
    assert refs[1]["Fc_lo" if edge == "lower" else "Fc_hi"] > 0.0


@pytest.mark.parametrize("edge", ["lower", "upper"])
def test_base_limits_on_a_kink(edge):
    """Every line's base limit equals its base-flow interval's mignitude
    (|c_f| - r_f) or magnitude (|c_f| + r_f) on box 2."""
    base = synth.make_config("c500")
    fac = oracle.factors(base)
    LO, HI = _boxes(base, seed=62)
    _, _, c_f, r_f = _elements(base, fac, LO[2], HI[2])
    t = np.abs(c_f) - r_f if edge == "lower" else np.abs(c_f) + r_f
    fb = np.where(t > 1e-3, t, np.asarray(base["fmax_base"], float))
    net = dict(base, fmax_base=fb)
    n = ibp.Network(net, device=0)
    register(fac, n)
    _all_paths(n, net, fac, LO, HI, f"base limits on {edge} kinks")


def _cancelling(net, lo, hi):
    """The box moved so that the injection centres cancel exactly: every
    endpoint on the 2^-10 grid, then the first generator's interval shifted so
    that sum gen centres = sum load centres (a multiple of 2^-11, exact in
    float32 and float64)."""
    G = np.asarray(net["gen_bus"]).size
    q = 2.0 ** -10
    a = np.floor(np.asarray(lo, float) / q) * q
    b = np.ceil(np.asarray(hi, float) / q) * q
    c = 0.5 * (a + b)
    target = np.sum(c[G:]) - np.sum(c[1:G])
    w = 0.5 * (b[0] - a[0])
    a[0], b[0] = target - w, target + w
    out_lo, out_hi = a.astype(np.float32), b.astype(np.float32)
    assert np.array_equal(out_lo.astype(float), a) and np.array_equal(out_hi.astype(float), b)
    cc = 0.5 * (out_lo.astype(float) + out_hi.astype(float))
    assert np.sum(cc[:G]) - np.sum(cc[G:]) == 0.0
    return out_lo, out_hi


def test_cancelling_injections():
    net = synth.make_config("c500")
    fac = oracle.factors(net)
    n = ibp.Network(net, device=0)
    register(fac, n)
    LO, HI = _boxes(net, seed=63)
    rows_lo, rows_hi = [], []
    for b in range(LO.shape[0]):
        a, c = _cancelling(net, LO[b], HI[b])
        rows_lo.append(a)
        rows_hi.append(c)
    # a zero-width box at a cancelling point: the imbalance sits exactly on its kink
    m = (0.5 * (rows_lo[1].astype(float) + rows_hi[1].astype(float)))
    G = np.asarray(net["gen_bus"]).size
    p = np.floor(m / 2.0 ** -10) * 2.0 ** -10
    p[0] = np.sum(p[G:]) - np.sum(p[1:G])
    rows_lo.append(p.astype(np.float32))
    rows_hi.append(p.astype(np.float32))
    LO, HI = np.asarray(rows_lo), np.asarray(rows_hi)
    refs = _all_paths(n, net, fac, LO, HI, "cancelling injections")
    assert refs[-1]["I_lo"] == 0.0 and refs[-1]["I_hi"] == 0.0
    assert all(r["I_lo"] == 0.0 for r in refs)


def test_tiny_limits_make_nearly_every_element_active():
    base = synth.make_config("c500")
    L = np.asarray(base["line_from"]).size
    net = dict(base, fmax_base=np.full(L, 1e-6), fmax_ctg=np.full(L, 1e-6))
    fac = oracle.factors(net)
    n = ibp.Network(net, device=0)
    register(fac, n)
    LO, HI = _boxes(net, seed=64)
    refs = _all_paths(n, net, fac, LO, HI, "limits 1e-6")
    C, R, c_f, r_f = _elements(net, fac, LO[1], HI[1])
    frac = np.mean((np.abs(C) + R)[np.isfinite(C)] > 1e-6)
    assert frac > 0.9, frac
    assert refs[1]["Fc_hi"] > 0 and refs[1]["Fb_hi"] > 0


def _near_guard(b_weak):
    """The 14-bus network plus bus 14, tied to bus 3 by a strong line (b = 50)
    and to bus 7 by a weak one (b = b_weak), with a generator and a load on
    it: outaging the strong line leaves the weak path, 1 - H_cc ~ b_weak / 50."""
    net = synth.make_config("tiny")
    net = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in net.items()}
    net["n_bus"] = 15
    net["line_from"] = np.append(net["line_from"], [14, 7]).astype(np.int32)
    net["line_to"] = np.append(net["line_to"], [3, 14]).astype(np.int32)
    net["line_b"] = np.append(net["line_b"], [50.0, b_weak])
    net["fmax_base"] = np.append(net["fmax_base"], [1.0, 0.8])
    net["fmax_ctg"] = np.append(net["fmax_ctg"], [1.0, 0.8])
    net["gen_bus"] = np.append(net["gen_bus"], 14).astype(np.int32)
    net["gen_cost"] = np.append(net["gen_cost"], 20.0)
    net["gen_pmin"] = np.append(net["gen_pmin"], 0.0)
    net["gen_pmax"] = np.append(net["gen_pmax"], 2.0)
    net["load_bus"] = np.append(net["load_bus"], 14).astype(np.int32)
    net["load_value"] = np.append(net["load_value"], 90.0)
    net["load_dmin"] = np.append(net["load_dmin"], 0.3)
    net["load_dmax"] = np.append(net["load_dmax"], 0.5)
    net["ctg_line"] = None
    return net


def test_outage_near_the_conditioning_guard():
    net = _near_guard(2e-4)
    fac = oracle.factors(net)
    n = ibp.Network(net, device=0)
    register(fac, n)
    assert 1e-6 < n.info.min_one_minus_hcc < 1e-4, n.info.min_one_minus_hcc
    L = np.asarray(net["line_from"]).size
    assert L - 2 in set(fac["ctg"].tolist())
    LO, HI = _boxes(net, seed=65)
    _all_paths(n, net, fac, LO, HI, "outage near the guard")
    with pytest.raises(ibp.IBPError) as e:
        ibp.Network(_near_guard(1e-5), device=0)
    assert e.value.name == "IBP_E_ILL_CONDITIONED"
