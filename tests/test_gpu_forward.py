"""GPU parity of the forward bounds against the FP64 oracle (through the C ABI).

Bar, per box and side:
  * enclosure with no slack: gpu_lo <= oracle_lo and gpu_hi >= oracle_hi;
  * the gap is at most the box's error budget (tests/error_budget.py): the
    sum of the pads the float32 padding rules put on every element and line
    whose penalty can be positive, derived from the magnitudes each pad covers
    (about 4 u of them, u = 2^-24).  Measured gaps sit at about half their
    budget, so a padding rule that doubled would fail this bar;
  * on the whole boxes of the headline workloads (``strict_f``), the gap is
    also within 1e-5 of max(|oracle|, 1 $).
On sub-boxes whose terms cancel to a small |f| the budget can exceed 1e-5 of
|f| (the objective is a difference of terms much larger than itself); bench.py
reports how often that happens on the batched workloads.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import ibp, synth
from tests.error_budget import budget

pytestmark = pytest.mark.gpu
TOL = 1e-5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _torch():
    import torch
    return torch


def gpu_bounds(net_obj, lo, hi, terms=False, flags=0):
    torch = _torch()
    tlo = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(lo), np.float32)).cuda()
    thi = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(hi), np.float32)).cuda()
    out = ibp.ibp_bound_boxes(net_obj, tlo, thi, terms=terms, flags=flags)
    torch.cuda.synchronize()
    return tuple(o.cpu().numpy() for o in out)


def term_scale(r, side):
    """Magnitude of the objective's terms on one side: |S| + zeta_inj I + zeta_f (Fb + Fc).

    f is a difference of these terms; float32 arithmetic cannot resolve f more
    finely than a small multiple of u times this scale (equal to |f| when no
    cancellation occurs)."""
    net = r["_net"]
    if side == "hi":
        return abs(r["S_hi"]) + net["zeta_inj"] * r["I_lo"] + net["zeta_f"] * (r["Fb_lo"] + r["Fc_lo"])
    return abs(r["S_lo"]) + net["zeta_inj"] * r["I_hi"] + net["zeta_f"] * (r["Fb_hi"] + r["Fc_hi"])


# phi_abs_err of the device network each oracle factor set belongs to
_PHI_ERR = {}


def register(fac, n):
    """Records the library network's PTDF error bound for the budget of boxes
    evaluated with these oracle factors."""
    _PHI_ERR[id(fac)] = (fac, float(n.info.phi_abs_err))


def assert_encloses(g_lo, g_hi, r, tol=TOL, what="", strict_f=False):
    """Enclosure with no slack, and each side's gap within the box's error
    budget; strict_f: also within tol relative to max(|f|, 1)."""
    o_lo, o_hi = r["f_lo"], r["f_hi"]
    assert g_lo <= o_lo, f"{what} lower bound not enclosing: gpu {g_lo!r} > oracle {o_lo!r}"
    assert g_hi >= o_hi, f"{what} upper bound not enclosing: gpu {g_hi!r} < oracle {o_hi!r}"
    bu = r["_budget"]
    assert o_lo - g_lo <= bu["lo"], f"{what} lo gap {o_lo - g_lo!r} above its budget {bu['lo']!r}"
    assert g_hi - o_hi <= bu["hi"], f"{what} hi gap {g_hi - o_hi!r} above its budget {bu['hi']!r}"
    if strict_f:
        assert (o_lo - g_lo) / max(abs(o_lo), 1.0) <= tol, f"{what} lo gap {o_lo - g_lo!r} (oracle {o_lo!r})"
        assert (g_hi - o_hi) / max(abs(o_hi), 1.0) <= tol, f"{what} hi gap {g_hi - o_hi!r} (oracle {o_hi!r})"


def orc_plain(net, lo, hi, fac):
    """The oracle's bounds of one box (no error budget)."""
    r = oracle.ibp(net, lo, hi, fac)
    r["_net"] = net
    return r


def orc(net, lo, hi, fac):
    """The oracle's bounds of one box with its error budget attached (the
    factors must belong to a network passed to register() or setup())."""
    assert id(fac) in _PHI_ERR, "register(fac, network) first"
    bu = budget(net, fac, lo, hi, _PHI_ERR[id(fac)][1])
    r = bu.pop("r")
    r["_net"] = net
    r["_budget"] = bu
    return r


def assert_terms_enclose(t, r):
    for i, key in enumerate(("S", "I", "Fb", "Fc")):
        assert t[2 * i] <= r[f"{key}_lo"] + 0.0, key
        assert t[2 * i + 1] >= r[f"{key}_hi"] - 0.0, key


_cache = {}


def setup(name):
    if name not in _cache:
        net = synth.make_config(name)
        print(f"[setup] {name}: building oracle factors and device network", flush=True)
        _cache[name] = (net, oracle.factors(net), ibp.Network(net, device=0))
        register(_cache[name][1], _cache[name][2])
    return _cache[name]


def test_three_bus_hand_derived_enclosed():
    with open(os.path.join(GOLDEN, "three_bus.json")) as f:
        g = json.load(f)
    net = {k: (np.asarray(v) if isinstance(v, list) else v) for k, v in g["network"].items()}
    net["ctg_line"] = None
    n = ibp.Network(net, device=0)
    lo = np.asarray(g["box_lo"], np.float32)
    hi = np.asarray(g["box_hi"], np.float32)
    f_lo, f_hi = gpu_bounds(n, lo, hi)
    assert f_lo[0] <= -181.0 and f_hi[0] >= 43.0
    assert abs(f_lo[0] + 181.0) <= 181.0 * 1e-6 and abs(f_hi[0] - 43.0) <= 43.0 * 1e-6


def test_tiny_full_sub_and_point_boxes():
    net, fac, n = setup("tiny")
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 16, seed=101)
    rng = np.random.default_rng(5)
    pts = (lo + rng.random((4, lo.size)) * (hi.astype(float) - lo)).astype(np.float32)
    LO = np.vstack([lo[None], blo, pts])
    HI = np.vstack([hi[None], bhi, pts])
    f_lo, f_hi, terms = gpu_bounds(n, LO, HI, terms=True)
    for b in range(LO.shape[0]):
        r = orc(net, LO[b], HI[b], fac)
        assert_encloses(f_lo[b], f_hi[b], r, what=f"box {b}")
        assert_terms_enclose(terms[b], r)


def test_c500_full_box_and_sub_boxes():
    net, fac, n = setup("c500")
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 6, seed=202)
    LO = np.vstack([lo[None], blo])
    HI = np.vstack([hi[None], bhi])
    f_lo, f_hi = gpu_bounds(n, LO, HI)
    for b in range(LO.shape[0]):
        assert_encloses(f_lo[b], f_hi[b], orc(net, LO[b], HI[b], fac), what=f"box {b}", strict_f=(b == 0))


def test_batch_is_independent_and_deterministic():
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 9, seed=7)
    # the batched (box-tiled) call is bitwise reproducible
    a_lo, a_hi = gpu_bounds(n, blo, bhi)
    b_lo, b_hi = gpu_bounds(n, blo, bhi)
    assert np.array_equal(a_lo, b_lo) and np.array_equal(a_hi, b_hi)
    # per-box kernels on a batch give each box exactly its single-box result
    p_lo, p_hi = gpu_bounds(n, blo, bhi, flags=ibp.IBP_F_PLAIN)
    for b in (0, 4, 8):
        s_lo, s_hi = gpu_bounds(n, blo[b], bhi[b])
        assert s_lo[0] == p_lo[b] and s_hi[0] == p_hi[b]
        r = orc(net, blo[b], bhi[b], fac)
        assert_encloses(a_lo[b], a_hi[b], r, what=f"batched box {b}")


def test_bad_boxes_poison_only_themselves():
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 4, seed=3)
    blo, bhi = blo.copy(), bhi.copy()
    blo[1, 2] = np.nan
    blo[2, 0], bhi[2, 0] = bhi[2, 0] + 1.0, blo[2, 0]      # lo > hi
    f_lo, f_hi = gpu_bounds(n, blo, bhi)
    assert np.isnan(f_lo[1]) and np.isnan(f_hi[1]) and np.isnan(f_lo[2]) and np.isnan(f_hi[2])
    for b in (0, 3):
        assert_encloses(f_lo[b], f_hi[b], orc(net, blo[b], bhi[b], fac))


def test_workspace_and_argument_errors():
    torch = _torch()
    net, fac, n = setup("tiny")
    lib = ibp.load_library()
    lo, hi = synth.full_box(net)
    tlo = torch.from_numpy(lo[None]).cuda()
    thi = torch.from_numpy(hi[None]).cuda()
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    need = n.workspace_bytes(1)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    import ctypes
    vp = ctypes.c_void_p
    st = lib.ibp_bound_boxes(n.handle, 1, vp(tlo.data_ptr()), vp(thi.data_ptr()), vp(out.data_ptr()),
                             vp(out.data_ptr() + 8), None, vp(ws.data_ptr()), need - 1, None, 0)
    assert ibp.STATUS[st] == "IBP_E_WORKSPACE"
    st = lib.ibp_bound_boxes(n.handle, 1, None, vp(thi.data_ptr()), vp(out.data_ptr()),
                             vp(out.data_ptr() + 8), None, vp(ws.data_ptr()), need, None, 0)
    assert ibp.STATUS[st] == "IBP_E_INVALID_ARG"
    st = lib.ibp_bound_boxes(n.handle, 0, None, None, None, None, None, None, 0, None, 0)
    assert st == 0
    st = lib.ibp_bound_boxes(n.handle, 1, vp(tlo.data_ptr()), vp(thi.data_ptr()), vp(out.data_ptr()),
                             vp(out.data_ptr() + 8), None, vp(ws.data_ptr()), need, None, 1 << 30)
    assert ibp.STATUS[st] == "IBP_E_INVALID_ARG"  # an undefined flag bit
    st = lib.ibp_bound_boxes(n.handle, 1, vp(tlo.data_ptr()), vp(thi.data_ptr()), vp(out.data_ptr()),
                             vp(out.data_ptr() + 8), None, vp(ws.data_ptr()), need, None,
                             ibp.IBP_F_SCREEN_UPPER | ibp.IBP_F_UPPER_ONLY)
    assert ibp.STATUS[st] == "IBP_E_INVALID_ARG"  # only for calls that bound f_lo


def test_device_factors_match_oracle():
    net, fac, n = setup("c500")
    ptdf, lodf = n.export()
    np.testing.assert_allclose(ptdf, fac["Phi"], atol=1e-11, rtol=0)


def test_c2000_period_boxes_subset():
    net, fac, n = setup("c2000")
    lo, hi, per = synth.period_boxes(net, 18, 4, seed=31)
    pick = np.array([0, 13, 27, 40, 55, 71])
    f_lo, f_hi = gpu_bounds(n, lo[pick], hi[pick])
    for i, b in enumerate(pick):
        assert_encloses(f_lo[i], f_hi[i], orc(net, lo[b], hi[b], fac), what=f"box {b}")


def test_c8316_single_full_box():
    """The large single-box workload at full size: 8316 buses, 14000 lines, 8000 outages."""
    net, fac, n = setup("c8316")
    lo, hi = synth.full_box(net)
    f_lo, f_hi = gpu_bounds(n, lo, hi)
    r = orc(net, lo, hi, fac)
    print(f"[c8316] gpu [{f_lo[0]!r}, {f_hi[0]!r}] oracle [{r['f_lo']!r}, {r['f_hi']!r}]", flush=True)
    assert_encloses(f_lo[0], f_hi[0], r, what="c8316 full box", strict_f=True)
    blo, bhi = synth.sub_boxes(net, 1, seed=41)
    f_lo, f_hi = gpu_bounds(n, blo, bhi)
    assert_encloses(f_lo[0], f_hi[0], orc(net, blo[0], bhi[0], fac), what="c8316 sub-box")


def test_radial_network_without_outages_and_empty_batch():
    """A tree has no non-islanding outage (K = 0): only base flows and imbalance."""
    torch = _torch()
    net = synth.make_network(30, 29, 6, 12, seed=8)
    fac = oracle.factors(net)
    assert fac["K"] == 0
    n = ibp.Network(net, device=0)
    register(fac, n)
    assert n.n_ctg == 0
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 6, seed=2)
    LO = np.vstack([lo[None], blo])
    HI = np.vstack([hi[None], bhi])
    for flags in (0, ibp.IBP_F_PLAIN):
        f_lo, f_hi = gpu_bounds(n, LO, HI, flags=flags)
        for b in range(LO.shape[0]):
            assert_encloses(f_lo[b], f_hi[b], orc(net, LO[b], HI[b], fac), what=f"box {b}")
    e = torch.empty((0, n.n_input), dtype=torch.float32, device="cuda")
    a, b = ibp.ibp_bound_boxes(n, e, e)
    assert a.numel() == 0 and b.numel() == 0


def test_huge_limits_and_zero_penalties():
    """Limits far above every flow leave the surplus and imbalance terms only;
    zero weights leave the surplus interval exactly (special cases of the objective)."""
    net = synth.make_config("c500")
    big = dict(net, fmax_base=np.full(700, 1e30), fmax_ctg=np.full(700, 1e30))
    n = ibp.Network(big, device=0)
    blo, bhi = synth.sub_boxes(net, 4, seed=6)
    f_lo, f_hi, t = gpu_bounds(n, blo, bhi, terms=True)
    assert np.all(t[:, 4:] == 0.0)
    fac = oracle.factors(big)
    register(fac, n)
    for b in range(4):
        assert_encloses(f_lo[b], f_hi[b], orc(big, blo[b], bhi[b], fac), what=f"box {b}")
    z = dict(net, zeta_inj=0.0, zeta_f=0.0)
    n = ibp.Network(z, device=0)
    f_lo, f_hi = gpu_bounds(n, blo, bhi)
    G = net["gen_bus"].size
    for b in range(4):
        S_hi = np.sum(net["load_value"] * bhi[b, G:].astype(float)) - np.sum(net["gen_cost"] * blo[b, :G].astype(float))
        S_lo = np.sum(net["load_value"] * blo[b, G:].astype(float)) - np.sum(net["gen_cost"] * bhi[b, :G].astype(float))
        assert f_lo[b] <= S_lo and f_hi[b] >= S_hi
        assert abs(f_lo[b] - S_lo) <= 1e-12 * abs(S_lo) + 1e-9 and abs(f_hi[b] - S_hi) <= 1e-12 * abs(S_hi) + 1e-9


def test_tile_choices_give_enclosing_bounds():
    """Every tile pair of the single-box kernels (and the autotuner's pick) encloses the oracle."""
    torch = _torch()
    net, fac, n = setup("c500")
    lo, hi = synth.full_box(net)
    r = orc(net, lo, hi, fac)
    for nc in (32, 64, 128, 256, 512):
        for kc in (16, 32, 64, 128):
            n.set_tile(nc, kc)
            f_lo, f_hi = gpu_bounds(n, lo, hi)
            assert_encloses(f_lo[0], f_hi[0], r, what=f"tile {nc},{kc}", strict_f=True)
    tl = torch.from_numpy(lo[None].copy()).cuda()
    th = torch.from_numpy(hi[None].copy()).cuda()
    nc, kc = ibp.ibp_autotune(n, tl, th)
    assert nc in (32, 64, 128, 256, 512) and kc in (16, 32, 64, 128)
    f_lo, f_hi = gpu_bounds(n, lo, hi)
    assert_encloses(f_lo[0], f_hi[0], r, what="autotuned", strict_f=True)


def test_distinct_contingency_limits():
    """Post-outage limits different from the base limits (per-line factors in
    [0.5, 1.5]): single-box, box-tiled and plain forms all enclose the oracle."""
    from tests.test_oracle_pins import _emergency
    net = _emergency(synth.make_config("c500"), 4)
    fac = oracle.factors(net)
    n = ibp.Network(net, device=0)
    register(fac, n)
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 7, seed=31)
    r = orc(net, lo, hi, fac)
    f_lo, f_hi, t = gpu_bounds(n, lo, hi, terms=True)
    assert_encloses(f_lo[0], f_hi[0], r, what="full box", strict_f=True)
    assert_terms_enclose(t[0], r)
    refs = [orc(net, blo[b], bhi[b], fac) for b in range(7)]
    for flags in (0, ibp.IBP_F_PLAIN):
        f_lo, f_hi, t = gpu_bounds(n, blo, bhi, terms=True, flags=flags)
        for b in range(7):
            assert_encloses(f_lo[b], f_hi[b], refs[b], what=f"box {b} flags {flags}")
            assert_terms_enclose(t[b], refs[b])


def one_sided_close(a, b, rtol=1e-6):
    """A box-tiled one-sided bound against the two-sided call's: the screened
    sweep adds the same outage penalties in another float32 order."""
    return bool(np.all(np.abs(a - b) <= rtol * np.maximum(np.abs(b), 1.0)))


@pytest.mark.parametrize("n_box", [1, 37])
def test_one_sided_calls(n_box):
    """IBP_F_UPPER_ONLY / IBP_F_LOWER_ONLY return the requested bound (bit for
    bit on the per-box path and for IBP_F_LOWER_ONLY alone; on the box-tiled
    path IBP_F_UPPER_ONLY, and IBP_F_LOWER_ONLY with IBP_F_SCREEN_UPPER, take
    the screened sweep, which sums the same outage penalties in another
    float32 order: 1e-6 relative) and a trivially valid other side."""
    torch = _torch()
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, n_box, seed=404)
    f_lo, f_hi, t = gpu_bounds(n, blo, bhi, terms=True)
    u_lo, u_hi, tu = gpu_bounds(n, blo, bhi, terms=True, flags=ibp.IBP_F_UPPER_ONLY)
    l_lo, l_hi, tl = gpu_bounds(n, blo, bhi, terms=True, flags=ibp.IBP_F_LOWER_ONLY)
    same = np.array_equal if n_box < 4 else one_sided_close
    assert same(u_hi, f_hi) and np.all(u_lo == -np.inf) and np.all(tu[:, 7] == np.inf)
    assert np.array_equal(l_lo, f_lo) and np.all(tl[:, 6] == 0.0)
    s_lo, _ = gpu_bounds(n, blo, bhi, flags=ibp.IBP_F_LOWER_ONLY | ibp.IBP_F_SCREEN_UPPER)
    assert same(s_lo, f_lo)
    assert np.all(l_hi >= f_hi)
    for b in (0, n_box - 1):
        r = orc(net, blo[b], bhi[b], fac)
        assert u_hi[b] >= r["f_hi"] and l_lo[b] <= r["f_lo"]
        # without the outage penalties' lower bound the upper bound still holds
        assert l_hi[b] >= r["f_hi"]
    tlo = torch.from_numpy(blo).cuda()
    thi = torch.from_numpy(bhi).cuda()
    with pytest.raises(ibp.IBPError):
        ibp.ibp_bound_boxes(n, tlo, thi, flags=ibp.IBP_F_UPPER_ONLY | ibp.IBP_F_LOWER_ONLY)
    c_lo, c_hi = ibp.ibp_crown_bound_boxes(n, tlo, thi)
    cu_lo, cu_hi = ibp.ibp_crown_bound_boxes(n, tlo, thi, flags=ibp.IBP_F_UPPER_ONLY)
    torch.cuda.synchronize()
    assert same(c_hi.cpu().numpy(), cu_hi.cpu().numpy()) and bool(torch.all(cu_lo == -float("inf")))


def test_read_probe_sums_what_it_streams():
    torch = _torch()
    x = torch.ones((1 << 20) + 12, dtype=torch.float32, device="cuda")   # ragged against the grid stride
    part = torch.empty(ibp_partials := 2048, dtype=torch.float32, device="cuda")
    ibp.ibp_read_probe(x, part)
    torch.cuda.synchronize()
    assert part.numel() == ibp_partials and float(part.sum()) == float(x.numel())
    with pytest.raises(ValueError):
        ibp.ibp_read_probe(x, torch.empty(16, dtype=torch.float32, device="cuda"))


def test_alu_probe_reaches_the_chains_fixed_point():
    torch = _torch()
    out = torch.empty(ibp.ALU_PROBE_LANES, dtype=torch.float32, device="cuda")
    for scalar in (False, True):
        out.fill_(0.0)
        ibp.ibp_alu_probe(out, 64, scalar)
        torch.cuda.synchronize()
        assert bool(torch.all(out == 16.0)), scalar
    with pytest.raises(ibp.IBPError):
        ibp.ibp_alu_probe(out, 0)
    with pytest.raises(ValueError):
        ibp.ibp_alu_probe(out[:16], 64)


def test_three_bus_box_tiled_and_relaxation_paths():
    """The hand-derived 3-bus box repeated 5 times takes the box-tiled kernels
    (matrix-core base flows with 3 buses: a partial step of four; relaxation
    products over one 16-line group) and must give the single-box bounds."""
    with open(os.path.join(GOLDEN, "three_bus.json")) as f:
        g = json.load(f)
    net = {k: (np.asarray(v) if isinstance(v, list) else v) for k, v in g["network"].items()}
    net["ctg_line"] = None
    n = ibp.Network(net, device=0)
    lo = np.repeat(np.asarray(g["box_lo"], np.float32)[None], 5, 0)
    hi = np.repeat(np.asarray(g["box_hi"], np.float32)[None], 5, 0)
    f_lo, f_hi = gpu_bounds(n, lo, hi)
    s_lo, s_hi = gpu_bounds(n, lo[:1], hi[:1])
    assert np.all(np.abs(f_lo - s_lo[0]) <= 1e-9 * abs(s_lo[0])) and np.all(np.abs(f_hi - s_hi[0]) <= 1e-9 * abs(s_hi[0]))
    torch = _torch()
    c_lo, c_hi = ibp.ibp_crown_bound_boxes(n, torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda())
    d_lo, d_hi = ibp.ibp_crown_bound_boxes(n, torch.from_numpy(lo[:1]).cuda(), torch.from_numpy(hi[:1]).cuda())
    torch.cuda.synchronize()
    c_hi, d_hi = c_hi.cpu().numpy(), d_hi.cpu().numpy()
    assert np.all(c_hi <= s_hi[0]) and np.all(np.abs(c_hi - d_hi[0]) <= 1e-9 * max(1.0, abs(d_hi[0])))
    rc = oracle.crown_upper(net, lo[0].astype(float), hi[0].astype(float), oracle.factors(net))
    if rc["near"] == 0:
        assert np.all(c_hi >= rc["f_hi"])


@pytest.mark.parametrize("name,nb,seed", [("tiny", 5, 3), ("c500", 37, 5), ("c2000", 70, 7)])
def test_screened_two_sided_forward_matches_the_dense_sweep(monkeypatch, name, nb, seed):
    """IBP_F_SCREEN_UPPER on a two-sided box-tiled call: both penalty sums
    over the lines the upper-penalty screen marks (a line with no active upper
    penalty has no active lower one), each element k3_elem's bit for bit:
    both bounds within 1e-6 relative of the dense sweep's, enclosing the
    oracle."""
    net = synth.make_config(name)
    fac = oracle.factors(net)
    n = ibp.Network(net, device=0)
    blo, bhi = synth.sub_boxes(net, nb, seed=seed)
    s_lo, s_hi = gpu_bounds(n, blo, bhi, flags=ibp.IBP_F_SCREEN_UPPER)
    d_lo, d_hi = gpu_bounds(n, blo, bhi)
    assert one_sided_close(s_lo, d_lo) and one_sided_close(s_hi, d_hi)
    for b in sorted({0, nb // 2, nb - 1}):
        r = orc_plain(net, blo[b], bhi[b], fac)
        assert s_lo[b] <= r["f_lo"] and s_hi[b] >= r["f_hi"], (b, s_lo[b], s_hi[b], r)


@pytest.mark.parametrize("name,nb,seed", [("tiny", 5, 3), ("c500", 37, 5), ("c2000", 70, 7)])
@pytest.mark.parametrize("side", ["upper", "lower"])
def test_screened_one_sided_forward_matches_the_dense_sweep(monkeypatch, name, nb, seed, side):
    """One-sided box-tiled calls (IBP_F_UPPER_ONLY; IBP_F_LOWER_ONLY with
    IBP_F_SCREEN_UPPER) sweep only the lines a screen marks per tile of 4
    boxes (IBP_TILE=k3s=0: every line).  Each element's penalty is the
    dense sweep's, bit for bit, so the bounds differ only by the float32
    summation order of the outage penalties (1e-6 relative; a missed line
    would drop whole penalties); both enclose the oracle.  Box counts ragged
    against the tiles; the boxes' centre points too (the splitting loop's
    lower bounds)."""
    net = synth.make_config(name)
    fac = oracle.factors(net)
    n = ibp.Network(net, device=0)
    monkeypatch.setenv("IBP_TILE", "k3s=0")
    nd = ibp.Network(net, device=0)
    monkeypatch.delenv("IBP_TILE")
    blo, bhi = synth.sub_boxes(net, nb, seed=seed)
    mid = (0.5 * (blo + bhi)).astype(np.float32)
    flag = ibp.IBP_F_UPPER_ONLY if side == "upper" else ibp.IBP_F_LOWER_ONLY | ibp.IBP_F_SCREEN_UPPER
    for lo, hi in ((blo, bhi), (mid, mid)):
        s_lo, s_hi = gpu_bounds(n, lo, hi, flags=flag)
        d_lo, d_hi = gpu_bounds(nd, lo, hi, flags=flag)
        s, d = (s_hi, d_hi) if side == "upper" else (s_lo, d_lo)
        assert one_sided_close(s, d), float(np.max(np.abs(s - d) / np.maximum(np.abs(d), 1.0)))
        for b in sorted({0, nb // 2, nb - 1}):
            r = orc_plain(net, lo[b], hi[b], fac)
            assert (s[b] >= r["f_hi"]) if side == "upper" else (s[b] <= r["f_lo"]), (b, s[b], r)


@pytest.mark.parametrize("limit", [1e-6, 1e30])
def test_screened_one_sided_forward_with_extreme_limits(monkeypatch, limit):
    """Outage limits of 1e-6 (most penalties active) and 1e30 (none): the
    screened one-sided bounds equal the dense sweep's within summation order."""
    net = dict(synth.make_config("c500"))
    net["fmax_ctg"] = np.full(len(net["fmax_ctg"]), limit)
    n = ibp.Network(net, device=0)
    monkeypatch.setenv("IBP_TILE", "k3s=0")
    nd = ibp.Network(net, device=0)
    monkeypatch.delenv("IBP_TILE")
    blo, bhi = synth.sub_boxes(net, 13, seed=9)
    for flag, pick in ((ibp.IBP_F_UPPER_ONLY, 1), (ibp.IBP_F_LOWER_ONLY | ibp.IBP_F_SCREEN_UPPER, 0)):
        s = gpu_bounds(n, blo, bhi, flags=flag)[pick]
        d = gpu_bounds(nd, blo, bhi, flags=flag)[pick]
        assert one_sided_close(s, d), (flag, float(np.max(np.abs(s - d) / np.maximum(np.abs(d), 1.0))))
        if limit == 1e30:
            np.testing.assert_array_equal(s, d)
