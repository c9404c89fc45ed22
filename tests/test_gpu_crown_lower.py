"""GPU parity of the chord-relaxation lower bound against the FP64 oracle,
through the C ABI.

Bar: the GPU bound is certified, so it never exceeds the oracle's relaxation
(whose chords are taken over the oracle's tighter intervals with unrounded
slopes), and it lies within 1e-5 of it relative to max(|f|, term scale, 1 $),
the bar of the IBP bounds.  The returned f_lo is max(IBP f_lo, relaxation
bound) and f_hi is IBP's.  On the 14-bus network the bound is also checked
against the minimum of f over all 2^16 vertices of each box (f is concave with
linear costs).
"""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_forward import gpu_bounds, orc_plain, setup, term_scale
from tests.test_oracle_crown import _vertices

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _torch():
    import torch
    return torch


def gpu_lower(n, lo, hi, flags=0, vertex=False):
    torch = _torch()
    tlo = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(lo), np.float32)).cuda()
    thi = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(hi), np.float32)).cuda()
    v = torch.empty_like(tlo) if vertex else None
    out = ibp.ibp_crown_lower_boxes(n, tlo, thi, crown=True, flags=flags, vertex=v)
    torch.cuda.synchronize()
    out = tuple(o.cpu().numpy() for o in out)
    return out + (v.cpu().numpy(),) if vertex else out


def check_box(net, fac, lo, hi, g_lo, g_hi, g_c, ibp_lo, ibp_hi, what):
    rc = oracle.crown_lower(net, lo, hi, fac)
    ri = orc_plain(net, lo, hi, fac)
    assert g_hi == ibp_hi, what
    assert g_lo == max(ibp_lo, g_c), what
    scale = max(abs(rc["f_lo"]), term_scale(ri, "lo"), 1.0)
    assert g_c <= rc["f_lo"], f"{what}: gpu {g_c!r} > oracle {rc['f_lo']!r}"
    assert (rc["f_lo"] - g_c) / scale <= TOL, f"{what}: gap {rc['f_lo'] - g_c!r} (oracle {rc['f_lo']!r})"
    print(f"[{what}] ibp {ri['f_lo']:.6e} chord gpu {g_c:.6e} oracle {rc['f_lo']:.6e} "
          f"active {rc['n_active']}", flush=True)
    return rc


def test_tiny_boxes_enclose_the_oracle_and_stay_below_the_vertex_minimum():
    net, fac, n = setup("tiny")
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 8, seed=3)
    x = (0.4 * lo + 0.6 * hi).astype(np.float32)
    LO = np.vstack([lo[None], blo, x[None]])
    HI = np.vstack([hi[None], bhi, x[None]])
    for flags in (0, ibp.IBP_F_PLAIN):
        f_lo, f_hi, c = gpu_lower(n, LO, HI, flags=flags)
        i_lo, i_hi = gpu_bounds(n, LO, HI, flags=flags)
        for b in range(LO.shape[0]):
            check_box(net, fac, LO[b], HI[b], f_lo[b], f_hi[b], c[b], i_lo[b], i_hi[b], f"tiny box {b} f{flags}")
            fmin = oracle.point_eval_many(net, _vertices(LO[b], HI[b]), fac["ctg"]).min()
            assert c[b] <= fmin
    # tighter than IBP on most boxes
    assert np.sum(c[:9] > i_lo[:9] + 1e-6 * np.abs(i_lo[:9])) >= 6


def test_single_box_calls_match_the_tiled_call():
    """One to three boxes run the per-box sweep, four or more the box-tiled one;
    the same box gets the same bound up to the float64 summation order of the
    transposed PTDF products."""
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 9, seed=4)
    _, _, c9 = gpu_lower(n, blo, bhi)
    for b in (0, 4, 8):
        _, _, c1 = gpu_lower(n, blo[b], bhi[b])
        assert abs(c1[0] - c9[b]) <= 1e-9 * max(1.0, abs(c9[b])), (b, c1[0], c9[b])
    _, _, c3 = gpu_lower(n, blo[:3], bhi[:3])
    assert np.all(np.abs(c3 - c9[:3]) <= 1e-9 * np.maximum(1.0, np.abs(c9[:3])))


def test_lower_only_flag_gives_the_same_lower_bound():
    """With IBP_F_LOWER_ONLY the chord bound is the same, bit for bit; the IBP
    lower bound it is combined with comes from the screened one-sided sweep
    (the same outage penalties in another float32 order: 1e-6 relative)."""
    from tests.test_gpu_forward import one_sided_close
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 6, seed=5)
    a_lo, a_hi, a_c = gpu_lower(n, blo, bhi)
    b_lo, b_hi, b_c = gpu_lower(n, blo, bhi, flags=ibp.IBP_F_LOWER_ONLY)
    assert one_sided_close(a_lo, b_lo) and np.array_equal(a_c, b_c)
    assert np.all(b_hi >= a_hi)


def test_c500_whole_box_and_sub_boxes():
    net, fac, n = setup("c500")
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 6, seed=9)
    LO = np.vstack([lo[None], blo])
    HI = np.vstack([hi[None], bhi])
    f_lo, f_hi, c = gpu_lower(n, LO, HI)
    i_lo, i_hi = gpu_bounds(n, LO, HI)
    for b in range(LO.shape[0]):
        check_box(net, fac, LO[b], HI[b], f_lo[b], f_hi[b], c[b], i_lo[b], i_hi[b], f"c500 box {b}")


def test_c2000_period_boxes_subset():
    net, fac, n = setup("c2000")
    lo, hi, _ = synth.period_boxes(net, 2, 4, seed=31)
    f_lo, f_hi, c = gpu_lower(n, lo, hi)
    i_lo, i_hi = gpu_bounds(n, lo, hi)
    for b in (0, 7):
        check_box(net, fac, lo[b], hi[b], f_lo[b], f_hi[b], c[b], i_lo[b], i_hi[b], f"c2000 box {b}")


def test_c8316_whole_box():
    net, fac, n = setup("c8316")
    lo, hi = synth.full_box(net)
    f_lo, f_hi, c = gpu_lower(n, lo, hi)
    i_lo, i_hi = gpu_bounds(n, lo, hi)
    check_box(net, fac, lo, hi, f_lo[0], f_hi[0], c[0], i_lo[0], i_hi[0], "c8316 whole box")


def test_curves_and_distinct_outage_limits():
    from tests.test_oracle_pins import _emergency
    net = _emergency(synth.with_pwl_costs(synth.make_config("c500"), seed=6), 4)
    fac = oracle.factors(net)
    n = ibp.Network(net, device=0)
    blo, bhi = synth.sub_boxes(net, 5, seed=2)
    f_lo, f_hi, c = gpu_lower(n, blo, bhi)
    i_lo, i_hi = gpu_bounds(n, blo, bhi)
    for b in range(5):
        check_box(net, fac, blo[b], bhi[b], f_lo[b], f_hi[b], c[b], i_lo[b], i_hi[b], f"curves box {b}")


def test_vertex_is_the_minimiser_of_the_linear_part():
    """The returned vertex takes lo_j where the oracle's coefficient is clearly
    positive and hi_j where it is clearly negative."""
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 5, seed=8)
    _, _, _, v = gpu_lower(n, blo, bhi, vertex=True)
    for b in range(5):
        G = oracle.crown_lower(net, blo[b], bhi[b], fac)["G"]
        clear = np.abs(G) > 1e-6 * np.max(np.abs(G))
        want = np.where(G >= 0, blo[b], bhi[b])
        assert np.array_equal(v[b][clear], want[clear]), b


def test_bad_boxes_radial_network_and_empty_batch():
    torch = _torch()
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 4, seed=5)
    blo[1, 2] = np.nan
    bhi[2, 0] = blo[2, 0] - 1.0
    f_lo, f_hi, c = gpu_lower(n, blo, bhi)
    assert np.isnan(f_lo[1]) and np.isnan(c[1]) and np.isnan(f_lo[2]) and np.isnan(c[2])
    for b in (0, 3):
        assert np.isfinite(c[b]) and c[b] <= oracle.crown_lower(net, blo[b], bhi[b], fac)["f_lo"]
    rad = synth.make_network(30, 29, 6, 12, seed=8)
    rfac = oracle.factors(rad)
    rn = ibp.Network(rad, device=0)
    lo, hi = synth.full_box(rad)
    f_lo, f_hi, c = gpu_lower(rn, lo, hi)
    i_lo, i_hi = gpu_bounds(rn, lo, hi)
    check_box(rad, rfac, lo, hi, f_lo[0], f_hi[0], c[0], i_lo[0], i_hi[0], "radial")
    e = torch.empty((0, n.n_input), dtype=torch.float32, device="cuda")
    a, b = ibp.ibp_crown_lower_boxes(n, e, e)
    assert a.numel() == 0 and b.numel() == 0


def test_vector_and_matrix_core_paths_agree(monkeypatch):
    """IBP_TILE=k2b=0 keeps the transposed PTDF products (and the base flows) on
    the vector ALUs; both paths bound the same quantity with the same error
    terms, summed in different orders.  37 boxes: ragged against the 32-box
    MFMA tile and the 4-box sweep tile."""
    net, fac, n = setup("c500")
    monkeypatch.setenv("IBP_TILE", "k2b=0")
    nv = ibp.Network(net, device=0)
    monkeypatch.delenv("IBP_TILE")
    blo, bhi = synth.sub_boxes(net, 37, seed=12)
    _, _, cm = gpu_lower(n, blo, bhi)
    _, _, cv = gpu_lower(nv, blo, bhi)
    scale = np.maximum(np.abs(cv), 1.0)
    assert np.all(np.abs(cm - cv) <= 1e-9 * scale), np.max(np.abs(cm - cv) / scale)
    for b in (0, 31, 32, 36):
        rc = oracle.crown_lower(net, blo[b], bhi[b], fac)
        assert cm[b] <= rc["f_lo"] and cv[b] <= rc["f_lo"], b


def test_c2000_1024_boxes_sampled():
    """The box-tiled launch at 1024 sub-boxes of the 2000-bus network (the
    bench's relaxation workload): every bound finite and >= IBP's f_lo - 0, and
    sampled boxes against the oracle."""
    net, fac, n = setup("c2000")
    blo, bhi = synth.sub_boxes(net, 1024, seed=61)
    f_lo, f_hi, c = gpu_lower(n, blo, bhi)
    i_lo, i_hi = gpu_bounds(n, blo, bhi)
    assert np.all(np.isfinite(c)) and np.array_equal(f_lo, np.maximum(i_lo, c))
    for b in (0, 517, 1023):
        check_box(net, fac, blo[b], bhi[b], f_lo[b], f_hi[b], c[b], i_lo[b], i_hi[b], f"c2000 box {b}")


def test_one_two_and_four_boxes_per_lane_agree(monkeypatch):
    """The box-tiled sweep keeps one box per lane by default; IBP_TILE=ckb=2
    and ckb=4 keep two and four.  Every per-box sum is formed in the same
    order either way, so the bounds are bitwise equal (37 boxes: ragged
    against every tile)."""
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 37, seed=14)
    a_lo, a_hi, a_c = gpu_lower(n, blo, bhi)
    for ckb in ("2", "4"):
        monkeypatch.setenv("IBP_TILE", "ckb=" + ckb)
        nk = ibp.Network(net, device=0)
        monkeypatch.delenv("IBP_TILE")
        b_lo, b_hi, b_c = gpu_lower(nk, blo, bhi)
        assert np.array_equal(a_c, b_c) and np.array_equal(a_lo, b_lo) and np.array_equal(a_hi, b_hi), ckb
        nk.close()
