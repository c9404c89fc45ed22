"""GPU parity of the backward (VJP) kernels against the FP64 oracle's analytic
gradient, finite differences of the GPU forward, batched vs per-box, and the
autograd wrapper.

The gradient is that of the unpadded IBP map; GPU and oracle take the kink
decisions in different precisions (float32 vs float64), so an element that
sits within rounding of a kink can switch sides.  Parity is therefore asserted
as a relative L2 error <= 1e-4 over all coordinates (1e-3 at full size).
"""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_forward import setup

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def gpu_grad(n, lo, hi, g_lo, g_hi, flags=0):
    torch = _torch()
    tlo = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(lo), np.float32)).cuda()
    thi = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(hi), np.float32)).cuda()
    gl = torch.as_tensor(np.atleast_1d(g_lo), dtype=torch.float64).cuda()
    gh = torch.as_tensor(np.atleast_1d(g_hi), dtype=torch.float64).cuda()
    d_lo, d_hi = ibp.ibp_bound_backward(n, tlo, thi, gl, gh, flags=flags)
    torch.cuda.synchronize()
    return d_lo.cpu().numpy(), d_hi.cpu().numpy()


def rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("gw", [(1.0, 0.0), (0.0, 1.0), (0.3, -0.7)])
def test_tiny_gradient_matches_oracle(gw):
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 6, seed=12)
    lo, hi = synth.full_box(net)
    LO = np.vstack([lo[None], blo])
    HI = np.vstack([hi[None], bhi])
    G_lo = np.full(LO.shape[0], gw[0])
    G_hi = np.full(LO.shape[0], gw[1])
    d_lo, d_hi = gpu_grad(n, LO, HI, G_lo, G_hi)
    for b in range(LO.shape[0]):
        o_lo, o_hi, near = oracle.grad(net, LO[b], HI[b], gw[0], gw[1], fac)
        ref = np.concatenate([o_lo, o_hi])
        got = np.concatenate([d_lo[b], d_hi[b]])
        assert rel_l2(got, ref) <= 1e-4, (b, rel_l2(got, ref), near)


def test_c500_gradient_matches_oracle():
    net, fac, n = setup("c500")
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 3, seed=77)
    LO = np.vstack([lo[None], blo])
    HI = np.vstack([hi[None], bhi])
    d_lo, d_hi = gpu_grad(n, LO, HI, np.full(4, 0.5), np.full(4, -1.5))
    for b in range(4):
        o_lo, o_hi, _ = oracle.grad(net, LO[b], HI[b], 0.5, -1.5, fac)
        assert rel_l2(np.concatenate([d_lo[b], d_hi[b]]), np.concatenate([o_lo, o_hi])) <= 1e-4, b


def test_c8316_gradient_matches_oracle():
    net, fac, n = setup("c8316")
    blo, bhi = synth.sub_boxes(net, 1, seed=41)
    d_lo, d_hi = gpu_grad(n, blo, bhi, np.array([1.0]), np.array([1.0]))
    o_lo, o_hi, _ = oracle.grad(net, blo[0], bhi[0], 1.0, 1.0, fac)
    assert rel_l2(np.concatenate([d_lo[0], d_hi[0]]), np.concatenate([o_lo, o_hi])) <= 1e-3


def test_gradient_against_central_differences_of_the_gpu_forward():
    """Central differences (h = 1e-4) of the GPU bounds, on coordinates whose
    oracle gradient is the same at x - h and x + h (no kink in between)."""
    torch = _torch()
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 1, seed=5)
    a, b = blo[0].astype(np.float64), bhi[0].astype(np.float64)
    d_lo, d_hi = gpu_grad(n, blo, bhi, np.array([1.0]), np.array([0.0]))
    h = 1e-4
    rows_lo, rows_hi, idx = [], [], []
    for j in range(a.size):
        for side in (0, 1):
            lp, hp, lm, hm = a.copy(), b.copy(), a.copy(), b.copy()
            if side == 0:
                lp[j] += h
                lm[j] -= h
                if lp[j] > b[j]:
                    continue
            else:
                hp[j] += h
                hm[j] -= h
                if hm[j] < a[j]:
                    continue
            gp = oracle.grad(net, lp, hp, 1.0, 0.0, fac)
            gm = oracle.grad(net, lm, hm, 1.0, 0.0, fac)
            if not (np.allclose(gp[side][j], gm[side][j], rtol=1e-9, atol=1e-9)):
                continue
            rows_lo += [lp, lm]
            rows_hi += [hp, hm]
            idx.append((j, side))
    # float32 endpoints: evaluate at the float32 grid points actually used
    LO = np.asarray(rows_lo, np.float32)
    HI = np.asarray(rows_hi, np.float32)
    tl = torch.from_numpy(LO).cuda()
    th = torch.from_numpy(HI).cuda()
    f_lo, _ = ibp.ibp_bound_boxes(n, tl, th)
    f = f_lo.cpu().numpy()
    checked = 0
    for i, (j, side) in enumerate(idx):
        step = (float(LO[2 * i, j]) - float(LO[2 * i + 1, j])) if side == 0 else \
               (float(HI[2 * i, j]) - float(HI[2 * i + 1, j]))
        fd = (f[2 * i] - f[2 * i + 1]) / step
        g = d_lo[0, j] if side == 0 else d_hi[0, j]
        # float32 bounds carry ~1e-7 relative noise: scale the tolerance with |f| / step
        tol = 1e-3 * max(abs(g), 1.0) + 4e-7 * max(abs(f[2 * i]), 1.0) / abs(step)
        assert abs(fd - g) <= tol, (j, side, fd, g)
        checked += 1
    assert checked >= 10


def test_batched_backward_equals_per_box_and_bad_boxes():
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 13, seed=5)
    blo, bhi = blo.copy(), bhi.copy()
    blo[3, 0] = np.nan
    g1 = np.linspace(-1, 1, 13)
    g2 = np.linspace(2, 0.5, 13)
    a_lo, a_hi = gpu_grad(n, blo, bhi, g1, g2)
    p_lo, p_hi = gpu_grad(n, blo, bhi, g1, g2, flags=ibp.IBP_F_PLAIN)
    assert np.all(np.isnan(a_lo[3])) and np.all(np.isnan(a_hi[3]))
    ok = np.arange(13) != 3
    assert rel_l2(a_lo[ok], p_lo[ok]) <= 1e-5 and rel_l2(a_hi[ok], p_hi[ok]) <= 1e-5
    for b in (0, 12):
        o_lo, o_hi, _ = oracle.grad(net, blo[b], bhi[b], g1[b], g2[b], fac)
        assert rel_l2(np.concatenate([a_lo[b], a_hi[b]]), np.concatenate([o_lo, o_hi])) <= 1e-4


def test_vector_and_matrix_core_transposed_products_agree(monkeypatch):
    """From 4 boxes on, the transposed PTDF products of the backward run on the
    float32 matrix cores by default and on the vector ALUs with
    IBP_TILE=k2b=0 (which also moves the base flows to the vector kernel).
    Both sum 32-line chunks in float32 and the chunk sums in float64; 70
    boxes are ragged against the 64-box tiles of both kernels.  Each box's
    gradient agrees between the two within 1e-5 relative L2, and sampled boxes
    match the oracle."""
    net, fac, n = setup("c500")
    monkeypatch.setenv("IBP_TILE", "k2b=0")
    nv = ibp.Network(net, device=0)
    monkeypatch.delenv("IBP_TILE")
    blo, bhi = synth.sub_boxes(net, 70, seed=17)
    g1 = np.linspace(-1.0, 0.5, 70)
    g2 = np.linspace(0.2, 1.5, 70)
    m_lo, m_hi = gpu_grad(n, blo, bhi, g1, g2)
    v_lo, v_hi = gpu_grad(nv, blo, bhi, g1, g2)
    for b in range(70):
        m = np.concatenate([m_lo[b], m_hi[b]])
        v = np.concatenate([v_lo[b], v_hi[b]])
        assert rel_l2(m, v) <= 1e-5, (b, rel_l2(m, v))
    for b in (0, 63, 64, 69):
        o_lo, o_hi, _ = oracle.grad(net, blo[b], bhi[b], g1[b], g2[b], fac)
        assert rel_l2(np.concatenate([m_lo[b], m_hi[b]]), np.concatenate([o_lo, o_hi])) <= 1e-4, b


def test_autograd_function():
    torch = _torch()
    from paper_2511_15624_amd.autograd import ibp_bound
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 5, seed=1)
    lo = torch.from_numpy(blo).cuda().requires_grad_(True)
    hi = torch.from_numpy(bhi).cuda().requires_grad_(True)
    f_lo, f_hi = ibp_bound(n, lo, hi)
    w = torch.linspace(0.1, 1.0, 5, dtype=torch.float64, device="cuda")
    (w * f_hi - 0.5 * f_lo).sum().backward()
    d_lo, d_hi = gpu_grad(n, blo, bhi, np.full(5, -0.5), np.linspace(0.1, 1.0, 5))
    np.testing.assert_allclose(lo.grad.cpu().numpy(), d_lo.astype(np.float32), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(hi.grad.cpu().numpy(), d_hi.astype(np.float32), rtol=1e-6, atol=1e-6)


def test_one_sided_backward_matches_zero_weights():
    """IBP_F_UPPER_ONLY (LOWER_ONLY) gives the VJP with g_lo (g_hi) = 0 without
    reading that weight: bit for bit up to the sign of zeros in the per-box
    path and for LOWER_ONLY; the box-tiled UPPER_ONLY call takes the screened
    sweep (same activity decisions, other float32 summation order: 2e-5 relative L2
    per box)."""
    torch = _torch()
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 9, seed=31)
    tlo, thi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    z = torch.zeros(9, dtype=torch.float64, device="cuda")
    g = torch.linspace(0.5, 1.5, 9, dtype=torch.float64, device="cuda")
    for plain in (0, ibp.IBP_F_PLAIN):
        a_lo, a_hi = ibp.ibp_bound_backward(n, tlo, thi, z, g, flags=plain)
        b_lo, b_hi = ibp.ibp_bound_backward(n, tlo, thi, None, g, flags=plain | ibp.IBP_F_UPPER_ONLY)
        c_lo, c_hi = ibp.ibp_bound_backward(n, tlo, thi, g, z, flags=plain)
        d_lo, d_hi = ibp.ibp_bound_backward(n, tlo, thi, g, None, flags=plain | ibp.IBP_F_LOWER_ONLY)
        torch.cuda.synchronize()
        for x, y in ((c_lo, d_lo), (c_hi, d_hi)) + (((a_lo, b_lo), (a_hi, b_hi)) if plain else ()):
            assert torch.equal(x, y), float((x - y).abs().max())
        if not plain:
            a = torch.cat([a_lo, a_hi], 1)
            b = torch.cat([b_lo, b_hi], 1)
            rel = ((a - b).norm(dim=1) / a.norm(dim=1).clamp_min(1e-30)).max().item()
            assert rel <= 2e-5, rel
    with pytest.raises(ValueError):
        ibp.ibp_bound_backward(n, tlo, thi, None, g)


def test_c2000_gradient_against_central_differences_at_4096_boxes():
    """The differentiation workload (2000 buses, 4096 sub-boxes, one backward
    call per bound, as bench.py times it): on 8 seeded boxes and 64 seeded
    endpoint coordinates each, the GPU's d f_lo and d f_hi agree with central
    differences (step 1e-4, endpoints moved in float64) of the FP64 oracle's
    bounds to 1e-4 relative, plus what float32 activity decisions can change:
    the GPU decides each penalty's activity in float32, so an element within
    float32 resolution of its kink may count where the oracle's does not, which
    moves the gradient by zeta_f times that element's own gradient; those
    elements are listed from the oracle's values and their effect on each
    coordinate is added to the bar (tests/error_budget.py, flip_allowance).
    A difference is used where it equals the oracle's analytic gradient to 1e-6
    (the map is piecewise linear, so that holds where no kink lies within the
    step); at least 48 of the 64 coordinates of every box and side, and 90% of
    all, must pass that screen.  The GPU gradient of each box is also within 1e-4 relative L2 of
    the oracle's over all coordinates."""
    from tests.error_budget import budget, flip_allowance
    from tests.fd_check import central_differences, coordinates
    torch = _torch()
    net, fac, n = setup("c2000")
    blo, bhi = synth.sub_boxes(net, 4096, seed=51)
    tlo, thi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    one = torch.ones(4096, dtype=torch.float64, device="cuda")
    dl_lo, dl_hi = ibp.ibp_bound_backward(n, tlo, thi, one, None, flags=ibp.IBP_F_LOWER_ONLY)
    dh_lo, dh_hi = ibp.ibp_bound_backward(n, tlo, thi, None, one, flags=ibp.IBP_F_UPPER_ONLY)
    torch.cuda.synchronize()
    gpu = {"lo": (dl_lo.cpu().numpy(), dl_hi.cpu().numpy()), "hi": (dh_lo.cpu().numpy(), dh_hi.cpu().numpy())}
    del dl_lo, dl_hi, dh_lo, dh_hi
    rng = np.random.default_rng(88)
    h = 1e-4
    worst, n_near, n_lin = 0.0, [], []
    for b in np.sort(rng.choice(4096, 8, replace=False)):
        coords = coordinates(blo[b], bhi[b], 64, h, rng)
        fd = dict(zip(("lo", "hi"), central_differences(net, fac, blo[b], bhi[b], coords, h)))
        bu = budget(net, fac, blo[b], bhi[b], n.info.phi_abs_err, near=True)
        for side, gw in (("lo", (1.0, 0.0)), ("hi", (0.0, 1.0))):
            o = oracle.grad(net, blo[b], bhi[b], gw[0], gw[1], fac)
            g = gpu[side]
            assert rel_l2(np.concatenate([g[0][b], g[1][b]]), np.concatenate(o[:2])) <= 1e-4, (b, side)
            scale = max(np.max(np.abs(o[0])), np.max(np.abs(o[1])))
            an = np.array([o[s][j] for s, j in coords])
            got = np.array([g[s][b, j] for s, j in coords])
            lin = np.abs(fd[side] - an) <= 1e-6 * np.maximum(np.abs(an), 1e-3 * scale)
            assert lin.sum() >= 48, (b, side, int(lin.sum()))
            n_lin.append(int(lin.sum()))
            allow = flip_allowance(net, fac, bu["near_" + side])
            n_near.append(len(bu["near_" + side]))
            al = np.array([allow[s][j] for s, j in coords])
            bar = 1e-4 * np.maximum(np.abs(fd[side]), 1e-3 * scale) + al
            err = np.abs(got - fd[side])
            assert np.all(err[lin] <= bar[lin]), (b, side, float(np.max((err - bar)[lin])))
            worst = max(worst, float(np.max(err[lin] / bar[lin])))
    assert sum(n_lin) >= 0.9 * 64 * len(n_lin), n_lin
    print(f"[c2000 central differences] kink-free coordinates {n_lin}; elements near a kink per box and side "
          f"{n_near}; largest error / bar {worst:.3f}", flush=True)


@pytest.mark.parametrize("name,nb,flags", [("c500", 37, 0), ("c500", 1, 0), ("c500", 6, ibp.IBP_F_PLAIN),
                                           ("tiny", 9, 0), ("tiny", 1, 0)])
def test_backward_reuses_the_forward_intermediates(name, nb, flags):
    """A forward with IBP_F_KEEP_PREP followed by a backward with
    IBP_F_REUSE_PREP on the same boxes and workspace gives bitwise the
    gradient of a standalone backward (both sides, and one-sided), runs none
    of the preparation kernels, and leaves the record for a second reuse;
    box-tiled, per-box, single-box and one-block paths."""
    torch = _torch()
    net, fac, n = setup(name)
    blo, bhi = synth.sub_boxes(net, nb, seed=41)
    lo, hi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    g1 = torch.linspace(-1.0, 0.5, nb, dtype=torch.float64, device="cuda")
    g2 = torch.linspace(0.3, 1.2, nb, dtype=torch.float64, device="cuda")
    ref_lo, ref_hi = ibp.ibp_bound_backward(n, lo, hi, g1, g2, flags=flags)
    ref1_lo, ref1_hi = ibp.ibp_bound_backward(n, lo, hi, None, g2, flags=flags | ibp.IBP_F_UPPER_ONLY)
    ws = ibp.Workspace(n)
    assert n.workspace_bytes(nb, flags | ibp.IBP_F_KEEP_PREP) == n.workspace_bytes(nb, flags | ibp.IBP_F_BACKWARD)
    f_lo, f_hi = ibp.ibp_bound_boxes(n, lo, hi, flags=flags | ibp.IBP_F_KEEP_PREP, ws=ws)
    p_lo, p_hi = ibp.ibp_bound_boxes(n, lo, hi, flags=flags)
    assert torch.equal(f_lo, p_lo) and torch.equal(f_hi, p_hi)
    n.set_kernel_timing(True)
    n.kernel_times()
    d_lo, d_hi = ibp.ibp_bound_backward(n, lo, hi, g1, g2, flags=flags | ibp.IBP_F_REUSE_PREP, ws=ws)
    kt = n.kernel_times()
    n.set_kernel_timing(False)
    assert not {"box_prep", "base_flows", "batched_base_flows", "line_epilogue"} & set(kt), kt
    e1_lo, e1_hi = ibp.ibp_bound_backward(n, lo, hi, None, g2, flags=flags | ibp.IBP_F_UPPER_ONLY |
                                          ibp.IBP_F_REUSE_PREP, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(d_lo, ref_lo) and torch.equal(d_hi, ref_hi)
    assert torch.equal(e1_lo, ref1_lo) and torch.equal(e1_hi, ref1_hi)


def test_reuse_is_refused_when_the_workspace_holds_something_else():
    torch = _torch()
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 8, seed=42)
    lo, hi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    g = torch.ones(8, dtype=torch.float64, device="cuda")
    up = ibp.IBP_F_UPPER_ONLY

    def refused(ws, lo_=lo, hi_=hi, flags=0):
        with pytest.raises(ibp.IBPError) as e:
            ibp.ibp_bound_backward(n, lo_, hi_, None, g, flags=flags | up | ibp.IBP_F_REUSE_PREP, ws=ws)
        assert e.value.name == "IBP_E_INVALID_ARG"

    ws = ibp.Workspace(n)
    refused(ws)                                              # nothing kept yet
    ibp.ibp_bound_boxes(n, lo, hi, ws=ws)                    # a forward without the flag keeps nothing
    refused(ws)
    ibp.ibp_bound_boxes(n, lo, hi, flags=ibp.IBP_F_KEEP_PREP, ws=ws)
    refused(ibp.Workspace(n))                                # another workspace
    refused(ws, lo.clone(), hi.clone())                      # other box arrays
    refused(ws, flags=ibp.IBP_F_PLAIN)                       # other kernels
    ibp.ibp_crown_bound_boxes(n, lo, hi, ws=ws)              # another call on the workspace
    refused(ws)
    ibp.ibp_bound_boxes(n, lo, hi, flags=ibp.IBP_F_KEEP_PREP, ws=ws)
    t = n.tiles()
    n.set_tile_batched(t["k3_bt"], t["k3_rows"], t["k3_xcd"], t["k2_mfma"], t["k2_by"])   # a tile change
    refused(ws)
    ibp.ibp_bound_backward(n, lo, hi, None, g, flags=up, ws=ws)    # a backward leaves its own
    a = ibp.ibp_bound_backward(n, lo, hi, None, g, flags=up | ibp.IBP_F_REUSE_PREP, ws=ws)
    b = ibp.ibp_bound_backward(n, lo, hi, None, g, flags=up)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    for bad in ((ibp.ibp_bound_boxes, dict(flags=ibp.IBP_F_REUSE_PREP)),):
        with pytest.raises(ibp.IBPError):
            bad[0](n, lo, hi, ws=ws, **bad[1])
    with pytest.raises(ibp.IBPError):
        ibp.ibp_bound_backward(n, lo, hi, None, g, flags=up | ibp.IBP_F_KEEP_PREP, ws=ws)


def test_autograd_reuses_the_forward_and_falls_back_when_it_cannot():
    """IBPBound keeps the forward's intermediates for its backward: the
    gradient equals a standalone backward's bit for bit (37 boxes, box-tiled);
    a second backward of the same graph, and one after a tile change, recompute
    them and give the same values."""
    torch = _torch()
    from paper_2511_15624_amd.autograd import ibp_bound
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 37, seed=43)
    w = torch.linspace(0.2, 1.0, 37, dtype=torch.float64, device="cuda")
    ref_lo, ref_hi = ibp.ibp_bound_backward(n, torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda(),
                                            -0.5 * torch.ones_like(w), w)
    ref_lo, ref_hi = ref_lo.float(), ref_hi.float()
    for tile_change in (False, True):
        lo = torch.from_numpy(blo).cuda().requires_grad_(True)
        hi = torch.from_numpy(bhi).cuda().requires_grad_(True)
        f_lo, f_hi = ibp_bound(n, lo, hi)
        if tile_change:
            t = n.tiles()
            n.set_tile_batched(t["k3_bt"], t["k3_rows"], t["k3_xcd"], t["k2_mfma"], t["k2_by"])
        loss = (w * f_hi - 0.5 * f_lo).sum()
        loss.backward(retain_graph=True)
        assert torch.equal(lo.grad, ref_lo) and torch.equal(hi.grad, ref_hi), tile_change
        loss.backward()
        assert torch.equal(lo.grad, 2 * ref_lo) and torch.equal(hi.grad, 2 * ref_hi), tile_change


def test_autograd_takes_the_one_sided_backward_when_one_bound_reaches_the_loss():
    """A loss on f_hi alone gives the one-sided backward (the screened sweep)
    bit for bit, and a loss on f_lo alone the LOWER_ONLY call; both within
    float32 summation order of the two-sided call with a zero weight."""
    torch = _torch()
    from paper_2511_15624_amd.autograd import ibp_bound
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 37, seed=47)
    tlo, thi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    w = torch.linspace(0.2, 1.0, 37, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(w)
    for side in ("hi", "lo"):
        lo = tlo.clone().requires_grad_(True)
        hi = thi.clone().requires_grad_(True)
        f_lo, f_hi = ibp_bound(n, lo, hi)
        ((w * f_hi) if side == "hi" else (w * f_lo)).sum().backward()
        if side == "hi":
            one = ibp.ibp_bound_backward(n, tlo, thi, None, w, flags=ibp.IBP_F_UPPER_ONLY)
            two = ibp.ibp_bound_backward(n, tlo, thi, z, w)
        else:
            one = ibp.ibp_bound_backward(n, tlo, thi, w, None, flags=ibp.IBP_F_LOWER_ONLY)
            two = ibp.ibp_bound_backward(n, tlo, thi, w, z)
        assert torch.equal(lo.grad, one[0].float()) and torch.equal(hi.grad, one[1].float()), side
        a = torch.cat([lo.grad.double(), hi.grad.double()], 1)
        b = torch.cat([two[0], two[1]], 1)
        rel = ((a - b).norm(dim=1) / b.norm(dim=1).clamp_min(1e-30)).max().item()
        assert rel <= 2e-5, (side, rel)


def _sparse_and_dense(monkeypatch, net):
    n = ibp.Network(net, device=0)
    monkeypatch.setenv("IBP_TILE", "k5s=0")
    nd = ibp.Network(net, device=0)
    monkeypatch.delenv("IBP_TILE")
    return n, nd


@pytest.mark.parametrize("name,nb,seed", [("tiny", 5, 3), ("c500", 37, 5), ("c500", 4, 6), ("c2000", 70, 7)])
def test_screened_sweep_matches_the_dense_sweep(monkeypatch, name, nb, seed):
    """The gradient of f_hi alone (IBP_F_UPPER_ONLY, 4 or more boxes) runs the
    outage sweep on the lines a screen marks per tile of four boxes; the dense
    sweep (IBP_TILE=k5s=0) runs every line.  Both take every activity decision
    with the same float32 operations, so the gradients differ only by
    summation order (float32 sums: 2e-5 relative L2 per box; a line the screen missed would
    drop whole elements, each worth zeta_f |g| on its line).  Box counts
    ragged against the 4-box tiles; sampled boxes also match the oracle."""
    torch = _torch()
    net = synth.make_config(name)
    n, nd = _sparse_and_dense(monkeypatch, net)
    blo, bhi = synth.sub_boxes(net, nb, seed=seed)
    tlo, thi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    g = torch.linspace(0.5, 1.5, nb, dtype=torch.float64, device="cuda")
    s_lo, s_hi = ibp.ibp_bound_backward(n, tlo, thi, None, g, flags=ibp.IBP_F_UPPER_ONLY)
    d_lo, d_hi = ibp.ibp_bound_backward(nd, tlo, thi, None, g, flags=ibp.IBP_F_UPPER_ONLY)
    torch.cuda.synchronize()
    s = torch.cat([s_lo, s_hi], 1).cpu().numpy()
    d = torch.cat([d_lo, d_hi], 1).cpu().numpy()
    for b in range(nb):
        assert rel_l2(s[b], d[b]) <= 2e-5, (b, rel_l2(s[b], d[b]))
    fac = oracle.factors(net)
    gh = np.linspace(0.5, 1.5, nb)
    for b in sorted({0, nb // 2, nb - 1}):
        o_lo, o_hi, _ = oracle.grad(net, blo[b], bhi[b], 0.0, gh[b], fac)
        assert rel_l2(s[b], np.concatenate([o_lo, o_hi])) <= 1e-4, b


@pytest.mark.parametrize("limit", ["tiny", "huge"])
def test_screened_sweep_when_every_or_no_line_is_a_candidate(monkeypatch, limit):
    """Outage limits of 1e-6 make every element whose post-outage flow interval
    excludes zero active (60% of them here, on 82-90% of each box's lines per
    the oracle; the screen marks at least 80% of the tile-lines); limits of 1e30
    leave none active (it marks none, and the outage terms of the gradient are
    exactly zero).  Both agree with the dense sweep."""
    torch = _torch()
    net = dict(synth.make_config("c500"))
    net["fmax_ctg"] = np.full(len(net["fmax_ctg"]), 1e-6 if limit == "tiny" else 1e30)
    n, nd = _sparse_and_dense(monkeypatch, net)
    blo, bhi = synth.sub_boxes(net, 13, seed=9)
    tlo, thi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    g = torch.ones(13, dtype=torch.float64, device="cuda")
    s = torch.cat(ibp.ibp_bound_backward(n, tlo, thi, None, g, flags=ibp.IBP_F_UPPER_ONLY), 1).cpu().numpy()
    d = torch.cat(ibp.ibp_bound_backward(nd, tlo, thi, None, g, flags=ibp.IBP_F_UPPER_ONLY), 1).cpu().numpy()
    for b in range(13):
        assert rel_l2(s[b], d[b]) <= 2e-5, (b, rel_l2(s[b], d[b]))
    ws = ibp.Workspace(n)
    ibp.ibp_bound_backward(n, tlo, thi, None, g, ws=ws, flags=ibp.IBP_F_UPPER_ONLY)
    marked, pairs = ibp.ibp_backward_screen_lines(n, 13, ws)
    assert pairs == 4 * n.n_line  # ceil(13 / 4) tiles
    assert (marked >= 0.8 * pairs) if limit == "tiny" else marked == 0, (marked, pairs)
    if limit == "huge":
        np.testing.assert_array_equal(s, d)


def test_screen_marks_a_minority_of_lines_at_the_differentiation_workload():
    """2000 buses, 4096 sub-boxes: the screen marks the lines of each 4-box
    tile that can hold an active lower penalty (about a fifth of them); the
    count query refuses sizes with no screened sweep."""
    torch = _torch()
    net, fac, n = setup("c2000")
    blo, bhi = synth.sub_boxes(net, 4096, seed=51)
    tlo, thi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    ws = ibp.Workspace(n)
    ibp.ibp_bound_backward(n, tlo, thi, None, torch.ones(4096, dtype=torch.float64, device="cuda"), ws=ws,
                           flags=ibp.IBP_F_UPPER_ONLY)
    marked, pairs = ibp.ibp_backward_screen_lines(n, 4096, ws)
    assert pairs == 1024 * n.n_line
    print(f"[screen] {marked} of {pairs} tile-lines marked ({marked / pairs:.3f})", flush=True)
    assert 0.05 * pairs < marked < 0.4 * pairs
    with pytest.raises(ibp.IBPError):
        ibp.ibp_backward_screen_lines(n, 3, ws)


def test_screened_paths_with_invalid_boxes_in_a_tile(monkeypatch):
    """A box with a NaN endpoint and an inverted box share 4-box tiles with
    valid ones: the screened one-sided forward and backward give the valid
    boxes the dense sweeps' results (summation order aside) and the invalid
    ones NaN."""
    torch = _torch()
    net = synth.make_config("c500")
    n = ibp.Network(net, device=0)
    monkeypatch.setenv("IBP_TILE", "k3s=0,k5s=0")
    nd = ibp.Network(net, device=0)
    monkeypatch.delenv("IBP_TILE")
    blo, bhi = synth.sub_boxes(net, 11, seed=21)
    blo[1, 3] = np.nan
    blo[6, 0], bhi[6, 0] = bhi[6, 0] + 1.0, blo[6, 0]
    bad = np.zeros(11, bool)
    bad[[1, 6]] = True
    tlo, thi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    g = torch.linspace(0.5, 1.5, 11, dtype=torch.float64, device="cuda")
    for flag, pick in ((ibp.IBP_F_UPPER_ONLY, 1), (ibp.IBP_F_LOWER_ONLY | ibp.IBP_F_SCREEN_UPPER, 0)):
        s = ibp.ibp_bound_boxes(n, tlo, thi, flags=flag)[pick].cpu().numpy()
        d = ibp.ibp_bound_boxes(nd, tlo, thi, flags=flag)[pick].cpu().numpy()
        assert np.all(np.isnan(s[bad])) and np.all(np.isnan(d[bad]))
        assert np.all(np.abs(s[~bad] - d[~bad]) <= 1e-6 * np.maximum(np.abs(d[~bad]), 1.0)), flag
    s = torch.cat(ibp.ibp_bound_backward(n, tlo, thi, None, g, flags=ibp.IBP_F_UPPER_ONLY), 1).cpu().numpy()
    d = torch.cat(ibp.ibp_bound_backward(nd, tlo, thi, None, g, flags=ibp.IBP_F_UPPER_ONLY), 1).cpu().numpy()
    assert np.all(np.isnan(s[bad])) and np.all(np.isnan(d[bad]))
    for b in np.flatnonzero(~bad):
        assert rel_l2(s[b], d[b]) <= 2e-5, (b, rel_l2(s[b], d[b]))
