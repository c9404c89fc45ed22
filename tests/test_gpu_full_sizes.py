"""GPU parity at the full batch sizes, in the launch configurations bench.py
times: every box of the call is checked against what holds at any size (finite,
f_lo <= f_hi, agreement with the per-box kernels on a sample), and sampled boxes
against the FP64 oracle one by one (enclosure and the 1e-5 bar of the forward
tests; gradients to the 1e-3 relative L2 bar of the full-size backward test).

- 2000 buses, 18 periods x 1024 sub-boxes in one call (18432 boxes);
- 8316 buses, 256 sub-boxes in one call;
- 2000 buses, backward over 4096 sub-boxes in one call;
- 8316 buses, the chord-relaxation lower bound over 256 sub-boxes.
"""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_backward import gpu_grad, rel_l2
from tests.test_gpu_forward import _torch, assert_encloses, gpu_bounds, orc, setup

pytestmark = pytest.mark.gpu


def _sample(n, k, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, n - 1], rng.choice(n, k, replace=False)]))


def _plain_agrees(n, lo, hi, idx, g_lo, g_hi):
    p_lo, p_hi = gpu_bounds(n, lo[idx], hi[idx], flags=ibp.IBP_F_PLAIN)
    for a, b in ((g_lo[idx], p_lo), (g_hi[idx], p_hi)):
        assert np.all(np.abs(a - b) <= 1e-6 * np.maximum(np.abs(b), 1.0)), np.max(np.abs(a - b))


def test_c2000_eighteen_periods_of_1024_boxes():
    net, fac, n = setup("c2000")
    lo, hi, _ = synth.period_boxes(net, 18, 1024, seed=31)
    f_lo, f_hi = gpu_bounds(n, lo, hi)
    assert f_lo.shape == (18432,) and np.all(np.isfinite(f_lo)) and np.all(np.isfinite(f_hi))
    assert np.all(f_lo <= f_hi)
    idx = _sample(18432, 30, seed=5)
    _plain_agrees(n, lo, hi, idx, f_lo, f_hi)
    for b in idx[:8]:
        assert_encloses(f_lo[b], f_hi[b], orc(net, lo[b], hi[b], fac), what=f"box {b}")


def test_c8316_256_boxes():
    net, fac, n = setup("c8316")
    blo, bhi = synth.sub_boxes(net, 256, seed=41)
    f_lo, f_hi = gpu_bounds(n, blo, bhi)
    assert np.all(np.isfinite(f_lo)) and np.all(np.isfinite(f_hi)) and np.all(f_lo <= f_hi)
    idx = _sample(256, 6, seed=6)
    _plain_agrees(n, blo, bhi, idx, f_lo, f_hi)
    for b in (0, 255):
        assert_encloses(f_lo[b], f_hi[b], orc(net, blo[b], bhi[b], fac), what=f"box {b}")


def test_c2000_backward_over_4096_boxes():
    net, fac, n = setup("c2000")
    blo, bhi = synth.sub_boxes(net, 4096, seed=51)
    d_lo, d_hi = gpu_grad(n, blo, bhi, np.zeros(4096), np.ones(4096))
    assert np.all(np.isfinite(d_lo)) and np.all(np.isfinite(d_hi))
    idx = _sample(4096, 6, seed=7)
    p_lo, p_hi = gpu_grad(n, blo[idx], bhi[idx], np.zeros(idx.size), np.ones(idx.size), flags=ibp.IBP_F_PLAIN)
    for j, b in enumerate(idx):
        got = np.concatenate([d_lo[b], d_hi[b]])
        assert rel_l2(got, np.concatenate([p_lo[j], p_hi[j]])) <= 1e-4, b
    for b in idx[:3]:
        o_lo, o_hi, _ = oracle.grad(net, blo[b], bhi[b], 0.0, 1.0, fac)
        assert rel_l2(np.concatenate([d_lo[b], d_hi[b]]), np.concatenate([o_lo, o_hi])) <= 1e-3, b


def test_more_boxes_than_one_tiled_launch():
    """16 x 65535 + 37 boxes: the box-tiled path runs as two chunks; every box
    gets exactly what the same box gets in a small call (forward, backward and
    the chord-relaxation lower bound)."""
    torch = _torch()
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 23, seed=9)
    nb = 16 * 65535 + 37
    idx = np.arange(nb) % 23
    lo, hi = blo[idx], bhi[idx]
    f_lo, f_hi = gpu_bounds(n, lo, hi)
    s_lo, s_hi = gpu_bounds(n, blo, bhi)
    assert np.array_equal(f_lo, s_lo[idx]) and np.array_equal(f_hi, s_hi[idx])
    tlo, thi = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    g1 = torch.ones(nb, dtype=torch.float64, device="cuda")
    d_lo, d_hi = ibp.ibp_bound_backward(n, tlo, thi, None, g1, flags=ibp.IBP_F_UPPER_ONLY)
    e_lo, e_hi = ibp.ibp_bound_backward(n, tlo[:23], thi[:23], None, g1[:23], flags=ibp.IBP_F_UPPER_ONLY)
    torch.cuda.synchronize()
    t = torch.from_numpy(idx).cuda()
    assert torch.equal(d_lo, e_lo[t]) and torch.equal(d_hi, e_hi[t])
    del d_lo, d_hi, e_lo, e_hi
    # the chord-relaxation lower bound over the same chunked call
    c_lo, c_hi, c = ibp.ibp_crown_lower_boxes(n, tlo, thi, crown=True)
    s_lo, s_hi, sc = ibp.ibp_crown_lower_boxes(n, tlo[:23].contiguous(), thi[:23].contiguous(), crown=True)
    torch.cuda.synchronize()
    assert torch.equal(c, sc[t]) and torch.equal(c_lo, s_lo[t]) and torch.equal(c_hi, s_hi[t])
    del tlo, thi, c_lo, c_hi, c
    torch.cuda.empty_cache()


def test_c8316_256_boxes_lower_relaxation():
    """The chord-relaxation lower bound at 256 sub-boxes of the 8316-bus network
    (box-tiled sweep, line-major adjoint for the matrix-core product): every box
    finite and combined with IBP's f_lo, sampled boxes equal to single-box calls
    (per-box sweep) up to float64 summation order, and two boxes against the
    oracle's relaxation."""
    from tests.test_gpu_crown_lower import check_box, gpu_lower
    net, fac, n = setup("c8316")
    blo, bhi = synth.sub_boxes(net, 256, seed=41)
    f_lo, f_hi, c = gpu_lower(n, blo, bhi)
    i_lo, i_hi = gpu_bounds(n, blo, bhi)
    assert np.all(np.isfinite(c)) and np.array_equal(f_lo, np.maximum(i_lo, c)) and np.array_equal(f_hi, i_hi)
    for b in (0, 131, 255):
        _, _, c1 = gpu_lower(n, blo[b], bhi[b])
        assert abs(c1[0] - c[b]) <= 1e-9 * max(1.0, abs(c[b])), (b, c1[0], c[b])
    for b in (0, 255):
        check_box(net, fac, blo[b], bhi[b], f_lo[b], f_hi[b], c[b], i_lo[b], i_hi[b], f"c8316 chord box {b}")
