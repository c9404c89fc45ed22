"""GPU parity of the box-tiled (batched) forward path.

Each box must enclose the FP64 oracle's interval to the same bar as the
single-box path, and agree with the per-box (IBP_F_PLAIN) kernels up to
summation order: the float64 base flows are summed in a different order, so a
line centre can round to a neighbouring float32 value, which moves a bound by
about u = 6e-8 of its terms (1e-6 is asserted).
"""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_forward import assert_encloses, gpu_bounds, orc, setup

pytestmark = pytest.mark.gpu


def _both(n, lo, hi):
    b_lo, b_hi = gpu_bounds(n, lo, hi)
    p_lo, p_hi = gpu_bounds(n, lo, hi, flags=ibp.IBP_F_PLAIN)
    return b_lo, b_hi, p_lo, p_hi


def _close(a, b, rel=1e-6):
    assert np.all(np.abs(a - b) <= rel * np.maximum(np.abs(b), 1.0)), np.max(np.abs(a - b))


def test_batched_c500_ragged_batch():
    net, fac, n = setup("c500")
    blo, bhi = synth.sub_boxes(net, 37, seed=303)       # 37: ragged against the 16-box block group
    b_lo, b_hi, p_lo, p_hi = _both(n, blo, bhi)
    _close(b_lo, p_lo)
    _close(b_hi, p_hi)
    for b in (0, 5, 17, 36):
        assert_encloses(b_lo[b], b_hi[b], orc(net, blo[b], bhi[b], fac), what=f"box {b}")


def test_batched_tiny_with_bad_boxes_and_points():
    net, fac, n = setup("tiny")
    blo, bhi = synth.sub_boxes(net, 23, seed=9)
    blo, bhi = blo.copy(), bhi.copy()
    blo[4] = bhi[4]                                        # zero-width box
    blo[7, 1] = np.inf                                     # invalid box
    b_lo, b_hi, p_lo, p_hi = _both(n, blo, bhi)
    assert np.isnan(b_lo[7]) and np.isnan(b_hi[7])
    ok = np.arange(23) != 7
    _close(b_lo[ok], p_lo[ok])
    _close(b_hi[ok], p_hi[ok])
    for b in range(23):
        if b != 7:
            assert_encloses(b_lo[b], b_hi[b], orc(net, blo[b], bhi[b], fac), what=f"box {b}")


def test_batched_c2000_periods():
    net, fac, n = setup("c2000")
    lo, hi, per = synth.period_boxes(net, 18, 8, seed=31)
    b_lo, b_hi, p_lo, p_hi = _both(n, lo, hi)
    _close(b_lo, p_lo)
    _close(b_hi, p_hi)
    for b in (0, 50, 101, 143):
        assert_encloses(b_lo[b], b_hi[b], orc(net, lo[b], hi[b], fac), what=f"box {b}")


def test_batched_c8316_sixteen_boxes():
    net, fac, n = setup("c8316")
    blo, bhi = synth.sub_boxes(net, 16, seed=41)
    b_lo, b_hi, p_lo, p_hi = _both(n, blo, bhi)
    _close(b_lo, p_lo)
    _close(b_hi, p_hi)
    for b in (0, 15):
        assert_encloses(b_lo[b], b_hi[b], orc(net, blo[b], bhi[b], fac), what=f"box {b}")


def test_vector_and_matrix_core_base_flows_agree(monkeypatch):
    """The box-tiled base flows run on the float64 matrix cores by default;
    IBP_TILE=k2b=0 at network build selects the vector-FMA kernel.  Both sum
    the same float64 products in different orders, so the bounds agree to
    summation order and both enclose the oracle.  45 boxes: ragged against the
    32-box MFMA tile and the 16-box vector group."""
    net, fac, n = setup("c500")
    monkeypatch.setenv("IBP_TILE", "k2b=0")
    nv = ibp.Network(net, device=0)
    monkeypatch.delenv("IBP_TILE")
    blo, bhi = synth.sub_boxes(net, 45, seed=77)
    m_lo, m_hi = gpu_bounds(n, blo, bhi)
    v_lo, v_hi = gpu_bounds(nv, blo, bhi)
    _close(m_lo, v_lo)
    _close(m_hi, v_hi)
    for b in (0, 31, 32, 44):
        r = orc(net, blo[b], bhi[b], fac)
        assert_encloses(m_lo[b], m_hi[b], r, what=f"matrix cores, box {b}")
        assert_encloses(v_lo[b], v_hi[b], r, what=f"vector FMA, box {b}")
