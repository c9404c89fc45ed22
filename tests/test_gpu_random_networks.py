"""GPU parity on seeded random networks of ragged sizes (bus, line, outage and
input counts that are not multiples of the kernels' tiles; many devices on
one bus; piecewise-linear curves on some), single-box and box-tiled calls,
against the FP64 oracle: enclosure and the 1e-5 bar of the forward tests,
the one-sided calls against the two-sided ones, and the chord-relaxation
lower bound (per box and box-tiled) against the oracle's.
"""
import numpy as np
import pytest

import oracle
from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_forward import assert_encloses, gpu_bounds, one_sided_close, orc, register

pytestmark = pytest.mark.gpu

CASES = [
    # (n_bus, n_line, n_gen, n_load, seed, curves)
    (5, 6, 2, 3, 11, False),
    (17, 23, 4, 19, 12, True),
    (33, 47, 9, 40, 13, False),
    (61, 70, 70, 5, 14, True),      # more generators than buses: several per bus
    (97, 131, 12, 150, 15, False),
    (130, 129, 20, 60, 16, False),  # a tree: no outage keeps it connected
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}_l{c[1]}" for c in CASES])
def test_random_network(case):
    n_bus, n_line, n_gen, n_load, seed, curves = case
    net = synth.make_network(n_bus, n_line, n_gen, n_load, seed=seed)
    if curves:
        net = synth.with_pwl_costs(net, seed=seed)
    fac = oracle.factors(net)
    n = ibp.Network(net, device=0)
    register(fac, n)
    lo, hi = synth.full_box(net)
    blo, bhi = synth.sub_boxes(net, 9, seed=seed + 100)
    LO = np.vstack([lo[None], blo])
    HI = np.vstack([hi[None], bhi])
    b_lo, b_hi = gpu_bounds(n, LO, HI)                              # box-tiled
    p_lo, p_hi = gpu_bounds(n, LO, HI, flags=ibp.IBP_F_PLAIN)       # per box
    u_lo, u_hi = gpu_bounds(n, LO, HI, flags=ibp.IBP_F_UPPER_ONLY)
    l_lo, l_hi = gpu_bounds(n, LO, HI, flags=ibp.IBP_F_LOWER_ONLY)
    assert one_sided_close(u_hi, b_hi) and one_sided_close(l_lo, b_lo)
    for b in range(LO.shape[0]):
        r = orc(net, LO[b], HI[b], fac)
        assert u_hi[b] >= r["f_hi"] and l_lo[b] <= r["f_lo"], f"{case} one-sided {b}"
        assert_encloses(b_lo[b], b_hi[b], r, what=f"{case} box-tiled {b}")
        assert_encloses(p_lo[b], p_hi[b], r, what=f"{case} per-box {b}")
    # chord-relaxation lower bound: ten boxes (tiled sweep) and the first alone (per-box sweep)
    from tests.test_gpu_crown_lower import check_box, gpu_lower
    c_lo, c_hi, c = gpu_lower(n, LO, HI)
    c1_lo, c1_hi, c1 = gpu_lower(n, LO[:1], HI[:1])
    for b in range(LO.shape[0]):
        check_box(net, fac, LO[b], HI[b], c_lo[b], c_hi[b], c[b], b_lo[b], b_hi[b], f"{case} chord {b}")
    check_box(net, fac, LO[0], HI[0], c1_lo[0], c1_hi[0], c1[0], p_lo[0], p_hi[0], f"{case} chord single")
