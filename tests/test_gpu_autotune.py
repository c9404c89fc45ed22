"""The box-tiled autotuner (batching over time indices and sub-boxes,
Sec. IV-A): every candidate tile choice gives bounds that enclose the FP64
oracle within the padding budget and agree with the default tiles up to float64
summation order; the tuner's pick and its JSON cache round trip."""
import json
import os

import numpy as np
import pytest

from paper_2511_15624_amd import ibp, synth
from tests.test_gpu_forward import assert_encloses, gpu_bounds, orc, setup

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _close(a, b, rel=1e-6):
    assert np.all(np.abs(a - b) <= rel * np.maximum(np.abs(b), 1.0)), float(np.max(np.abs(a - b)))


@pytest.mark.parametrize("name,nb", [("c500", 37), ("c2000", 64)])
def test_every_candidate_encloses_and_agrees(name, nb):
    net, fac, n = setup(name)
    blo, bhi = synth.sub_boxes(net, nb, seed=515)
    n.set_tile_batched(4, 0, -1, 1, 0)
    d_lo, d_hi = gpu_bounds(n, blo, bhi)
    check = (0, nb // 2, nb - 1)
    refs = {b: orc(net, blo[b], bhi[b], fac) for b in check}
    try:
        for bt in (2, 4, 8):
            for rows in (0, 1, 7):
                for xcd in (0, 1):
                    for mfma, by in ((1, 0), (1, 2), (0, 0)):
                        n.set_tile_batched(bt, rows, xcd, mfma, by)
                        f_lo, f_hi = gpu_bounds(n, blo, bhi)
                        what = f"{name} bt={bt} rows={rows} xcd={xcd} mfma={mfma} by={by}"
                        _close(f_lo, d_lo)
                        _close(f_hi, d_hi)
                        for b in check:
                            assert_encloses(f_lo[b], f_hi[b], refs[b], what=f"{what} box {b}")
    finally:
        n.set_tile_batched(4, 0, -1, 1, 0)


def test_autotune_picks_a_candidate_and_caches_it(tmp_path):
    torch = _torch()
    net, fac, n = setup("c2000")
    blo, bhi = synth.sub_boxes(net, 96, seed=516)
    lo, hi = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    cache = str(tmp_path / "tiles.json")
    try:
        tiles, cached = ibp.ibp_autotune_batched(n, lo, hi, cache=cache)
        assert not cached and tiles["k3_bt"] in (2, 4, 8) and tiles["k2_mfma"] in (0, 1)
        assert tiles["screen_upper"] in (0, 1)
        with open(cache) as f:
            table = json.load(f)
        key = ibp._tile_cache_key(n, 96)
        assert key.endswith("|B128") and table[key]["k3_bt"] == tiles["k3_bt"]
        assert table[key]["screen_upper"] == tiles["screen_upper"]
        n.set_tile_batched(4, 0, -1, 1, 0)
        n.set_screen_upper(1 - tiles["screen_upper"])
        again, cached = ibp.ibp_autotune_batched(n, lo, hi, cache=cache)
        assert cached and again == tiles
        f_lo, f_hi = gpu_bounds(n, blo, bhi)
        for b in (0, 95):
            assert_encloses(f_lo[b], f_hi[b], orc(net, blo[b], bhi[b], fac), what=f"tuned box {b}")
    finally:
        n.set_tile_batched(4, 0, -1, 1, 0)
        n.set_screen_upper(0)
    assert os.path.exists(cache)


@pytest.mark.parametrize("name,nb", [("c500", 37), ("c2000", 70)])
def test_screen_upper_setting_is_the_flag(name, nb):
    """The screen-upper setting makes box-tiled calls that bound f_lo take the
    upper-penalty screen as IBP_F_SCREEN_UPPER does: the same kernels, so the
    same bits; calls bounding f_hi alone are untouched; the workspace those
    calls need grows by the screen's regions."""
    net, fac, n = setup(name)
    blo, bhi = synth.sub_boxes(net, nb, seed=517)
    assert not n.screen_upper()
    base_ws = n.workspace_bytes(nb, 0)
    f2 = gpu_bounds(n, blo, bhi, flags=ibp.IBP_F_SCREEN_UPPER)
    fl = gpu_bounds(n, blo, bhi, flags=ibp.IBP_F_LOWER_ONLY | ibp.IBP_F_SCREEN_UPPER)
    fu = gpu_bounds(n, blo, bhi, flags=ibp.IBP_F_UPPER_ONLY)
    try:
        n.set_screen_upper(1)
        assert n.screen_upper() and n.tiles()["screen_upper"] == 1
        assert n.workspace_bytes(nb, 0) > base_ws
        for got, want in ((gpu_bounds(n, blo, bhi), f2),
                          (gpu_bounds(n, blo, bhi, flags=ibp.IBP_F_LOWER_ONLY), fl),
                          (gpu_bounds(n, blo, bhi, flags=ibp.IBP_F_UPPER_ONLY), fu)):
            np.testing.assert_array_equal(got[0], want[0])
            np.testing.assert_array_equal(got[1], want[1])
    finally:
        n.set_screen_upper(0)
    assert n.workspace_bytes(nb, 0) == base_ws
    for b in (0, nb - 1):
        r = orc(net, blo[b], bhi[b], fac)
        assert_encloses(f2[0][b], f2[1][b], r, what=f"{name} screened box {b}")


def test_tile_environment_sets_the_screen_upper_setting(monkeypatch):
    net = synth.make_config("tiny")
    monkeypatch.setenv("IBP_TILE", "scru=1")
    n = ibp.Network(net, device=0)
    monkeypatch.delenv("IBP_TILE")
    assert n.screen_upper() and n.tiles()["screen_upper"] == 1
    n.close()
    n = ibp.Network(net, device=0)
    assert not n.screen_upper()
    n.close()
