"""Central finite differences of the FP64 oracle's bounds, for gradient checks.

Test infrastructure (imports the oracle).  The IBP map is piecewise linear in
the box endpoints, so a central difference with step h is exact wherever the
map is linear on [x - h, x + h] along that coordinate.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def coordinates(lo, hi, k, h, rng):
    """k seeded (side, input) pairs whose endpoint can move by h both ways and
    stay inside the box (side 0: lo_j, side 1: hi_j)."""
    width = np.asarray(hi, float) - np.asarray(lo, float)
    ok = np.flatnonzero(width > 2.5 * h)
    js = rng.choice(ok, size=min(k, ok.size), replace=False)
    sides = rng.integers(0, 2, size=js.size)
    return list(zip(sides.tolist(), js.tolist()))


def central_differences(net, fac, lo, hi, coords, h, workers=8):
    """(f(x + h e) - f(x - h e)) / 2h of the oracle's f_lo and f_hi for each
    (side, j) coordinate, endpoints moved in float64.  Returns two arrays."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    jobs = []
    for side, j in coords:
        for sgn in (1.0, -1.0):
            a, b = lo.copy(), hi.copy()
            if side == 0:
                a[j] += sgn * h
            else:
                b[j] += sgn * h
            jobs.append((a, b))

    def run(ab):
        r = oracle.ibp(net, ab[0], ab[1], fac)
        return r["f_lo"], r["f_hi"]

    with ThreadPoolExecutor(max_workers=workers) as ex:
        vals = np.array(list(ex.map(run, jobs))).reshape(len(coords), 2, 2)   # coord, sign, (f_lo, f_hi)
    fd = (vals[:, 0, :] - vals[:, 1, :]) / (2.0 * h)
    return fd[:, 0], fd[:, 1]
