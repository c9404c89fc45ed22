"""Per-box error budget of the library's float32 bounds, for the parity tests.

Test infrastructure (imports the oracle).  The library computes in float32 with
outward padding: radii are inflated for every rounding, for the float32 storage
of the factors and for the float64 construction error of the PTDF.  Its
interval is therefore wider than the oracle's float64 interval by an amount
that scales with the magnitudes the padding covers, not with |f|.  For one
post-outage element (k, l) the pads add up to at most 4 u (u = 2^-24) times

    sigma_e = A_l + |c_l| + fmax_l + |LODF_lk| (A_c + |c_c| + r_c),

where c_l is line l's base-flow centre, c_c and r_c the outaged line's centre
and radius, and A_l = sum_n |Phi_ln| (|c_n| + r_n) the absolute base flow on
line l.  Term by term: the base-flow radius carries u |Phi| (|c_n| + r_n) for
the float32 PTDF and the float32 injections (2 u A_l); rounding the line centre
to float32 and the element's own float32 operations add u |c_l| three times and
2 u fmax_l; the outaged line's flow enters through |LODF| with the same terms
plus the float32 storage of the factor itself (4 u A_c + 3 u |c_c| + 3 u r_c).
For a base-case line the pads are below 4 u sigma_l, sigma_l = A_l + |c_l| +
fmax_l.  The float64 construction error of the PTDF (e = the library's
a-posteriori bound on |Phi64 - Phi_exact|) adds, without a factor u,
e sum_n (|c_n| + r_n) per line radius, that times (1 + |LODF|) per element, and
2 e (V + |LODF| (|c_c| + r_c) / (1 - H_cc)) per element for the outage factors
built from the PTDF, V = max_k (|c_c| + r_c) / (1 - H_cc).

Only elements whose penalty can be positive somewhere in the padded interval
contribute (the rest are zero on both sides).  The budget of one side is
zeta_f times the sum of those pads, plus the float32 summation of the outage
penalties (8 u of their sum), the float64 sums of the surplus, imbalance and
penalties (64 u64 per addition level of every term) and, with piecewise-linear
curves, the curve padding.

``floor_*``: what no method that reads float32 factors can avoid.  A float32
copy of a factor fixes the float64 value only to within u of its magnitude, so
over the elements whose penalty is active the bound must leave room for
u (A_l + |LODF| (A_c + |c_c| + r_c)) each (first order), and u A_l per base line.
"""
import math

import numpy as np

import oracle

U32 = 2.0 ** -24
U64 = 2.0 ** -53
K_ELEM = 4.0   # per-element pad, units of u sigma_e
K_LINE = 4.0   # per-line pad, units of u sigma_l

_lodf_cache = {}


def _lodf(net, fac):
    key = id(fac)
    if key not in _lodf_cache:
        _lodf_cache[key] = (fac, oracle.lodf(net, fac))
    return _lodf_cache[key][1]


def _curve_pad(net, lo, hi):
    if net.get("seg_ptr") is None:
        return 0.0
    ptr = np.asarray(net["seg_ptr"])
    a, b, U = (np.asarray(net[k], float) for k in ("seg_a", "seg_b", "seg_U"))
    c = 0.5 * (np.asarray(lo, float) + np.asarray(hi, float))
    r = 0.5 * (np.asarray(hi, float) - np.asarray(lo, float))
    tot = 0.0
    for j in range(ptr.size - 1):
        s0, s1 = int(ptr[j]), int(ptr[j + 1])
        if s1 == s0:
            continue
        T = np.sum(np.abs(a[s0:s1]) * (abs(c[j]) + np.abs(b[s0:s1]) + r[j]))
        Uf = U[s0:s1][np.isfinite(U[s0:s1])]
        Um = float(np.max(np.abs(Uf))) if Uf.size else 0.0
        tot += 16.0 * (s1 - s0 + 6) * U64 * (T + Um)
    return tot


def budget(net, fac, lo, hi, phi_err, chunk=256, near=False):
    """Error budget of each side for one box.

    ``phi_err``: the library's bound on the float64 PTDF error (network info
    ``phi_abs_err``).  Returns ``hi`` / ``lo`` (the largest gap the padding
    rules allow between the library's f_hi (f_lo) and the oracle's),
    ``floor_hi`` / ``floor_lo``, the term scales ``T_hi`` / ``T_lo`` and the
    oracle's result under ``r``.  With ``near``, also ``near_hi`` / ``near_lo``:
    the outage elements (k, l) and base lines l whose penalty's activity on
    that side is within one pad of switching (|pre-activation - limit| or, for
    an active element, |centre| within its pad), as lists of (k or -1, l)."""
    r = oracle.ibp(net, lo, hi, fac, keep_intermediates=True)
    lodf = _lodf(net, fac)
    Phi = fac["Phi"]
    ctg = fac["ctg"]
    c_f, r_f = r["c_f"], r["r_f"]
    ab = np.abs(r["c_inj"]) + r["r_inj"]
    A = np.abs(Phi) @ ab
    Eline = phi_err * float(np.sum(ab)) * (1.0 + 1e-9)
    fb = np.asarray(net["fmax_base"], float)
    fc = np.asarray(net["fmax_ctg"], float)
    zi, zf = float(net["zeta_inj"]), float(net["zeta_f"])
    a = np.abs(c_f)

    # base lines
    s_l = A + a + fb
    pad_l = K_LINE * U32 * s_l + Eline
    Mb_hi = math.fsum(pad_l[a + r_f - fb > -pad_l])       # upper penalty (f_lo side)
    Mb_lo = math.fsum(pad_l[a - r_f - fb > -pad_l])       # lower penalty (f_hi side)
    nears = {"hi": [], "lo": []}
    if near:
        for side, t in (("lo", a + r_f - fb), ("hi", a - r_f - fb)):
            sel = (np.abs(t) <= pad_l) | ((t > -pad_l) & (a <= pad_l))
            nears[side] += [(-1, int(l)) for l in np.flatnonzero(sel)]
    Fb_floor_lo = math.fsum((U32 * A)[a - r_f - fb > 0])
    Fb_floor_hi = math.fsum((U32 * A)[a + r_f - fb > 0])

    # outage elements
    K = ctg.size
    if K:
        fr = np.asarray(net["line_from"])[ctg]
        to = np.asarray(net["line_to"])[ctg]
        omh = 1.0 - (Phi[ctg, fr] - Phi[ctg, to])
        V = float(np.max((a[ctg] + r_f[ctg]) / omh))
    Mc_hi, Mc_lo, fl_hi, fl_lo = [], [], [], []
    for k0 in range(0, K, chunk):
        k1 = min(K, k0 + chunk)
        lam = lodf[:, k0:k1].T                             # k x L
        cc = ctg[k0:k1]
        al = np.abs(lam)
        C = c_f[None, :] + lam * c_f[cc][:, None]
        R = r_f[None, :] + al * r_f[cc][:, None]
        mc = (a[cc] + r_f[cc])[:, None]
        pad = K_ELEM * U32 * ((A + a + fc)[None, :] + al * (A[cc][:, None] + mc))
        pad += Eline * (1.0 + al) + 2.0 * phi_err * (V + al * mc / omh[k0:k1, None])
        pad[np.arange(k1 - k0), cc] = 0.0
        aC = np.abs(C)
        Mc_hi.append(float(np.sum(pad[aC + R - fc[None, :] > -pad])))
        Mc_lo.append(float(np.sum(pad[aC - R - fc[None, :] > -pad])))
        if near:
            own = np.zeros_like(pad, dtype=bool)
            own[np.arange(k1 - k0), cc] = True
            for side, t in (("lo", aC + R - fc[None, :]), ("hi", aC - R - fc[None, :])):
                sel = ((np.abs(t) <= pad) | ((t > -pad) & (aC <= pad))) & ~own
                kk, ll = np.nonzero(sel)
                nears[side] += list(zip((kk + k0).tolist(), ll.tolist()))
        fe = U32 * (A[None, :] + al * (A[cc][:, None] + mc))
        fe[np.arange(k1 - k0), cc] = 0.0
        fl_hi.append(float(np.sum(fe[aC + R - fc[None, :] > 0])))
        fl_lo.append(float(np.sum(fe[aC - R - fc[None, :] > 0])))

    T_hi = abs(r["S_hi"]) + zi * r["I_lo"] + zf * (r["Fb_lo"] + r["Fc_lo"])
    T_lo = abs(r["S_lo"]) + zi * r["I_hi"] + zf * (r["Fb_hi"] + r["Fc_hi"])
    levels = 4096 + fac["L"] + K + 2 * (np.asarray(lo).size + fac["N"])
    common = 64.0 * levels * U64 * (T_hi + T_lo + zi * float(np.sum(ab))) + _curve_pad(net, lo, hi)
    b_hi = zf * (math.fsum(Mc_lo) + Mb_lo + 8.0 * U32 * r["Fc_lo"]) + common
    b_lo = zf * (math.fsum(Mc_hi) + Mb_hi + 8.0 * U32 * r["Fc_hi"]) + common
    out = dict(hi=b_hi, lo=b_lo, floor_hi=zf * (math.fsum(fl_lo) + Fb_floor_lo),
               floor_lo=zf * (math.fsum(fl_hi) + Fb_floor_hi), T_hi=T_hi, T_lo=T_lo, r=r)
    if near:
        out["near_hi"], out["near_lo"] = nears["hi"], nears["lo"]
    return out


def flip_allowance(net, fac, near):
    """How much the gradient of one bound can move, per box endpoint, if the
    float32 activity decision of each listed element differs from the
    oracle's float64 one: a flip adds or removes zeta_f times the element's
    pre-activation gradient, and a centre whose sign is uncertain changes it by
    twice its centre part; summed in absolute value over the elements.
    ``near``: (k or -1, l) pairs from budget(..., near=True).  Returns
    (allow_lo, allow_hi), one entry per input, for d/d lo_j and d/d hi_j."""
    Phi = fac["Phi"]
    ctg = fac["ctg"]
    gb, lb = np.asarray(net["gen_bus"]), np.asarray(net["load_bus"])
    X = gb.size + lb.size
    W = np.zeros((int(net["n_bus"]), X))                   # bus injection per input: +1 generators, -1 loads
    W[gb, np.arange(gb.size)] = 1.0
    W[lb, gb.size + np.arange(lb.size)] = -1.0
    zf = float(net["zeta_f"])
    acc_c = np.zeros(X)
    acc_r = np.zeros(X)
    if near:
        lodf = _lodf(net, fac)
        for k, l in near:
            if k < 0:
                gc, gr = Phi[l], np.abs(Phi[l])
            else:
                c = ctg[k]
                lam = lodf[l, k]
                gc = Phi[l] + lam * Phi[c]
                gr = np.abs(Phi[l]) + abs(lam) * np.abs(Phi[c])
            acc_c += 2.0 * np.abs(W.T @ gc)
            acc_r += np.abs(W).T @ gr
    allow_lo = 0.5 * zf * (acc_c + acc_r)
    allow_hi = 0.5 * zf * (acc_c + acc_r)
    return allow_lo, allow_hi


def crown_near_allowance(net, fac, lo, hi, near_rel=1e-5, chunk=256):
    """How far the box-slope linear relaxation of the upper bound can move if
    the slope decisions the oracle reports as near their switch (within
    near_rel of |c| + r + t, the criterion of oracle.crown_upper) go the other
    way.  Switching one element between s = sign(c) and s = 0 changes its line
    by sign(c) z - t, which over the element's interval [c - r, c + r] stays
    within 2 r + | |c| - r - t | of zero; the bound (a maximum of the sum of
    lines over the box) moves by at most the weight times that.  Returns
    (number of near elements, allowance in $), summed over the imbalance
    (weight zeta_inj, t = 0), the base lines and the outage elements (zeta_f)."""
    r0 = oracle.ibp(net, lo, hi, fac, keep_intermediates=True)
    c_inj, r_inj = r0["c_inj"], r0["r_inj"]
    zi, zf = float(net["zeta_inj"]), float(net["zeta_f"])
    count, allow = 0, 0.0

    def near(c, r, t, w):
        m = np.abs(c) - r - t
        sel = (np.abs(m) <= near_rel * (np.abs(c) + r + t)) & (c != 0)
        return int(np.sum(sel)), w * float(np.sum((2.0 * r + np.abs(m))[sel]))

    W2 = oracle.ibp_oracle._imbalance_matrix(net)
    n, a = near(W2 @ c_inj, abs(W2) @ r_inj, 0.0, zi)
    count, allow = count + n, allow + a
    n, a = near(r0["c_f"], r0["r_f"], np.asarray(net["fmax_base"], float), zf)
    count, allow = count + n, allow + a
    M, Bm, K = fac["M"], fac["B"], fac["K"]
    fc = np.asarray(net["fmax_ctg"], float)
    for k0 in range(0, K, chunk):
        k1 = min(K, k0 + chunk)
        Mk, Bk = M[k0:k1], Bm[k0:k1]
        Cc = Mk * r0["c_f"][None, :] - Bk * r0["c_u"][k0:k1, None]
        Rc = np.abs(Mk) * r0["r_f"][None, :] + np.abs(Bk) * r0["r_u"][k0:k1, None]
        Cc = np.where(Mk != 0, Cc, 0.0)       # the outaged line's own entry has no penalty
        n, a = near(Cc, Rc, fc[None, :], zf)
        count, allow = count + n, allow + a
    return count, allow
