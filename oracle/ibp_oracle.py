"""FP64 CPU oracle: interval bound propagation (IBP) through the SC-DCOPF graph.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run this module.  The product
path (the HIP library and its Python binding) never calls it, and this module
imports nothing from the product package: it takes a network as a plain dict
of numpy arrays (keys as produced by the seeded instance generator) and float32
box endpoints, and computes everything itself in float64 with numpy/scipy.

What it computes (paper: "Fast and Certified Bounding of Security-Constrained
DCOPF via Interval Bound Propagation", Tekeler, Chevalier, Zhong, Zhang):

* DC power-flow maps and the reduced PTDF, Sec. II-A, eqs. (DCPF mappings) and
  (line flow ptdf); the full PTDF pads the slack column with zeros.
* Device-to-bus maps N_g, N_d and the net injection p_inj = N_g p_g - N_d p_d,
  Sec. II-A.
* Nodal-imbalance expression s_inj = |(E^T Phi - I) p_inj|, Sec. III-A eq.
  (slack-sinj); base overload s_fb = max(|Phi p_inj| - p_fb^max, 0), eq.
  (slack-sfb).
* Contingency flows in the paper's loop-free form
  P_fc = M (x) 1 (Phi p)^T - B (x) (U p) 1^T, Sec. III-A eq. (ctg flow matrix
  form), with b_i = M_i Y_D E_r u_i g_i, u_i = Y_Br^{-1} e_i,
  g_i = y_i / (1 + e_i^T u_i y_i), y_i = -(Y_D)_ii, Sec. II-C eqs.
  (nodal admittance rank-1 update) and (ctg flow simplified).
* Overloads S_fc = max(|P_fc| - 1 p_fc^max^T, 0) and s_agg = 1^T S_fc 1,
  eqs. (slack-Sc), (slack-sagg).
* Objective f_ibp, Appendix eq. (ibp_f) (= eq. (penalized-objective)) with
  linear costs, and its IBP enclosure over the box of eq. (f-ibp), using the
  centre-radius rule of Sec. III-C eq. (IBP) for every affine node and the
  tight interval absolute value for |.| (readings listed below).
* Optional piecewise-linear cost (generators) and value (loads) curves of
  Sec. III-B, eqs. (single ReLU) and (combined ReLUs): F*_0 = 0,
  F*_i(x) = min(F*_{i-1}(x) + a_i ReLU(x - b_i), U_i); the surplus adds
  F* of every load and subtracts F* of every generator, beside the linear
  terms.  IBP takes the curve node by node.
* A linear-relaxation (CROWN-style) upper bound on max f (``crown_upper``):
  each convex penalty replaced by a global linear minorant whose slope comes
  from its IBP pre-activation interval, then the exact maximum of the
  resulting linear function over the box.
* Its counterpart for the lower bound (``crown_lower``): each penalty replaced
  by its chord over the IBP pre-activation interval (a linear majorant there),
  then the exact minimum of the resulting linear function over the box.

Readings taken where the paper is silent:

* Slack bus: an explicit parameter (``slack_bus``); row/column removed from
  the reduced matrices.
* E^T Phi - I: its exact value is -e_slack 1^T (the non-slack rows of
  E_r^T Phi_r are the identity and the columns of E^T sum to zero); the oracle
  uses that exact matrix, and a test checks it against the numerically formed
  product.
* |.| under IBP: tight interval magnitude |c| + r and mignitude
  max(|c| - r, 0); max(. - fmax, 0) is monotone and applied to both ends.
* Two penalty weights: zeta_inj on s_inj, zeta_f on both base and
  contingency overloads (as eq. (penalized-objective) is written).
* Islanding outages (1 - H_cc = 0) are excluded; the default contingency set
  is every line whose removal leaves the network connected, ascending.
* Reductions: numpy pairwise sums per chunk, combined with math.fsum.
* Gradient: sign(0) = 0; max(z, 0) is active iff z > 0; min(x, U) passes the
  gradient to x iff x <= U (min(x, U) = x - max(x - U, 0)).

Parity pins live in tests/test_oracle_*.py.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla

__all__ = [
    "incidence",
    "reduced_admittance",
    "factors",
    "islanding_lines",
    "lodf",
    "ibp",
    "ibp_lodf_form",
    "grad",
    "point_eval",
    "point_eval_many",
    "center_radius",
    "curve_value",
    "curve_interval",
    "crown_upper",
    "crown_upper_iterated",
    "crown_lower",
]


# ----------------------------------------------------------------------------
# network matrices (Sec. II-A)
# ----------------------------------------------------------------------------

def _n_line(net):
    return int(np.asarray(net["line_from"]).size)


def incidence(net) -> sp.csr_matrix:
    """Branch-bus incidence E (L x N): +1 at the from bus, -1 at the to bus."""
    L = _n_line(net)
    N = int(net["n_bus"])
    rows = np.repeat(np.arange(L), 2)
    cols = np.stack([np.asarray(net["line_from"]), np.asarray(net["line_to"])], 1).ravel()
    vals = np.tile([1.0, -1.0], L)
    return sp.csr_matrix((vals, (rows, cols)), shape=(L, N))


def reduced_admittance(net, line_b=None):
    """(E_r, Y_D, Y_Br, keep): E_r drops the slack column, Y_Br = E_r^T Y_D E_r.

    Sec. II-A: p_inj,r = Y_Br theta_r and p_f = Y_D E_r theta_r.  ``line_b``
    overrides the susceptances (used to take a line out for direct N-1 flows).
    """
    N = int(net["n_bus"])
    s = int(net["slack_bus"])
    keep = np.array([n for n in range(N) if n != s], dtype=np.int64)
    E = incidence(net)
    E_r = E[:, keep].tocsc()
    b = np.asarray(net["line_b"] if line_b is None else line_b, dtype=np.float64)
    Y_D = sp.diags(b)
    Y_Br = (E_r.T @ Y_D @ E_r).tocsc()
    return E_r, Y_D, Y_Br, keep


def _injection_map(net) -> sp.csr_matrix:
    """W_inj (N x X) with p_inj = N_g p_g - N_d p_d, inputs ordered gens then loads."""
    N = int(net["n_bus"])
    gb = np.asarray(net["gen_bus"])
    lb = np.asarray(net["load_bus"])
    G, D = gb.size, lb.size
    rows = np.concatenate([gb, lb])
    cols = np.arange(G + D)
    vals = np.concatenate([np.ones(G), -np.ones(D)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, G + D))


def islanding_lines(net) -> np.ndarray:
    """Mask of lines whose single outage disconnects the network.

    Brute force: remove each line in turn and count connected components.
    """
    N = int(net["n_bus"])
    fr = np.asarray(net["line_from"])
    to = np.asarray(net["line_to"])
    L = fr.size
    out = np.zeros(L, dtype=bool)
    for l in range(L):
        m = np.ones(L, dtype=bool)
        m[l] = False
        g = sp.coo_matrix((np.ones(m.sum()), (fr[m], to[m])), shape=(N, N))
        ncomp, _ = csgraph.connected_components(g, directed=False)
        out[l] = ncomp > 1
    return out


def _spd_inverse(A: np.ndarray) -> np.ndarray:
    """Inverse of a symmetric positive definite matrix (LAPACK potrf + potri)."""
    c, info = scipy.linalg.lapack.dpotrf(A, lower=1, clean=1, overwrite_a=0)
    if info != 0:
        raise np.linalg.LinAlgError("reduced admittance matrix is not positive definite "
                                    "(is the network connected?)")
    inv, info = scipy.linalg.lapack.dpotri(c, lower=1, overwrite_c=1)
    if info != 0:
        raise np.linalg.LinAlgError("potri failed")
    inv = np.tril(inv) + np.tril(inv, -1).T
    return inv


def factors(net, with_paper_form: bool = True) -> dict:
    """Everything the IBP graph needs that depends on the network only.

    * ``Phi`` (L x N): Phi_r = Y_D E_r (E_r^T Y_D E_r)^{-1}, padded with a zero
      slack column, eq. (line flow ptdf).
    * ``ctg`` (K,): outaged line of each contingency.
    * ``U`` (K x N): rows u'_i = [0 u_i^T] (slack entry zero), u_i = Y_Br^{-1} e_i.
    * ``B`` (K x L): rows b_i = M_i Y_D E_r u_i g_i, g_i = y_i/(1 + e_i^T u_i y_i).
    * ``M`` (K x L): all ones except the outaged line, Sec. III-A.
    """
    N = int(net["n_bus"])
    L = _n_line(net)
    E_r, Y_D, Y_Br, keep = reduced_admittance(net)
    if N > 1:
        ncomp, _ = csgraph.connected_components(
            sp.coo_matrix((np.ones(L), (np.asarray(net["line_from"]), np.asarray(net["line_to"]))),
                          shape=(N, N)), directed=False)
        if ncomp > 1:
            raise ValueError("network is not connected")
    Binv = _spd_inverse(Y_Br.toarray())
    YE = (Y_D @ E_r).tocsr()
    Phi_r = np.asarray(YE @ Binv)                      # L x (N-1)
    Phi = np.zeros((L, N))
    Phi[:, keep] = Phi_r
    b = np.asarray(net["line_b"], dtype=np.float64)

    if net.get("ctg_line") is not None:
        ctg = np.asarray(net["ctg_line"], dtype=np.int64)
        if ctg.size and (ctg.min() < 0 or ctg.max() >= L):
            raise ValueError("contingency line out of range")
        if np.unique(ctg).size != ctg.size:
            raise ValueError("duplicate contingency line")
    else:
        ctg = np.flatnonzero(~islanding_lines(net)).astype(np.int64)
    K = ctg.size
    out = dict(Phi=Phi, ctg=ctg, keep=keep, Binv=Binv, L=L, N=N, K=K)
    if not with_paper_form:
        return out
    # u_i = Y_Br^{-1} e_i with e_i the i-th row of E_r (as a column)
    E_r_csr = E_r.tocsr()
    Er_rows = E_r_csr[ctg].toarray()                    # K x (N-1)
    U_r = Er_rows @ Binv                                # K x (N-1); Binv symmetric
    y = -b[ctg]
    eu = np.einsum("kn,kn->k", Er_rows, U_r)           # e_i^T u_i
    denom = 1.0 + eu * y
    if K and np.min(np.abs(denom)) < 1e-9:
        raise ValueError("an outage islands the network (1 + e^T u y = 0)")
    g = y / denom
    Bm = np.asarray(YE @ U_r.T).T * g[:, None]          # rows Y_D E_r u_i g_i
    M = np.ones((K, L))
    M[np.arange(K), ctg] = 0.0
    Bm = M * Bm
    U = np.zeros((K, N))
    U[:, keep] = U_r
    out.update(U=U, B=Bm, M=M, g=g)
    return out


def lodf(net, fac) -> np.ndarray:
    """Line outage distribution factors (L x K): LODF[l, k] = H[l, c] / (1 - H[c, c]),
    H[:, m] = Phi[:, from(m)] - Phi[:, to(m)], c = outaged line of contingency k.

    The classical rule; the tests use it to check the paper-form factors
    (M, B, U) of Sec. III-A, to which it is algebraically identical."""
    Phi = fac["Phi"]
    ctg = fac["ctg"]
    fr = np.asarray(net["line_from"])[ctg]
    to = np.asarray(net["line_to"])[ctg]
    H = Phi[:, fr] - Phi[:, to]                          # L x K
    Hcc = H[ctg, np.arange(ctg.size)]
    return H / (1.0 - Hcc)[None, :]


# ----------------------------------------------------------------------------
# IBP (Sec. III-C) through the graph of Sec. III-A / Appendix
# ----------------------------------------------------------------------------

def center_radius(lo, hi):
    """x_mu = (hi + lo)/2, x_sigma = (hi - lo)/2 in float64 (exact for float32 inputs)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if not (np.all(np.isfinite(lo)) and np.all(np.isfinite(hi))):
        raise ValueError("box endpoints must be finite")
    if np.any(lo > hi):
        raise ValueError("box has lo > hi")
    return 0.5 * (hi + lo), 0.5 * (hi - lo)


def _abs_interval(c, r):
    """Tight interval |.|: (mignitude, magnitude)."""
    a = np.abs(c)
    return np.maximum(a - r, 0.0), a + r


def _fsum_pairwise(x) -> float:
    return float(np.sum(x))


def _imbalance_matrix(net) -> sp.csr_matrix:
    """E^T Phi - I in closed form: -1 in every column of the slack row, else 0."""
    N = int(net["n_bus"])
    s = int(net["slack_bus"])
    return sp.csr_matrix((-np.ones(N), (np.full(N, s), np.arange(N))), shape=(N, N))


# ----------------------------------------------------------------------------
# piecewise-linear curves (Sec. III-B, eqs. (single ReLU) and (combined ReLUs))
# ----------------------------------------------------------------------------

def _curves(net):
    """Segment lists per input as (ptr, a, b, U), or None for linear costs only."""
    ptr = net.get("seg_ptr")
    if ptr is None:
        return None
    return (np.asarray(ptr, dtype=np.int64), np.asarray(net["seg_a"], float),
            np.asarray(net["seg_b"], float), np.asarray(net["seg_U"], float))


def curve_value(a, b, U, x):
    """F*(x) at points x (scalar or array): F*_0 = 0 and
    F*_i = min(F*_{i-1} + a_i ReLU(x - b_i), U_i) for i = 1..n."""
    F = np.zeros_like(np.asarray(x, dtype=np.float64))
    for ai, bi, Ui in zip(a, b, U):
        F = np.minimum(F + ai * np.maximum(x - bi, 0.0), Ui)
    return F


def curve_interval(a, b, U, c, r):
    """IBP of F* over [c - r, c + r], node by node: the affine node a_i (x - b_i)
    by eq. (IBP) (centre a_i (c - b_i), radius |a_i| r), then the ReLU and the
    min with U_i (monotone, so applied to both ends), and the sum with the
    running interval of F*_{i-1}."""
    lo = hi = 0.0
    for ai, bi, Ui in zip(a, b, U):
        cy = ai * (c - bi)
        ry = abs(ai) * r
        lo = min(lo + max(cy - ry, 0.0), Ui)
        hi = min(hi + max(cy + ry, 0.0), Ui)
    return lo, hi


def _curve_vjp(a, b, U, c, r, d_lo, d_hi):
    """Adjoint of (c, r) for the upstream adjoints (d_lo, d_hi) of curve_interval's
    output; returns (dc, dr, near-kink count)."""
    n = len(a)
    cys, rys, plo, phi = [], [], [], []
    lo = hi = 0.0
    for ai, bi, Ui in zip(a, b, U):
        cy = ai * (c - bi)
        ry = abs(ai) * r
        cys.append(cy)
        rys.append(ry)
        plo.append(lo + max(cy - ry, 0.0))
        phi.append(hi + max(cy + ry, 0.0))
        lo = min(plo[-1], Ui)
        hi = min(phi[-1], Ui)
    dc = dr = 0.0
    near = 0
    for i in range(n - 1, -1, -1):
        Ui = U[i]
        d_lo = d_lo if plo[i] <= Ui else 0.0
        d_hi = d_hi if phi[i] <= Ui else 0.0
        near += (abs(plo[i] - Ui) < 1e-9) + (abs(phi[i] - Ui) < 1e-9)
        zl, zh = cys[i] - rys[i], cys[i] + rys[i]
        near += (abs(zl) < 1e-9) + (abs(zh) < 1e-9)
        dcy = (d_lo if zl > 0 else 0.0) + (d_hi if zh > 0 else 0.0)
        dry = -(d_lo if zl > 0 else 0.0) + (d_hi if zh > 0 else 0.0)
        dc += a[i] * dcy
        dr += abs(a[i]) * dry
    return dc, dr, near


def _curve_surplus(net, mu, sg):
    """[lo, hi] of sum over loads of F*_d minus sum over generators of F*_g."""
    cv = _curves(net)
    if cv is None:
        return 0.0, 0.0
    ptr, A, B, U = cv
    G = np.asarray(net["gen_bus"]).size
    los, his = [], []
    for j in range(mu.size):
        s0, s1 = ptr[j], ptr[j + 1]
        if s1 == s0:
            continue
        l, h = curve_interval(A[s0:s1], B[s0:s1], U[s0:s1], mu[j], sg[j])
        if j < G:
            l, h = -h, -l
        los.append(l)
        his.append(h)
    return math.fsum(los), math.fsum(his)


def ibp(net, lo, hi, fac=None, chunk: int = 256, keep_intermediates: bool = False) -> dict:
    """IBP bounds [f_lo, f_hi] of f_ibp over the box [lo, hi] (inputs: gens then loads).

    Returns a dict with ``f_lo``, ``f_hi`` and the interval terms
    ``S`` (surplus), ``I`` (1^T s_inj), ``Fb`` (1^T s_fb), ``Fc`` (s_agg),
    each as ``*_lo``/``*_hi``.
    """
    if fac is None:
        fac = factors(net)
    mu, sg = center_radius(lo, hi)
    G = np.asarray(net["gen_bus"]).size
    W = _injection_map(net)
    c_inj = W @ mu
    r_inj = abs(W) @ sg

    # surplus sum_j c_j(p_d) - sum_i g_i(p_g), linear costs: affine node
    w = np.concatenate([-np.asarray(net["gen_cost"], float), np.asarray(net["load_value"], float)])
    S_c = math.fsum(w * mu)
    S_r = math.fsum(np.abs(w) * sg)

    # s_inj = |(E^T Phi - I) p_inj|, then 1^T s_inj
    W2 = _imbalance_matrix(net)
    cz = W2 @ c_inj
    rz = abs(W2) @ r_inj
    mig, mag = _abs_interval(cz, rz)
    I_lo, I_hi = math.fsum(mig), math.fsum(mag)

    # base flows Phi p_inj and s_fb = max(|.| - fmax, 0)
    Phi = fac["Phi"]
    c_f = Phi @ c_inj
    r_f = np.abs(Phi) @ r_inj
    fb = np.asarray(net["fmax_base"], float)
    mig, mag = _abs_interval(c_f, r_f)
    Fb_lo = math.fsum(np.maximum(mig - fb, 0.0))
    Fb_hi = math.fsum(np.maximum(mag - fb, 0.0))

    # contingency flows P_fc = M (x) 1 (Phi p)^T - B (x) (U p) 1^T
    U, Bm, M = fac["U"], fac["B"], fac["M"]
    c_u = U @ c_inj
    r_u = np.abs(U) @ r_inj
    fc = np.asarray(net["fmax_ctg"], float)
    K = fac["K"]
    parts_lo, parts_hi = [], []
    for k0 in range(0, K, chunk):
        k1 = min(K, k0 + chunk)
        Mk, Bk = M[k0:k1], Bm[k0:k1]
        Cc = Mk * c_f[None, :] - Bk * c_u[k0:k1, None]
        Rc = np.abs(Mk) * r_f[None, :] + np.abs(Bk) * r_u[k0:k1, None]
        mig, mag = _abs_interval(Cc, Rc)
        parts_lo.append(_fsum_pairwise(np.maximum(mig - fc[None, :], 0.0)))
        parts_hi.append(_fsum_pairwise(np.maximum(mag - fc[None, :], 0.0)))
    Fc_lo, Fc_hi = math.fsum(parts_lo), math.fsum(parts_hi)

    zi, zf = float(net["zeta_inj"]), float(net["zeta_f"])
    P_lo, P_hi = _curve_surplus(net, mu, sg)
    S_lo, S_hi = (S_c - S_r) + P_lo, (S_c + S_r) + P_hi
    f_hi = S_hi - zi * I_lo - zf * (Fb_lo + Fc_lo)
    f_lo = S_lo - zi * I_hi - zf * (Fb_hi + Fc_hi)
    out = dict(f_lo=f_lo, f_hi=f_hi, S_lo=S_lo, S_hi=S_hi, I_lo=I_lo, I_hi=I_hi,
               Fb_lo=Fb_lo, Fb_hi=Fb_hi, Fc_lo=Fc_lo, Fc_hi=Fc_hi)
    if keep_intermediates:
        out.update(c_inj=c_inj, r_inj=r_inj, c_f=c_f, r_f=r_f, c_u=c_u, r_u=r_u)
    return out


def ibp_lodf_form(net, lo, hi, fac=None, chunk: int = 256) -> dict:
    """Same bounds through the classical LODF rule f_l + LODF[l, c] f_c, with the
    outaged line's own entry forced to zero.  Only used to check that the
    paper's (M, B, U) form gives identical intervals."""
    if fac is None:
        fac = factors(net)
    base = ibp(net, lo, hi, fac, keep_intermediates=True)
    Lam = lodf(net, fac)                                # L x K
    ctg = fac["ctg"]
    c_f, r_f = base["c_f"], base["r_f"]
    fc = np.asarray(net["fmax_ctg"], float)
    K = ctg.size
    parts_lo, parts_hi = [], []
    for k0 in range(0, K, chunk):
        k1 = min(K, k0 + chunk)
        lam = Lam[:, k0:k1].T                            # k x L
        cc = ctg[k0:k1]
        C = c_f[None, :] + lam * c_f[cc][:, None]
        R = r_f[None, :] + np.abs(lam) * r_f[cc][:, None]
        C[np.arange(k1 - k0), cc] = 0.0
        R[np.arange(k1 - k0), cc] = 0.0
        mig, mag = _abs_interval(C, R)
        parts_lo.append(_fsum_pairwise(np.maximum(mig - fc[None, :], 0.0)))
        parts_hi.append(_fsum_pairwise(np.maximum(mag - fc[None, :], 0.0)))
    Fc_lo, Fc_hi = math.fsum(parts_lo), math.fsum(parts_hi)
    zi, zf = float(net["zeta_inj"]), float(net["zeta_f"])
    f_hi = base["S_hi"] - zi * base["I_lo"] - zf * (base["Fb_lo"] + Fc_lo)
    f_lo = base["S_lo"] - zi * base["I_hi"] - zf * (base["Fb_hi"] + Fc_hi)
    return dict(f_lo=f_lo, f_hi=f_hi, Fc_lo=Fc_lo, Fc_hi=Fc_hi)


# ----------------------------------------------------------------------------
# analytic vector-Jacobian product of (f_lo, f_hi) w.r.t. the box endpoints
# ----------------------------------------------------------------------------

def grad(net, lo, hi, g_lo: float = 1.0, g_hi: float = 0.0, fac=None, chunk: int = 256):
    """d(g_lo f_lo + g_hi f_hi) / d(lo, hi) of the IBP map above.

    Subgradient convention: sign(0) = 0, max(z, 0) active iff z > 0.  Returns
    (d_lo, d_hi) float64 arrays of length X and a count of elements that sit
    within 1e-9 of a kink (callers use it to decide if a finite difference is
    meaningful).
    """
    if fac is None:
        fac = factors(net)
    mu, sg = center_radius(lo, hi)
    W = _injection_map(net)
    Wa = abs(W)
    c_inj = W @ mu
    r_inj = Wa @ sg
    zi, zf = float(net["zeta_inj"]), float(net["zeta_f"])
    near = 0

    # surplus: f_hi gets S_c + S_r, f_lo gets S_c - S_r
    w = np.concatenate([-np.asarray(net["gen_cost"], float), np.asarray(net["load_value"], float)])
    d_mu = (g_lo + g_hi) * w
    d_sg = (g_hi - g_lo) * np.abs(w)
    cv = _curves(net)
    if cv is not None:
        # loads add [F_lo, F_hi] to [S_lo, S_hi]; generators subtract [F_hi, F_lo]
        ptr, A, B, Uc = cv
        G = np.asarray(net["gen_bus"]).size
        for j in range(mu.size):
            s0, s1 = ptr[j], ptr[j + 1]
            if s1 == s0:
                continue
            a_lo, a_hi = (-g_hi, -g_lo) if j < G else (g_lo, g_hi)
            dc, dr, nk = _curve_vjp(A[s0:s1], B[s0:s1], Uc[s0:s1], mu[j], sg[j], a_lo, a_hi)
            d_mu[j] += dc
            d_sg[j] += dr
            near += nk
    d_cinj = np.zeros_like(c_inj)
    d_rinj = np.zeros_like(r_inj)

    def abs_penalty_grads(c, r, thr):
        """d/dc, d/dr of max(|c| + r - thr, 0) [used by f_lo] and of
        max(|c| - r - thr, 0) [used by f_hi], plus near-kink count."""
        a = np.abs(c)
        t_hi = a + r - thr
        t_lo = a - r - thr
        act_hi = (t_hi > 0).astype(float)
        act_lo = (t_lo > 0).astype(float)
        s = np.sign(c)
        nk = int(np.sum(np.abs(t_hi) < 1e-9) + np.sum(np.abs(t_lo) < 1e-9)
                 + np.sum((np.abs(c) < 1e-9) & ((act_hi + act_lo) > 0)))
        dc = -g_lo * s * act_hi - g_hi * s * act_lo
        dr = -g_lo * act_hi + g_hi * act_lo
        return dc, dr, nk

    # imbalance: I_hi = sum |cz| + rz ; I_lo = sum max(|cz| - rz, 0)
    W2 = _imbalance_matrix(net)
    cz = W2 @ c_inj
    rz = abs(W2) @ r_inj
    dcz, drz, nk = abs_penalty_grads(cz, rz, 0.0)
    near += nk
    d_cinj += zi * (W2.T @ dcz)
    d_rinj += zi * (abs(W2).T @ drz)

    Phi = fac["Phi"]
    c_f = Phi @ c_inj
    r_f = np.abs(Phi) @ r_inj
    dcf, drf, nk = abs_penalty_grads(c_f, r_f, np.asarray(net["fmax_base"], float))
    near += nk
    dcf = zf * dcf
    drf = zf * drf

    U, Bm, M = fac["U"], fac["B"], fac["M"]
    c_u = U @ c_inj
    r_u = np.abs(U) @ r_inj
    fc = np.asarray(net["fmax_ctg"], float)
    K = fac["K"]
    dcu = np.zeros(K)
    dru = np.zeros(K)
    for k0 in range(0, K, chunk):
        k1 = min(K, k0 + chunk)
        Mk, Bk = M[k0:k1], Bm[k0:k1]
        Cc = Mk * c_f[None, :] - Bk * c_u[k0:k1, None]
        Rc = np.abs(Mk) * r_f[None, :] + np.abs(Bk) * r_u[k0:k1, None]
        dC, dR, nk = abs_penalty_grads(Cc, Rc, fc[None, :])
        near += nk
        dC *= zf
        dR *= zf
        dcf += np.sum(Mk * dC, axis=0)
        drf += np.sum(np.abs(Mk) * dR, axis=0)
        dcu[k0:k1] = -np.sum(Bk * dC, axis=1)
        dru[k0:k1] = np.sum(np.abs(Bk) * dR, axis=1)

    d_cinj += Phi.T @ dcf + U.T @ dcu
    d_rinj += np.abs(Phi).T @ drf + np.abs(U).T @ dru
    d_mu += W.T @ d_cinj
    d_sg += Wa.T @ d_rinj
    d_lo = 0.5 * (d_mu - d_sg)
    d_hi = 0.5 * (d_mu + d_sg)
    return d_lo, d_hi, near


# ----------------------------------------------------------------------------
# linear-relaxation (CROWN-style) upper bound on max f over the box
# ----------------------------------------------------------------------------

def _crown_slopes(c, r, t, near_rel):
    """Slope s = sign(c) where |c| - r > t (the interval [c - r, c + r] lies on one
    linear piece of max(|z| - t, 0) with non-zero slope), else 0; and the count
    of elements within near_rel of that decision."""
    m = np.abs(c) - r - t
    s = np.sign(c) * (m > 0)
    k = int(np.sum((np.abs(m) <= near_rel * (np.abs(c) + r + t)) & (c != 0)))
    return s, k


def _crown_point_slopes(z, t, near_rel):
    """Slope s = sign(z) where |z| > t at a reference point (the gradient of
    max(|z| - t, 0) there), else 0; and the count within near_rel of that decision."""
    m = np.abs(z) - t
    s = np.sign(z) * (m > 0)
    k = int(np.sum((np.abs(m) <= near_rel * (np.abs(z) + t)) & (z != 0)))
    return s, k


def crown_upper(net, lo, hi, fac=None, chunk: int = 256, near_rel: float = 1e-5, ref=None) -> dict:
    """Upper bound on max f over the box from linear relaxations of the penalties
    (the convex-relaxation family the paper cites beside IBP, Sec. I).

    Every penalty phi(z) = max(|z| - t, 0) of the graph is convex, so for any
    s in {-1, 0, 1} the line s z - |s| t lies below it for every z; the
    imbalance |z| likewise lies above s z.  Replacing each penalty by such a
    line turns -f into a linear function of the inputs plus the surplus, whose
    maximum over the box is exact: sum_j max over x_j of (G_j x_j), plus the
    curve part through its IBP interval.  The slope of an element is the sign
    of its pre-activation interval (IBP, exact for these affine nodes) when the
    whole interval lies beyond the threshold, and 0 otherwise, so each line's
    minimum over the box equals IBP's lower penalty and the bound is never
    above IBP's f_hi.

    With ``ref`` (a point), the slopes are instead the gradients of the
    penalties at that point: sign(z(ref)) where |z(ref)| > t, else 0 (any
    slopes give a valid bound).

    Returns ``f_hi`` (the bound), ``n_active`` (elements with a non-zero
    slope), ``near`` (elements whose slope decision sits within ``near_rel`` of
    switching, relative to |C| + R + t, or |z| + t at the point), and
    ``vertex``: the box vertex maximising the linear part (hi_j where its
    coefficient is >= 0, else lo_j).
    """
    if fac is None:
        fac = factors(net)
    mu, sg = center_radius(lo, hi)
    W = _injection_map(net)
    c_inj = W @ mu
    r_inj = abs(W) @ sg
    zi, zf = float(net["zeta_inj"]), float(net["zeta_f"])
    w = np.concatenate([-np.asarray(net["gen_cost"], float), np.asarray(net["load_value"], float)])
    near = 0
    n_active = 0

    if ref is not None:
        p_ref = W @ np.asarray(ref, dtype=np.float64)

    def slopes(c, r, t, zref=None):
        if ref is not None:
            return _crown_point_slopes(zref, t, near_rel)
        return _crown_slopes(c, r, t, near_rel)

    # imbalance 1^T |(E^T Phi - I) p_inj|: |z| >= s z
    W2 = _imbalance_matrix(net)
    cz = W2 @ c_inj
    rz = abs(W2) @ r_inj
    s_I, k = slopes(cz, rz, 0.0, None if ref is None else W2 @ p_ref)
    near += k
    # base lines
    Phi = fac["Phi"]
    c_f = Phi @ c_inj
    r_f = np.abs(Phi) @ r_inj
    fb = np.asarray(net["fmax_base"], float)
    s_b, k = slopes(c_f, r_f, fb, None if ref is None else Phi @ p_ref)
    near += k
    n_active += int(np.count_nonzero(s_b))
    const = [zf * math.fsum(np.abs(s_b) * fb)]
    # contingency elements, paper form z = M f - B (U p)
    U, Bm, M = fac["U"], fac["B"], fac["M"]
    c_u = U @ c_inj
    r_u = np.abs(U) @ r_inj
    fc = np.asarray(net["fmax_ctg"], float)
    K = fac["K"]
    v_f = s_b.astype(float).copy()
    v_u = np.zeros(K)
    if ref is not None:
        f_ref = Phi @ p_ref
        u_ref = U @ p_ref
    for k0 in range(0, K, chunk):
        k1 = min(K, k0 + chunk)
        Mk, Bk = M[k0:k1], Bm[k0:k1]
        Cc = Mk * c_f[None, :] - Bk * c_u[k0:k1, None]
        Rc = np.abs(Mk) * r_f[None, :] + np.abs(Bk) * r_u[k0:k1, None]
        zr = None if ref is None else Mk * f_ref[None, :] - Bk * u_ref[k0:k1, None]
        s, k = slopes(Cc, Rc, fc[None, :], zr)
        s = s * (Mk != 0)          # the outaged line's own entry carries no penalty
        near += k
        n_active += int(np.count_nonzero(s))
        const.append(zf * _fsum_pairwise(np.abs(s) * fc[None, :]))
        v_f += np.sum(Mk * s, axis=0)
        v_u[k0:k1] = -np.sum(Bk * s, axis=1)
    # coefficient of x in the relaxed objective: surplus - zeta_inj s_I z_I - zeta_f sum s z
    G = w - zi * (W.T @ (W2.T @ s_I)) - zf * (W.T @ (Phi.T @ v_f + U.T @ v_u))
    P_lo, P_hi = _curve_surplus(net, mu, sg)
    c0 = math.fsum(const)
    f_hi = c0 + math.fsum(G * mu) + math.fsum(np.abs(G) * sg) + P_hi
    vertex = np.where(G >= 0, np.asarray(hi, np.float64), np.asarray(lo, np.float64))
    return dict(f_hi=f_hi, n_active=n_active, near=near, G=G, const=c0, vertex=vertex)


def _chord(c, r, t):
    """Chord of phi(z) = max(|z| - t, 0) over [c - r, c + r]: slope a and
    intercept b of the line through (z_lo, phi(z_lo)) and (z_hi, phi(z_hi)).
    phi is convex, so the chord lies above it on the whole interval.  A
    zero-width interval gets a = 0, b = phi(c)."""
    zl, zu = c - r, c + r
    pl = np.maximum(np.abs(zl) - t, 0.0)
    pu = np.maximum(np.abs(zu) - t, 0.0)
    w = zu - zl
    pos = w > 0
    a = np.where(pos, (pu - pl) / np.where(pos, w, 1.0), 0.0)
    b = np.where(pos, pl - a * zl, pl)
    return a, b


def crown_lower(net, lo, hi, fac=None, chunk: int = 256, keep_slopes: bool = False) -> dict:
    """Lower bound on min f over the box from linear relaxations of the
    penalties (the convex-relaxation family the paper cites beside IBP, Sec. I),
    the counterpart of ``crown_upper`` for f_lo.

    Every penalty phi(z) = max(|z| - t, 0) (and the imbalance |z|, t = 0) is
    convex, so on its IBP pre-activation interval [C - R, C + R] (the same
    centre-radius intervals ``ibp`` forms, exact for these affine nodes) it
    lies below its chord a z + b.  Hence f(x) >= S(x) - zeta_inj (a_I z_I(x) +
    b_I) - zeta_f sum_e (a_e z_e(x) + b_e) for every x in the box; the right
    side is linear in x (plus the curve part) and its minimum over the box is
    exact: sum_j (G_j c_j - |G_j| r_j) + const, with the curve part through its
    IBP interval.  Because the minimum of a sum is at least the sum of the
    minima and each chord's maximum over its interval is IBP's upper penalty,
    the bound is never below IBP's f_lo.

    Returns ``f_lo``, ``G`` (coefficients of x), ``const``, ``n_active``
    (elements with a non-zero slope) and ``vertex`` (lo_j where G_j >= 0, else
    hi_j: the minimiser of the linear part).  With ``keep_slopes`` also the
    slopes and intercepts: ``chord_imb`` (a_I, b_I), ``chord_base`` (a, b per
    line) and ``chord_ctg`` (a, b as K x L arrays; the outaged line's own entry
    is 0).
    """
    if fac is None:
        fac = factors(net)
    mu, sg = center_radius(lo, hi)
    W = _injection_map(net)
    c_inj = W @ mu
    r_inj = abs(W) @ sg
    zi, zf = float(net["zeta_inj"]), float(net["zeta_f"])
    w = np.concatenate([-np.asarray(net["gen_cost"], float), np.asarray(net["load_value"], float)])
    out = {}
    # imbalance 1^T |(E^T Phi - I) p_inj| <= a_I z_I + b_I
    W2 = _imbalance_matrix(net)
    cz = W2 @ c_inj
    rz = abs(W2) @ r_inj
    a_I, b_I = _chord(cz, rz, 0.0)
    const = [-zi * math.fsum(b_I)]
    # base lines
    Phi = fac["Phi"]
    c_f = Phi @ c_inj
    r_f = np.abs(Phi) @ r_inj
    fb = np.asarray(net["fmax_base"], float)
    a_b, b_b = _chord(c_f, r_f, fb)
    const.append(-zf * math.fsum(b_b))
    n_active = int(np.count_nonzero(a_b))
    # contingency elements, paper form z = M f - B (U p)
    U, Bm, M = fac["U"], fac["B"], fac["M"]
    c_u = U @ c_inj
    r_u = np.abs(U) @ r_inj
    fc = np.asarray(net["fmax_ctg"], float)
    K = fac["K"]
    v_f = a_b.copy()
    v_u = np.zeros(K)
    if keep_slopes:
        A_all = np.zeros((K, Phi.shape[0]))
        B_all = np.zeros((K, Phi.shape[0]))
    for k0 in range(0, K, chunk):
        k1 = min(K, k0 + chunk)
        Mk, Bk = M[k0:k1], Bm[k0:k1]
        Cc = Mk * c_f[None, :] - Bk * c_u[k0:k1, None]
        Rc = np.abs(Mk) * r_f[None, :] + np.abs(Bk) * r_u[k0:k1, None]
        a, b = _chord(Cc, Rc, fc[None, :])
        keep = Mk != 0              # the outaged line's own entry carries no penalty
        a = a * keep
        b = b * keep
        n_active += int(np.count_nonzero(a))
        const.append(-zf * _fsum_pairwise(b))
        v_f += np.sum(Mk * a, axis=0)
        v_u[k0:k1] = -np.sum(Bk * a, axis=1)
        if keep_slopes:
            A_all[k0:k1] = a
            B_all[k0:k1] = b
    # coefficient of x in the relaxed objective: surplus - zeta_inj a_I z_I - zeta_f sum a z
    G = w - zi * (W.T @ (W2.T @ a_I)) - zf * (W.T @ (Phi.T @ v_f + U.T @ v_u))
    P_lo, _ = _curve_surplus(net, mu, sg)
    c0 = math.fsum(const)
    f_lo = c0 + math.fsum(G * mu) - math.fsum(np.abs(G) * sg) + P_lo
    vertex = np.where(G >= 0, np.asarray(lo, np.float64), np.asarray(hi, np.float64))
    out.update(f_lo=f_lo, G=G, const=c0, n_active=n_active, vertex=vertex)
    if keep_slopes:
        out.update(chord_imb=(a_I, b_I), chord_base=(a_b, b_b), chord_ctg=(A_all, B_all))
    return out


def crown_upper_iterated(net, lo, hi, fac=None, iters: int = 4, near_rel: float = 1e-5) -> dict:
    """The smallest of several relaxation bounds: the interval slope rule, then
    ``iters`` point-gradient slope rules at reference points x_0 = (lo + hi)/2
    and x_{i+1} = x_i/2 + v_i/2 (float32 arithmetic), where v_i is the vertex
    that maximised relaxation i.  Returns ``f_hi``, the per-relaxation bounds
    and the total ``near`` count."""
    if fac is None:
        fac = factors(net)
    r = crown_upper(net, lo, hi, fac, near_rel=near_rel)
    bounds = [r["f_hi"]]
    near = r["near"]
    half = np.float32(0.5)
    x = half * np.asarray(lo, np.float32) + half * np.asarray(hi, np.float32)
    for _ in range(iters):
        r = crown_upper(net, lo, hi, fac, near_rel=near_rel, ref=x.astype(np.float64))
        bounds.append(r["f_hi"])
        near += r["near"]
        x = half * x + half * r["vertex"].astype(np.float32)
    return dict(f_hi=min(bounds), bounds=bounds, near=near)


# ----------------------------------------------------------------------------
# point evaluation f(x) by direct DC power flow (no PTDF, no LODF, no IBP)
# ----------------------------------------------------------------------------

def point_eval_many(net, X, ctg=None) -> np.ndarray:
    """f(x) of eq. (penalized-objective) with the slacks of Remark 1, at each row of X.

    Base flows come from solving Y_Br theta_r = p_inj,r; the imbalance is the
    literal KCL residual E^T p_f - p_inj (= (E^T Phi - I) p_inj); every
    outage rebuilds Y_Br without the line and solves again.
    """
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    G = np.asarray(net["gen_bus"]).size
    W = _injection_map(net)
    P = W @ X.T                                           # N x n
    E = incidence(net)
    E_r, Y_D, Y_Br, keep = reduced_admittance(net)
    lu = spla.splu(Y_Br.tocsc())
    theta = np.zeros_like(P)
    theta[keep] = lu.solve(np.ascontiguousarray(P[keep]))
    pf = Y_D @ (E @ theta)                                # L x n
    s_inj = np.abs(E.T @ pf - P)
    fb = np.asarray(net["fmax_base"], float)[:, None]
    s_fb = np.maximum(np.abs(pf) - fb, 0.0)
    if ctg is None:
        ctg = factors(net, with_paper_form=False)["ctg"]
    fc = np.asarray(net["fmax_ctg"], float)[:, None]
    b = np.asarray(net["line_b"], float)
    s_fc = np.zeros(X.shape[0])
    for c in ctg:
        bc = b.copy()
        bc[c] = 0.0
        _, YDc, YBc, _ = reduced_admittance(net, line_b=bc)
        luc = spla.splu(YBc.tocsc())
        th = np.zeros_like(P)
        th[keep] = luc.solve(np.ascontiguousarray(P[keep]))
        pfc = YDc @ (E @ th)
        s_fc += np.sum(np.maximum(np.abs(pfc) - fc, 0.0), axis=0)
    w = np.concatenate([-np.asarray(net["gen_cost"], float), np.asarray(net["load_value"], float)])
    surplus = X @ w
    cv = _curves(net)
    if cv is not None:
        ptr, A, B, U = cv
        for j in range(X.shape[1]):
            s0, s1 = ptr[j], ptr[j + 1]
            F = curve_value(A[s0:s1], B[s0:s1], U[s0:s1], X[:, j])
            surplus = surplus - F if j < G else surplus + F
    zi, zf = float(net["zeta_inj"]), float(net["zeta_f"])
    return surplus - zi * s_inj.sum(0) - zf * (s_fb.sum(0) + s_fc)


def point_eval(net, x, ctg=None) -> float:
    return float(point_eval_many(net, np.asarray(x)[None, :], ctg)[0])
