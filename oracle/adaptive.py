"""Adaptive subdivision with local re-solve (Sec. 7: Alg. 5, 6 and 7),
written out plainly in FP64.

TEST INFRASTRUCTURE ONLY, like the rest of the package: nothing in the
product path imports, calls or links it.

What is computed:

* Panels of unequal length.  A panel is the piece of curve c between
  normalised arc lengths lo < hi; it carries g Gauss-Legendre nodes at the
  GL roots of its own normalised arc length and s chord segments of equal
  arc length, exactly as the equal panels of the base discretisation
  (App. A, B; Sec. 5.2).
* Legendre tail (Sec. 7.1, Alg. 5): the coefficients of the degree g-1
  Legendre expansion of the nodal density of a panel,
      a_k = (2k+1)/2 sum_i w_i sigma_i P_k(x_i),
  (exact for a polynomial of degree < g sampled at the roots); the tail of a
  panel is max over the colour channels of |a_{g-1}|.
* Subdivision (Alg. 5): a panel whose tail exceeds eps2 and whose arc length
  is at least eps1 is cut at its arc-length midpoint into two panels with g
  nodes each.
* Warm start (Sec. 7.1.1): the old density, Legendre-interpolated from the
  parent panel's nodes to its children's nodes; unchanged panels keep theirs.
* Re-solving curves (Sec. 7.1.4, label_curves): for each subdivided curve
  S_a, v = G_H rho with rho = 1 on S_a and 0 elsewhere (one unit charge per
  length on the curve); a curve S_b is re-solved when
      max(v on S_b) - min(v on S_b) > 0.9 (max(v on S_a) - min(v on S_a)).
  The subdivided curves are re-solved as well.
* Local re-solve (Eq. local_resolve_mat, Alg. 6): with r the re-solving
  and c the constrained (unchanged) nodes,
      (G_H)_rr sigma_r = b_r - (G_H)_rc sigma_c,
  b = (u+ + u-)/2 - F_H mu at the new nodes.

Readings (also listed with the design notes): the tail takes the largest
channel; the right-hand side at the new nodes is computed from the colours
rather than Legendre-interpolated from the old one (the system a global
re-solve would solve; the local re-solve then differs from it only by
holding sigma_c fixed); a panel takes part in the subdivision test only when
one of its chords meets the viewport (curves outside it are the fixed curves
of Sec. 7.4).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg

from . import dcoracle as dco

__all__ = [
    "uniform_panels", "discretize_panels", "legendre_coefficients", "legendre_tails",
    "panel_lengths", "panels_in_viewport", "select_panels", "split_panels",
    "warm_start", "label_curves", "local_resolve", "global_resolve",
]


def uniform_panels(n_curves, panels):
    """Panel list of the base discretisation: P equal panels per curve."""
    curve = np.repeat(np.arange(n_curves), panels)
    p = np.tile(np.arange(panels), n_curves)
    return curve, p / panels, (p + 1.0) / panels


def discretize_panels(ctrl, panel_curve, panel_lo, panel_hi, gl, segs):
    """Nodes, chords and scales of panels of any lengths (App. A, B;
    Sec. 5.2): panel k covers normalised arc length [lo_k, hi_k] of curve
    panel_curve[k]; panels are listed curve by curve, in order along it."""
    ctrl = np.asarray(ctrl, dtype=float)
    panel_curve = np.asarray(panel_curve, dtype=np.int64)
    lo = np.asarray(panel_lo, dtype=float)
    hi = np.asarray(panel_hi, dtype=float)
    n = ctrl.shape[0]
    x_gl, _ = dco.gauss_legendre(gl)
    tau_edge = -1.0 + 2.0 * np.arange(segs + 1) / segs
    lens = np.array([dco.curve_length(ctrl[c]) for c in range(n)])
    node_xy = np.empty((len(lo) * gl, 2))
    node_lam = np.empty(len(lo) * gl)
    p1 = np.empty((len(lo) * segs, 2))
    p2 = np.empty((len(lo) * segs, 2))
    ell = np.empty(len(lo) * segs)
    for c in range(n):
        ks = np.nonzero(panel_curve == c)[0]
        if ks.size == 0:
            continue
        w = (hi[ks] - lo[ks])[:, None]
        lam_node = lo[ks][:, None] + w * 0.5 * (x_gl[None, :] + 1.0)      # [k, g]
        lam_edge = lo[ks][:, None] + w * 0.5 * (tau_edge[None, :] + 1.0)  # [k, s+1]
        total = lens[c]
        par = dco.arclength_to_param(ctrl[c], np.concatenate([lam_node.ravel(),
                                                              lam_edge.ravel()]) * total,
                                     total)
        pts = dco.bezier_point(ctrl[c], par)
        nodes = pts[: lam_node.size].reshape(len(ks), gl, 2)
        edges = pts[lam_node.size:].reshape(len(ks), segs + 1, 2)
        for m, k in enumerate(ks):
            node_xy[k * gl:(k + 1) * gl] = nodes[m]
            node_lam[k * gl:(k + 1) * gl] = lam_node[m]
            p1[k * segs:(k + 1) * segs] = edges[m, :-1]
            p2[k * segs:(k + 1) * segs] = edges[m, 1:]
            ell[k * segs:(k + 1) * segs] = total * (hi[k] - lo[k]) / segs
    chord = np.hypot(*(p2 - p1).T)
    jloc = np.floor((x_gl + 1.0) * segs / 2.0).astype(np.int64)
    tstar_loc = (x_gl - (-1.0 + 2.0 * jloc / segs)) / (2.0 / segs)
    n_p = len(lo)
    panel_of_node = np.arange(n_p * gl) // gl
    return dco.Discretization(
        0, gl, segs, n, node_xy, node_lam, panel_of_node * segs + np.tile(jloc, n_p),
        np.tile(tstar_loc, n_p), p1, p2, ell, ell / chord, lens, dco.interp_matrix(gl, segs),
        panel_curve=panel_curve, panel_lo=lo, panel_hi=hi)


def legendre_coefficients(values, g):
    """a_k = (2k+1)/2 sum_i w_i v_i P_k(x_i) for every panel: values [..., N]
    (panels of g consecutive nodes) -> [..., N/g, g]."""
    x, w = dco.gauss_legendre(g)
    eye = np.eye(g)
    pk = np.stack([npleg.legval(x, eye[k]) for k in range(g)])          # [k, i]
    blocks = np.asarray(values, dtype=float).reshape(np.shape(values)[:-1] + (-1, g))
    scale = (2.0 * np.arange(g) + 1.0) / 2.0
    return np.einsum("...pi,ki,i->...pk", blocks, pk, w) * scale


def legendre_tails(disc, sigma):
    """Tail of every panel: max over channels of |a_{g-1}| (Alg. 5)."""
    a = legendre_coefficients(sigma, disc.gl)             # [3, panels, g]
    return np.abs(a[..., -1]).max(axis=0)


def panel_lengths(disc):
    """Arc length of every panel."""
    return disc.seg_ell.reshape(-1, disc.segs).sum(axis=1)


def panels_in_viewport(disc, viewport):
    """Panels with at least one chord meeting the viewport rectangle."""
    cx, cy, w, h = viewport[:4]
    xa, xb, ya, yb = cx - 0.5 * w, cx + 0.5 * w, cy - 0.5 * h, cy + 0.5 * h
    hit = dco.segments_meet_box(disc.seg_p1, disc.seg_p2, xa, xb, ya, yb)
    return hit.reshape(-1, disc.segs).any(axis=1)


def select_panels(disc, tails, eps2, eps1, viewport=None):
    """Alg. 5: panels to cut (tail > eps2, arc length >= eps1, and meeting
    the viewport when one is given)."""
    ok = (np.asarray(tails) > eps2) & (panel_lengths(disc) >= eps1)
    if viewport is not None:
        ok &= panels_in_viewport(disc, viewport)
    return np.nonzero(ok)[0]


def split_panels(panel_curve, panel_lo, panel_hi, chosen):
    """Each chosen panel replaced by its two halves (in arc length).
    Returns the new lists and, per new panel, (parent, half) with half -1
    for an unchanged panel, 0 / 1 for the first / second half."""
    cut = np.zeros(len(panel_lo), bool)
    cut[np.asarray(chosen, dtype=np.int64)] = True
    curve, lo, hi, parent, half = [], [], [], [], []
    for k in range(len(panel_lo)):
        if cut[k]:
            mid = 0.5 * (panel_lo[k] + panel_hi[k])
            for hh, (a, b) in enumerate(((panel_lo[k], mid), (mid, panel_hi[k]))):
                curve.append(panel_curve[k]); lo.append(a); hi.append(b)
                parent.append(k); half.append(hh)
        else:
            curve.append(panel_curve[k]); lo.append(panel_lo[k]); hi.append(panel_hi[k])
            parent.append(k); half.append(-1)
    return (np.array(curve, np.int64), np.array(lo), np.array(hi),
            np.array(parent, np.int64), np.array(half, np.int64))


def warm_start(sigma_old, parent, half, g):
    """Old density at the new nodes (Sec. 7.1.1): a child panel takes the
    Lagrange interpolant of its parent's g nodal values (Eq. legendre_poly)
    at its own nodes, which sit at (x + 1)/2 - 1 (first half) or (x + 1)/2
    (second half) of the parent's [-1, 1]; other panels keep their values."""
    x, _ = dco.gauss_legendre(g)
    old = np.asarray(sigma_old, dtype=float).reshape(3, -1, g)
    out = np.empty((3, len(parent), g))

    def lagrange(at):
        m = np.ones((len(at), g))
        for i in range(g):
            for j in range(g):
                if j != i:
                    m[:, i] *= (at - x[j]) / (x[i] - x[j])
        return m

    child_at = [lagrange(0.5 * (x + 1.0) - 1.0), lagrange(0.5 * (x + 1.0))]
    for k, (par, hh) in enumerate(zip(parent, half)):
        out[:, k] = old[:, par] if hh < 0 else old[:, par] @ child_at[hh].T
    return out.reshape(3, -1)


def label_curves(disc, subdivided, ratio=0.9):
    """Re-solving curves (Sec. 7.1.4): the subdivided curves and every curve
    whose potential range under a unit density on a subdivided curve exceeds
    ratio times that curve's own range.  Returns a bool array [n_curves]
    and the ranges [len(subdivided), n_curves]."""
    node_curve = disc.node_curve
    seg_curve = np.repeat(disc.panel_curve_of(), disc.segs)
    r = np.zeros(disc.n_curves, bool)
    ranges = np.zeros((len(subdivided), disc.n_curves))
    for ia, a in enumerate(subdivided):
        cols = np.nonzero(seg_curve == a)[0]
        G, _ = dco.node_operator_rows(disc, np.arange(disc.N), cols)
        v = G.sum(axis=1)
        for b in range(disc.n_curves):
            vb = v[node_curve == b]
            ranges[ia, b] = vb.max() - vb.min()
        r |= ranges[ia] > ratio * ranges[ia, a]
        r[a] = True
    return r, ranges


def _rhs(disc, up, um):
    GH, FH = dco.hybrid_matrices(disc)
    mu = np.asarray(up) - np.asarray(um)
    b = 0.5 * (np.asarray(up) + np.asarray(um)) - mu @ FH.T       # [3, N]
    return GH, b


def local_resolve(disc, up, um, sigma_c, resolve_curves):
    """Eq. local_resolve_mat by dense LU: sigma_c [3, N] supplies the
    constrained nodes' values (its r entries are ignored); returns the full
    density [3, N]."""
    GH, b = _rhs(disc, up, um)
    rmask = np.asarray(resolve_curves, bool)[disc.node_curve]
    r = np.nonzero(rmask)[0]
    c = np.nonzero(~rmask)[0]
    rhs = b[:, r] - sigma_c[:, c] @ GH[np.ix_(r, c)].T
    out = np.array(sigma_c, dtype=float, copy=True)
    out[:, r] = np.linalg.solve(GH[np.ix_(r, r)], rhs.T).T
    return out


def global_resolve(disc, up, um):
    """The whole system of Eq. db_mat_solve at the new nodes (dense LU)."""
    GH, b = _rhs(disc, up, um)
    return np.linalg.solve(GH, b.T).T
