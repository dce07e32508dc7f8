"""Plain FP64 oracle: hybrid representation formula by direct summation.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Slow on purpose:
every function is the definition written out, so that a reader can check it
against the paper by eye.  Citations name the paper's sections, equations
and appendices (Bang, Serkh, Stein, Jacobson, ACM TOG 42(6), 2023).

What is computed (the discrete quantity the fast method approximates):

* Geometry (App. A, B; Sec. 4.3): each cubic Bezier is cut into P panels of
  equal arc length; every panel carries g Gauss-Legendre nodes (placed at the
  GL roots of normalised panel arc length) and s chord segments of equal arc
  length.  Each chord integral is scaled by kappa = (arc length)/(chord
  length) so that solution and evaluation integrate the true length (App. A).
* Interpolation (Eq. coefs_interp, Eq. legendre_poly, Sec. 5.2): the nodal
  density is mapped to segment midpoints by Pi = Pbar Pring^-1.
* Closed-form segment integrals of G and F (App. D, re-derived because the
  printed antiderivatives are garbled: the reading is
  int ln|p-x| dS = xi2 ln r2 - xi1 ln r1 - |a| + h*theta on the chord, and
  int F dS = -theta/(2 pi)), with the singular self-segment rule of App. C.1
  and App. D.3/D.4 for a collocation node.
* Solve (Eq. db_mat_solve, Alg. 3 without the FMM): dense LU of the hybrid
  collocation system, one right-hand side per colour channel.
* Render (Eq. int_V_dbnd discretised as in Alg. 4, without the FMM): direct
  sum over every chord segment at every pixel centre.

Readings where the paper is silent (normal orientation, where nodes sit on a
panel, tie-breaks) are listed with the design notes of the repository.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.integrate import quad, quad_vec
import scipy.linalg

TWO_PI = 2.0 * np.pi

__all__ = [
    "bezier_point", "bezier_tangent", "curve_length", "arclength_to_param",
    "gauss_legendre", "interp_matrix", "Discretization", "discretize",
    "colour_at", "boundary_values", "chord_integrals", "self_segment_G",
    "node_operator_rows", "assemble", "solve", "solve_stops", "hybrid_matrices",
    "solve_mixed",
    "pixel_centres", "evaluate", "render", "TWO_PI",
    "pixel_box", "segments_meet_box", "aa_edge_mask", "render_aa",
]


# --------------------------------------------------------------------------
# Geometry: cubic Bezier and its arc length (App. B)
# --------------------------------------------------------------------------
def bezier_point(ctrl, t):
    """B(t) = (1-t)^3 C0 + 3t(1-t)^2 C1 + 3t^2(1-t) C2 + t^3 C3 (App. B)."""
    t = np.asarray(t, dtype=float)[..., None]
    s = 1.0 - t
    return (s ** 3) * ctrl[0] + 3.0 * t * s ** 2 * ctrl[1] + \
        3.0 * t ** 2 * s * ctrl[2] + t ** 3 * ctrl[3]


def bezier_tangent(ctrl, t):
    """B'(t), the derivative of the Bernstein form above."""
    t = np.asarray(t, dtype=float)[..., None]
    s = 1.0 - t
    return 3.0 * (s ** 2 * (ctrl[1] - ctrl[0]) + 2.0 * t * s * (ctrl[2] - ctrl[1])
                  + t ** 2 * (ctrl[3] - ctrl[2]))


def _speed(ctrl, t):
    d = bezier_tangent(ctrl, t)
    return np.hypot(d[..., 0], d[..., 1])


def curve_length(ctrl):
    """L(1) = int_0^1 |B'(t)| dt by adaptive quadrature (App. B)."""
    val, _ = quad(lambda t: float(_speed(ctrl, t)), 0.0, 1.0,
                  epsabs=0.0, epsrel=2e-14, limit=500)
    return val


def _lengths_at(ctrl, t):
    """L(t_k) for a vector of parameters: adaptive quadrature of |B'| on the
    gaps between the sorted parameters, then a running sum."""
    t = np.asarray(t, dtype=float)
    order = np.argsort(t)
    ts = t[order]
    lo = np.concatenate([[0.0], ts[:-1]])
    width = ts - lo

    def f(u):
        return width * _speed(ctrl, lo + u * width)

    inc, _ = quad_vec(f, 0.0, 1.0, epsabs=0.0, epsrel=1e-15, norm="max",
                      limit=2000)
    out = np.empty_like(t)
    out[order] = np.cumsum(inc)
    return out


def arclength_to_param(ctrl, targets, total, tol=4e-14, max_iter=80):
    """Invert L(t) = T by Newton's method, t <- t - (L(t)-T)/L'(t) (App. B),
    with L by quadrature; each iterate is kept inside a bisection bracket."""
    T = np.asarray(targets, dtype=float)
    lo = np.zeros_like(T)
    hi = np.ones_like(T)
    t = np.clip(T / total, 0.0, 1.0)
    for _ in range(max_iter):
        f = _lengths_at(ctrl, t) - T
        done = np.abs(f) <= tol * total
        if np.all(done):
            return t
        lo = np.where(f < 0.0, t, lo)
        hi = np.where(f > 0.0, t, hi)
        d = _speed(ctrl, t)
        with np.errstate(divide="ignore", invalid="ignore"):
            tn = t - f / d
        bad = ~((tn > lo) & (tn < hi))
        tn = np.where(bad, 0.5 * (lo + hi), tn)
        t = np.where(done, t, tn)
    raise RuntimeError("arc-length inversion did not converge")


# --------------------------------------------------------------------------
# Gauss-Legendre nodes and the Legendre interpolation matrix (Sec. 4.3, 5.2)
# --------------------------------------------------------------------------
def gauss_legendre(g):
    """Roots x_i of P_g and weights w_i on [-1, 1]."""
    return npleg.leggauss(g)


def interp_matrix(g, s):
    """Pi = Pbar Pring^-1 (Eq. coefs_interp, Eq. legendre_poly, Sec. 5.2).

    Pring[i, k] = P_k(x_i) at the GL roots, Pbar[j, k] = P_k(taubar_j) at the
    arc-length midpoints taubar_j = -1 + (2j+1)/s of the s equal segments.
    """
    x, _ = gauss_legendre(g)
    tbar = -1.0 + (2.0 * np.arange(s) + 1.0) / s
    eye = np.eye(g)
    p_ring = np.stack([npleg.legval(x, eye[k]) for k in range(g)], axis=1)
    p_bar = np.stack([npleg.legval(tbar, eye[k]) for k in range(g)], axis=1)
    return p_bar @ np.linalg.inv(p_ring)


# --------------------------------------------------------------------------
# Discretisation of a set of curves
# --------------------------------------------------------------------------
@dataclass
class Discretization:
    panels: int
    gl: int
    segs: int
    n_curves: int
    node_xy: np.ndarray      # [N, 2] GL node positions q_i
    node_lam: np.ndarray     # [N] normalised arc length of node on its curve
    node_self: np.ndarray    # [N] global index of the self segment
    node_tstar: np.ndarray   # [N] arc-length fraction of the node on it
    seg_p1: np.ndarray       # [S, 2] chord start
    seg_p2: np.ndarray       # [S, 2] chord end
    seg_ell: np.ndarray      # [S] arc length of the segment
    seg_kappa: np.ndarray    # [S] arc length / chord length (App. A)
    curve_len: np.ndarray    # [n] total arc length per curve
    Pi: np.ndarray           # [s, g] interpolation matrix
    # Panels of unequal length (adaptive subdivision, Sec. 7): the curve of
    # each panel and its normalised arc-length range; None for P equal
    # panels per curve (panels above).
    panel_curve: np.ndarray | None = None
    panel_lo: np.ndarray | None = None
    panel_hi: np.ndarray | None = None

    @property
    def N(self):
        return self.node_xy.shape[0]

    def panel_curve_of(self):
        """Curve of every panel [N / g]."""
        if self.panel_curve is not None:
            return np.asarray(self.panel_curve)
        return np.repeat(np.arange(self.n_curves), self.panels)

    @property
    def node_curve(self):
        """Curve of every node [N]."""
        return np.repeat(self.panel_curve_of(), self.gl)

    @property
    def S(self):
        return self.seg_p1.shape[0]

    def interpolate(self, nodal):
        """Segment midpoint values Pi @ (nodal values of each panel).

        nodal: [..., N] -> [..., S]; panels are consecutive blocks of g nodes
        and of s segments."""
        nodal = np.asarray(nodal, dtype=float)
        lead = nodal.shape[:-1]
        blocks = nodal.reshape(lead + (-1, self.gl))          # [..., panels, g]
        seg = np.einsum("jg,...pg->...pj", self.Pi, blocks)    # [..., panels, s]
        return seg.reshape(lead + (-1,))


def _discretize_curve(args):
    ctrl, panels, gl, segs = args
    x_gl, _ = gauss_legendre(gl)
    tau_edge = -1.0 + 2.0 * np.arange(segs + 1) / segs
    total = curve_length(ctrl)
    p = np.arange(panels)[:, None]
    t_node = total * (p + 0.5 * (x_gl[None, :] + 1.0)) / panels     # [P, g]
    t_edge = total * (p + 0.5 * (tau_edge[None, :] + 1.0)) / panels  # [P, s+1]
    targets = np.concatenate([t_node.ravel(), t_edge.ravel()])
    par = arclength_to_param(ctrl, targets, total)
    pts = bezier_point(ctrl, par)
    nodes = pts[: panels * gl]
    edges = pts[panels * gl:].reshape(panels, segs + 1, 2)
    lam = (t_node / total).ravel()
    return total, nodes, edges, lam


def _pool(workers):
    import multiprocessing as mp
    return mp.get_context("fork").Pool(workers)


def discretize(ctrl, panels, gl, segs, workers=1):
    """Nodes, chord segments and scales of every curve (App. A, B; Sec. 5.2)."""
    ctrl = np.asarray(ctrl, dtype=float)
    n = ctrl.shape[0]
    jobs = [(ctrl[c], panels, gl, segs) for c in range(n)]
    if workers > 1 and n > 1:
        with _pool(workers) as pool:
            res = pool.map(_discretize_curve, jobs)
    else:
        res = [_discretize_curve(j) for j in jobs]
    x_gl, _ = gauss_legendre(gl)
    node_xy, node_lam, p1, p2, ell = [], [], [], [], []
    lens = np.empty(n)
    for c, (total, nodes, edges, lam) in enumerate(res):
        lens[c] = total
        node_xy.append(nodes)
        node_lam.append(lam)
        p1.append(edges[:, :-1, :].reshape(-1, 2))
        p2.append(edges[:, 1:, :].reshape(-1, 2))
        ell.append(np.full(panels * segs, total / (panels * segs)))
    node_xy = np.concatenate(node_xy)
    p1 = np.concatenate(p1)
    p2 = np.concatenate(p2)
    ell = np.concatenate(ell)
    chord = np.hypot(*(p2 - p1).T)
    # Self segment of node k of a panel: tau_j <= x_k < tau_{j+1} (App. C.1).
    jloc = np.floor((x_gl + 1.0) * segs / 2.0).astype(np.int64)
    tstar_loc = (x_gl - (-1.0 + 2.0 * jloc / segs)) / (2.0 / segs)
    panel_of_node = np.arange(n * panels * gl) // gl
    node_self = panel_of_node * segs + np.tile(jloc, n * panels)
    node_tstar = np.tile(tstar_loc, n * panels)
    return Discretization(panels, gl, segs, n, node_xy, np.concatenate(node_lam),
                          node_self, node_tstar, p1, p2, ell, ell / chord, lens,
                          interp_matrix(gl, segs))


# --------------------------------------------------------------------------
# Boundary data: colours on each side (Sec. 5.3)
# --------------------------------------------------------------------------
def colour_at(stops, lam):
    """Piecewise-linear colour through stops at lambda = k/(n_stops-1)."""
    stops = np.asarray(stops, dtype=float)
    knots = np.linspace(0.0, 1.0, stops.shape[0])
    return np.stack([np.interp(lam, knots, stops[:, ch]) for ch in range(3)])


def boundary_values(disc, left, right):
    """u_plus (left colour, the side the left normal points to) and u_minus
    (right colour) at every node, each [3, N]."""
    up = np.empty((3, disc.N))
    um = np.empty((3, disc.N))
    node_curve = disc.node_curve
    for c in range(disc.n_curves):
        sl = node_curve == c
        up[:, sl] = colour_at(left[c], disc.node_lam[sl])
        um[:, sl] = colour_at(right[c], disc.node_lam[sl])
    return up, um


# --------------------------------------------------------------------------
# Closed-form chord integrals (App. D, Sec. 4.1 Eq. green_G, Eq. green_F)
# --------------------------------------------------------------------------
def chord_integrals(x, y, p1, p2):
    """Integrals over the straight chord p1 -> p2 of G(p, x) and F(p, x) dS.

    G(p,x) = -ln|p-x| / (2 pi); F(p,x) = -(p-x).n / (2 pi |p-x|^2) with n the
    left normal of the chord.  In chord coordinates xi1 = (p1-x).t,
    xi2 = xi1 + |a|, h = (p1-x).n, r_i^2 = xi_i^2 + h^2 and
    theta = atan2(h |a|, h^2 + xi1 xi2) (the signed angle the chord subtends):
        int ln|p-x| dS = xi2 ln r2 - xi1 ln r1 - |a| + h theta
        int F dS       = -theta / (2 pi)
    A target exactly on the open chord (h = 0, xi1 < 0 < xi2) gets the
    principal value 0 for F; 0 ln 0 := 0 at an endpoint.
    Broadcasts over x, y (targets) against p1, p2 (chords)."""
    ax = p2[..., 0] - p1[..., 0]
    ay = p2[..., 1] - p1[..., 1]
    la = np.hypot(ax, ay)
    tx, ty = ax / la, ay / la
    nx, ny = -ty, tx
    dx = p1[..., 0] - x
    dy = p1[..., 1] - y
    xi1 = dx * tx + dy * ty
    xi2 = xi1 + la
    h = dx * nx + dy * ny
    r1sq = xi1 * xi1 + h * h
    r2sq = xi2 * xi2 + h * h
    theta = np.arctan2(h * la, h * h + xi1 * xi2)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(r1sq > 0.0, xi1 * 0.5 * np.log(r1sq), 0.0)
        t2 = np.where(r2sq > 0.0, xi2 * 0.5 * np.log(r2sq), 0.0)
    int_log = t2 - t1 - la + h * theta
    on_chord = (h == 0.0) & (xi1 < 0.0) & (xi2 > 0.0)
    theta_f = np.where(on_chord, 0.0, theta)
    return -int_log / TWO_PI, -theta_f / TWO_PI


def self_segment_G(ell, tstar):
    """Singular single layer of the segment a collocation node lies on
    (App. D.3): (1/2pi)(l - e1 ln e1 - e2 ln e2), e1 = t* l, e2 = (1-t*) l,
    lengths taken along the arc (App. A).  The double layer is 0 there
    (App. D.4; the +-mu/2 jump is already in the averaged equation, Sec. 5.3)."""
    e1 = tstar * ell
    e2 = (1.0 - tstar) * ell
    with np.errstate(divide="ignore", invalid="ignore"):
        l1 = np.where(e1 > 0, e1 * np.log(e1), 0.0)
        l2 = np.where(e2 > 0, e2 * np.log(e2), 0.0)
    return (ell - l1 - l2) / TWO_PI


# --------------------------------------------------------------------------
# Hybrid collocation system (Eq. hybrid_sys, Eq. db_mat_solve)
# --------------------------------------------------------------------------
def node_operator_rows(disc, rows, seg_cols):
    """kappa-scaled chord integrals Ghat[i, j], Fhat[i, j] between collocation
    nodes `rows` and segments `seg_cols`, with the self-segment override
    (App. C.1, D.3, D.4).  Returns two arrays [len(rows), len(seg_cols)]."""
    rows = np.asarray(rows)
    seg_cols = np.asarray(seg_cols)
    xy = disc.node_xy[rows]
    G, F = chord_integrals(xy[:, 0:1], xy[:, 1:2],
                           disc.seg_p1[seg_cols][None], disc.seg_p2[seg_cols][None])
    kap = disc.seg_kappa[seg_cols][None, :]
    G = G * kap
    F = F * kap
    self_j = disc.node_self[rows]
    hit = self_j[:, None] == seg_cols[None, :]
    ii, jj = np.nonzero(hit)
    if ii.size:
        G[ii, jj] = self_segment_G(disc.seg_ell[seg_cols[jj]],
                                   disc.node_tstar[rows[ii]])
        F[ii, jj] = 0.0
    return G, F


_ASM_STATE = {}


def _panel_block(panel):
    disc, mu_bar = _ASM_STATE["disc"], _ASM_STATE["mu_bar"]
    s = disc.segs
    cols = np.arange(panel * s, (panel + 1) * s)
    G, F = node_operator_rows(disc, np.arange(disc.N), cols)
    a_cols = G @ disc.Pi                                  # [N, g]  Eq. hybrid_sys
    fmu = F @ mu_bar[:, cols].T                           # [N, 3]
    return a_cols, fmu


def assemble(disc, mu_nodes, workers=1, out=None):
    """A = Ghat_H Pbar Pring^-1 (N x N) and F_H mu (N x 3), panel by panel."""
    N, g = disc.N, disc.gl
    n_panels = N // g
    mu_bar = disc.interpolate(mu_nodes)
    A = out if out is not None else np.empty((N, N), order="F")
    fmu = np.zeros((N, 3))
    _ASM_STATE.update(disc=disc, mu_bar=mu_bar)
    try:
        if workers > 1:
            with _pool(workers) as pool:
                for p, (ac, fm) in enumerate(pool.imap(_panel_block, range(n_panels),
                                                       chunksize=4)):
                    A[:, p * g:(p + 1) * g] = ac
                    fmu += fm
        else:
            for p in range(n_panels):
                ac, fm = _panel_block(p)
                A[:, p * g:(p + 1) * g] = ac
                fmu += fm
    finally:
        _ASM_STATE.clear()
    return A, fmu


def solve(disc, u_plus, u_minus, workers=1, report=None):
    """Densities sigma [3, N] of Eq. db_mat_solve by dense LU (Alg. 3 with a
    direct solver in place of GMRES):
        1/2 (u+ + u-) = G_H sigma + F_H mu,   mu = u+ - u-  (Sec. 5.3)."""
    mu = np.asarray(u_plus) - np.asarray(u_minus)
    A, fmu = assemble(disc, mu, workers=workers)
    rhs = 0.5 * (np.asarray(u_plus) + np.asarray(u_minus)).T - fmu   # [N, 3]
    if report is not None:
        report["anorm1"] = float(np.abs(A).sum(axis=0).max())
        A_copy = A.copy(order="F") if disc.N <= 8192 else None
    lu, piv = scipy.linalg.lu_factor(A, overwrite_a=True, check_finite=False)
    sigma = scipy.linalg.lu_solve((lu, piv), rhs, check_finite=False)
    if report is not None:
        report["rcond"] = float(scipy.linalg.lapack.dgecon(lu, report["anorm1"])[0])
        if A_copy is not None:
            r = A_copy @ sigma - rhs
            report["rel_residual"] = (np.linalg.norm(r, axis=0)
                                      / np.linalg.norm(rhs, axis=0)).tolist()
    return sigma.T.copy(), mu


def hybrid_matrices(disc):
    """G_H = Ghat Pbar Pring^-1 and F_H = Fhat Pbar Pring^-1 (N x N each, the
    self-segment rule of App. C.1, D.3, D.4 included), panel by panel."""
    N, g, s = disc.N, disc.gl, disc.segs
    GH = np.empty((N, N))
    FH = np.empty((N, N))
    for p in range(N // g):
        cols = np.arange(p * s, (p + 1) * s)
        G, F = node_operator_rows(disc, np.arange(N), cols)
        GH[:, p * g:(p + 1) * g] = G @ disc.Pi
        FH[:, p * g:(p + 1) * g] = F @ disc.Pi
    return GH, FH


def solve_mixed(disc, neumann, values):
    """Mixed Dirichlet/Neumann conditions on closed curves (Sec. 5.4,
    Eq. neumann_mat), for the domain the curves enclose on their left (the
    left normal points into it, so F u is the double layer of Green's third
    identity).  At every node i, 1/2 u_i = (G_H psi)_i + (F_H u)_i, with
    psi the outward normal derivative.  neumann [N] bool marks the Neumann
    nodes; values [3, N] holds u* at Dirichlet nodes and psi* at Neumann
    nodes.  The unknowns psi_d (Dirichlet nodes) and u_n (Neumann nodes)
    solve
        G_H[:, d] psi_d + F_H[:, n] u_n - 1/2 u_n (rows n)
            = 1/2 u*_d (rows d) - G_H[:, n] psi*_n - F_H[:, d] u*_d
    by dense LU.  Returns psi [3, N] and u [3, N] (known and solved parts);
    the interior field is evaluate(disc, psi, u, points)."""
    neumann = np.asarray(neumann, bool)
    dirichlet = ~neumann
    values = np.asarray(values, float)
    GH, FH = hybrid_matrices(disc)
    A = np.where(dirichlet[None, :], GH, FH)
    idx = np.nonzero(neumann)[0]
    A[idx, idx] -= 0.5
    known_psi = np.where(neumann[None, :], values, 0.0)
    known_u = np.where(dirichlet[None, :], values, 0.0)
    rhs = 0.5 * known_u - known_psi @ GH.T - known_u @ FH.T      # [3, N]
    lu, piv = scipy.linalg.lu_factor(A)
    x = scipy.linalg.lu_solve((lu, piv), rhs.T).T
    psi = np.where(dirichlet[None, :], x, values)
    u = np.where(neumann[None, :], x, values)
    return psi, u


def solve_stops(disc, left, right, workers=1, report=None):
    """Solve with colours given as stops along each curve (Sec. 5.3)."""
    up, um = boundary_values(disc, left, right)
    return solve(disc, up, um, workers=workers, report=report)


# --------------------------------------------------------------------------
# Evaluation at targets and pixels (Eq. int_V_dbnd, Alg. 4 without the FMM)
# --------------------------------------------------------------------------
def pixel_centres(viewport):
    """Pixel (row r, col k) centre: x = cx - w/2 + (k+1/2) w/W,
    y = cy + h/2 - (r+1/2) h/H (row 0 at the top, y up)."""
    cx, cy, w, h, W, H = viewport
    xs = cx - 0.5 * w + (np.arange(W) + 0.5) * (w / W)
    ys = cy + 0.5 * h - (np.arange(H) + 0.5) * (h / H)
    return xs, ys


_EVAL_STATE = {}


def _eval_block(args):
    lo, hi = args
    st = _EVAL_STATE
    return _evaluate_serial(st["pts"][lo:hi], st["p1"], st["p2"], st["ws"], st["wm"],
                            pt_chunk=st["pt_chunk"])


def _evaluate_serial(pts, p1, p2, wsig, wmu, seg_chunk=8192, pt_chunk=64):
    out = np.zeros((pts.shape[0], 3))
    for a in range(0, pts.shape[0], pt_chunk):
        x = pts[a:a + pt_chunk, 0:1]
        y = pts[a:a + pt_chunk, 1:2]
        acc = np.zeros((x.shape[0], 3))
        for b in range(0, p1.shape[0], seg_chunk):
            G, F = chord_integrals(x, y, p1[None, b:b + seg_chunk],
                                   p2[None, b:b + seg_chunk])
            acc += G @ wsig[b:b + seg_chunk] + F @ wmu[b:b + seg_chunk]
        out[a:a + pt_chunk] = acc
    return out


def evaluate(disc, sigma, mu, pts, workers=1, pt_chunk=64):
    """u_c(x) = sum_j kappa_j [int_j G sigma_bar_cj + int_j F mu_bar_cj] at the
    points pts [n, 2]; returns [n, 3].  pt_chunk points share one sweep over
    the segments (the sums run over the segments in the same order for any
    pt_chunk; larger chunks read the segments fewer times)."""
    pts = np.asarray(pts, dtype=float)
    wsig = (disc.interpolate(sigma) * disc.seg_kappa).T.copy()   # [S, 3]
    wmu = (disc.interpolate(mu) * disc.seg_kappa).T.copy()
    if workers > 1 and pts.shape[0] > 256:
        _EVAL_STATE.update(pts=pts, p1=disc.seg_p1, p2=disc.seg_p2, ws=wsig, wm=wmu,
                           pt_chunk=pt_chunk)
        bounds = np.linspace(0, pts.shape[0], 4 * workers + 1).astype(int)
        jobs = [(bounds[i], bounds[i + 1]) for i in range(len(bounds) - 1)]
        with _pool(workers) as pool:
            parts = pool.map(_eval_block, jobs)
        _EVAL_STATE.clear()
        return np.concatenate(parts)
    return _evaluate_serial(pts, disc.seg_p1, disc.seg_p2, wsig, wmu, pt_chunk=pt_chunk)


def render(disc, sigma, mu, viewport, rows=None, cols=None, workers=1):
    """Image [H, W, 3] (or the sub-grid rows x cols) of the viewport."""
    xs, ys = pixel_centres(viewport)
    rows = np.arange(len(ys)) if rows is None else np.asarray(rows)
    cols = np.arange(len(xs)) if cols is None else np.asarray(cols)
    X, Y = np.meshgrid(xs[cols], ys[rows])
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    return evaluate(disc, sigma, mu, pts, workers=workers).reshape(
        len(rows), len(cols), 3)


# --------------------------------------------------------------------------
# Anti-aliasing (Sec. 8): area-weighted pixel values where curves cross
# --------------------------------------------------------------------------
def pixel_box(viewport, r, k):
    """Closed square of pixel (row r, column k): [xa, xb] x [ya, yb] with
    xa = x0 + k pw, xb = x0 + (k+1) pw, ya = y1 - (r+1) ph, yb = y1 - r ph,
    x0 = cx - w/2, y1 = cy + h/2, pw = w/W, ph = h/H."""
    cx, cy, w, h, W, H = viewport
    x0, y1 = cx - 0.5 * w, cy + 0.5 * h
    pw, ph = w / W, h / H
    return x0 + k * pw, x0 + (k + 1) * pw, y1 - (r + 1) * ph, y1 - r * ph


def segments_meet_box(p1, p2, xa, xb, ya, yb):
    """For every chord p1 -> p2 (closed segment): does it meet the closed box
    [xa, xb] x [ya, yb]?  Clips the parameter t in [0, 1] by the four half
    planes (Liang-Barsky); the box is met when the interval stays nonempty."""
    dx = p2[:, 0] - p1[:, 0]
    dy = p2[:, 1] - p1[:, 1]
    t0 = np.zeros(len(p1))
    t1 = np.ones(len(p1))
    ok = np.ones(len(p1), bool)
    for p, q in ((-dx, p1[:, 0] - xa), (dx, xb - p1[:, 0]),
                 (-dy, p1[:, 1] - ya), (dy, yb - p1[:, 1])):
        zero = p == 0.0
        ok &= ~(zero & (q < 0.0))
        with np.errstate(divide="ignore", invalid="ignore"):
            r = q / np.where(zero, 1.0, p)
        t0 = np.where(~zero & (p < 0.0), np.maximum(t0, r), t0)
        t1 = np.where(~zero & (p > 0.0), np.minimum(t1, r), t1)
        ok &= t0 <= t1
    return ok


def aa_edge_mask(disc, viewport):
    """[H, W] bool: pixels whose closed square meets a chord segment."""
    W, H = viewport[4], viewport[5]
    mask = np.zeros((H, W), bool)
    for r in range(H):
        for k in range(W):
            mask[r, k] = segments_meet_box(disc.seg_p1, disc.seg_p2,
                                           *pixel_box(viewport, r, k)).any()
    return mask


def render_aa(disc, sigma, mu, viewport, aa, rows, cols, workers=1):
    """Anti-aliased pixel values (Sec. 8) at pixels (rows[i], cols[i]): a pixel
    whose square meets a chord takes the mean of u at the centres of its
    aa x aa equal sub-squares (area weighting over one level of sub-cells),
    (x0 + (k + (i+1/2)/aa) pw, y1 - (r + (j+1/2)/aa) ph); any other pixel
    its centre value.  Returns [n, 3] and the edge flags [n]."""
    cx, cy, w, h, W, H = viewport
    x0, y1 = cx - 0.5 * w, cy + 0.5 * h
    pw, ph = w / W, h / H
    xs, ys = pixel_centres(viewport)
    rows, cols = np.asarray(rows), np.asarray(cols)
    edge = np.array([segments_meet_box(disc.seg_p1, disc.seg_p2,
                                       *pixel_box(viewport, r, k)).any()
                     for r, k in zip(rows, cols)], bool)
    frac = (np.arange(aa) + 0.5) / aa
    pts = []
    for r, k, e in zip(rows, cols, edge):
        if e:
            sx = x0 + (k + frac[None, :]) * pw + 0.0 * frac[:, None]
            sy = y1 - (r + frac[:, None]) * ph + 0.0 * frac[None, :]
            pts.append(np.stack([sx.ravel(), sy.ravel()], axis=1))
        else:
            pts.append(np.array([[xs[k], ys[r]]]))
    vals = evaluate(disc, sigma, mu, np.concatenate(pts), workers=workers)
    out = np.empty((len(rows), 3))
    at = 0
    for i, p in enumerate(pts):
        out[i] = vals[at:at + len(p)].mean(axis=0)
        at += len(p)
    return out, edge


def default_workers():
    return max(1, min(16, os.cpu_count() or 1))
