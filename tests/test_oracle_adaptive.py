"""Pins of the oracle's adaptive subdivision (Sec. 7, Alg. 5-7) against
closed forms and exact properties, on the CPU."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
from oracle import adaptive as ad


def line_ctrl(p0, p3):
    """A straight cubic with evenly spaced control points: B(t) = p0 + t (p3 - p0),
    so arc length is linear in t."""
    p0, p3 = np.asarray(p0, float), np.asarray(p3, float)
    return np.stack([p0 + k / 3.0 * (p3 - p0) for k in range(4)])


@pytest.mark.parametrize("g", [4, 8, 16])
def test_legendre_coefficients_of_polynomials(g):
    """a_k of a polynomial of degree < g sampled at the GL roots are its
    Legendre coefficients: P_j itself gives e_j, x^2 = (P_0 + 2 P_2)/3."""
    x, _ = npleg.leggauss(g)
    for j in range(g):
        vals = npleg.legval(x, np.eye(g)[j])
        a = ad.legendre_coefficients(vals[None], g)[0, 0]
        assert np.abs(a - np.eye(g)[j]).max() < 1e-13
    a = ad.legendre_coefficients((x ** 2)[None], g)[0, 0]
    want = np.zeros(g)
    want[0] = 1.0 / 3.0
    if g > 2:
        want[2] = 2.0 / 3.0
    assert np.abs(a[:3] - want[:3]).max() < 1e-14
    assert np.abs(a[3:]).max() < 1e-14


def test_legendre_tail_takes_largest_channel():
    g = 8
    x, _ = npleg.leggauss(g)
    top = npleg.legval(x, np.eye(g)[g - 1])
    sigma = np.zeros((3, 2 * g))
    sigma[1, :g] = 5.0 * top            # panel 0: tail 5 in channel 1
    sigma[0, :g] = -2.0 * top
    sigma[2, g:] = 1.0 + x - 3.0 * top  # panel 1: tail 3 in channel 2
    disc = type("D", (), {"gl": g})()
    t = ad.legendre_tails(disc, sigma)
    assert np.allclose(t, [5.0, 3.0], rtol=0, atol=1e-12)


def test_discretize_panels_on_a_straight_curve():
    """On a straight, evenly parametrised cubic, a panel [lo, hi] puts node
    k at p0 + (lo + (hi - lo)(x_k + 1)/2)(p3 - p0) and its segments have
    arc length L (hi - lo)/s and kappa = 1."""
    p0, p3 = np.array([0.1, 0.2]), np.array([0.9, 0.6])
    ctrl = line_ctrl(p0, p3)[None]
    L = np.hypot(*(p3 - p0))
    pc = np.array([0, 0, 0])
    lo = np.array([0.0, 0.25, 0.375])
    hi = np.array([0.25, 0.375, 1.0])
    g, s = 6, 12
    d = ad.discretize_panels(ctrl, pc, lo, hi, g, s)
    x, _ = npleg.leggauss(g)
    for k in range(3):
        lam = lo[k] + (hi[k] - lo[k]) * 0.5 * (x + 1.0)
        want = p0[None] + lam[:, None] * (p3 - p0)[None]
        assert np.abs(d.node_xy[k * g:(k + 1) * g] - want).max() < 1e-13
        assert np.allclose(d.seg_ell[k * s:(k + 1) * s], L * (hi[k] - lo[k]) / s, rtol=1e-13)
    assert np.allclose(d.seg_kappa, 1.0, rtol=1e-12)
    assert np.array_equal(d.node_curve, np.zeros(3 * g))
    # segments tile the curve end to end
    assert np.abs(d.seg_p2[:-1] - d.seg_p1[1:]).max() < 1e-13
    assert np.allclose(ad.panel_lengths(d), L * (hi - lo), rtol=1e-13)


def test_uniform_panel_list_is_the_base_discretisation():
    """P equal panels as a list give the same nodes and chords as discretize."""
    import scenegen
    sc = scenegen.uniform_scene(n_curves=2, n_stops=2, seed=0, panels=3, gl=6, segs=12)
    pc, lo, hi = ad.uniform_panels(2, 3)
    a = ad.discretize_panels(sc["ctrl"], pc, lo, hi, 6, 12)
    b = oracle.discretize(sc["ctrl"], 3, 6, 12)
    assert np.abs(a.node_xy - b.node_xy).max() < 1e-13
    assert np.abs(a.seg_p1 - b.seg_p1).max() < 1e-13
    assert np.array_equal(a.node_self, b.node_self)
    up_a, _ = oracle.boundary_values(a, sc["left"], sc["right"])
    up_b, _ = oracle.boundary_values(b, sc["left"], sc["right"])
    assert np.abs(up_a - up_b).max() < 1e-13


def test_split_panels_and_warm_start_are_exact_for_polynomials():
    """Children halve their parent in arc length; the warm start reproduces
    a polynomial of degree < g at the children's nodes exactly."""
    g = 8
    pc = np.array([0, 0, 1])
    lo = np.array([0.0, 0.5, 0.0])
    hi = np.array([0.5, 1.0, 1.0])
    npc, nlo, nhi, par, half = ad.split_panels(pc, lo, hi, [1, 2])
    assert np.array_equal(npc, [0, 0, 0, 1, 1])
    assert np.allclose(nlo, [0.0, 0.5, 0.75, 0.0, 0.5])
    assert np.allclose(nhi, [0.5, 0.75, 1.0, 0.5, 1.0])
    assert np.array_equal(par, [0, 1, 1, 2, 2]) and np.array_equal(half, [-1, 0, 1, 0, 1])
    x, _ = npleg.leggauss(g)

    def f(t, ch):                     # degree 7 < g on the parent's [-1, 1]
        return (ch + 1.0) * t ** 7 - 2.0 * t ** 3 + 0.5 * t + ch

    old = np.stack([np.concatenate([f(x, ch) for _ in range(3)]) for ch in range(3)])
    new = ad.warm_start(old, par, half, g).reshape(3, 5, g)
    for ch in range(3):
        assert np.abs(new[ch, 0] - f(x, ch)).max() < 1e-13            # unchanged panel
        assert np.abs(new[ch, 1] - f(0.5 * (x + 1) - 1, ch)).max() < 1e-12
        assert np.abs(new[ch, 2] - f(0.5 * (x + 1), ch)).max() < 1e-12


def test_select_panels_obeys_length_and_viewport():
    ctrl = np.stack([line_ctrl([0, 0], [1, 0]), line_ctrl([5, 0], [6, 0])])
    pc, lo, hi = ad.uniform_panels(2, 4)
    d = ad.discretize_panels(ctrl, pc, lo, hi, 4, 8)
    tails = np.array([10, 0.5, 10, 10, 10, 10, 0.5, 10], float)
    assert list(ad.select_panels(d, tails, 1.0, 0.0)) == [0, 2, 3, 4, 5, 7]
    # panels are 0.25 long: eps1 above that blocks every cut
    assert len(ad.select_panels(d, tails, 1.0, 0.3)) == 0
    # a viewport around the first curve only
    assert list(ad.select_panels(d, tails, 1.0, 0.0, viewport=(0.5, 0.0, 1.2, 0.4))) == [0, 2, 3]
    # the viewport's right edge at x = 0.6 reaches panel 2 ([0.5, 0.75]) but not 3
    assert list(ad.select_panels(d, tails, 1.0, 0.0, viewport=(0.3, 0.0, 0.6, 0.4))) == [0, 2]


def _two_clusters():
    import scenegen
    sc = scenegen.uniform_scene(n_curves=6, n_stops=2, seed=0, panels=2, gl=8, segs=16)
    ctrl = np.array(sc["ctrl"], float)
    ctrl[3:, :, 0] += 40.0
    return ctrl, sc["left"], sc["right"]


def test_label_curves_keeps_far_curves_constrained():
    """Sec. 7.1.4: a unit density on a cut curve changes the potential over
    a curve 40 units away far less than over the cut curve itself, so the
    far cluster is not re-solved; the cut curve always is."""
    ctrl, left, right = _two_clusters()
    pc, lo, hi = ad.uniform_panels(6, 2)
    d = ad.discretize_panels(ctrl, pc, lo, hi, 8, 16)
    r, ranges = ad.label_curves(d, [1])
    assert r[1] and not r[3:].any()
    assert (ranges[0, 3:] < 0.05 * ranges[0, 1]).all()
    # the rule itself: re-solved exactly where the range exceeds 0.9 of the own
    assert np.array_equal(r, (ranges[0] > 0.9 * ranges[0, 1]) | (np.arange(6) == 1))


def test_local_resolve_identities():
    """Eq. local_resolve_mat: re-solving every curve is the global solve;
    holding sigma_c at its global values returns the global solution; the
    constrained values are kept and the re-solved rows hold exactly."""
    ctrl, left, right = _two_clusters()
    pc, lo, hi = ad.uniform_panels(6, 2)
    d = ad.discretize_panels(ctrl, pc, lo, hi, 8, 16)
    up, um = oracle.boundary_values(d, left, right)
    glob = ad.global_resolve(d, up, um)
    every = ad.local_resolve(d, up, um, np.zeros_like(glob), np.ones(6, bool))
    assert np.abs(every - glob).max() <= 1e-9 * np.abs(glob).max()
    r = np.array([True, True, True, False, False, False])
    same = ad.local_resolve(d, up, um, glob, r)
    assert np.abs(same - glob).max() <= 1e-9 * np.abs(glob).max()
    held = glob * 1.01
    loc = ad.local_resolve(d, up, um, held, r)
    cn = ~r[d.node_curve]
    assert np.array_equal(loc[:, cn], held[:, cn])
    GH, FH = oracle.hybrid_matrices(d)
    b = 0.5 * (up + um) - (up - um) @ FH.T
    res = (loc @ GH.T - b)[:, ~cn]
    assert np.abs(res).max() <= 1e-10 * np.abs(b).max()
