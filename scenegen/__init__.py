"""Seeded synthetic inputs for the diffusion-curve solver and its oracle.

This module only draws random numbers and lays them out as arrays: control
points of cubic Bezier curves, colour stops and viewports.  It holds none of
the method's arithmetic (no arc length, no quadrature, no kernels), so the
oracle and the GPU library can both be fed from it without sharing code.

Array conventions (shared by every consumer):
  ctrl  float64 [n, 4, 2]   control points C0..C3 of each curve, y up
  left  float64 [n, k, 3]   RGB colour stops on the left side of each curve
  right float64 [n, k, 3]   RGB colour stops on the right side
  stops are placed at normalised arc length k/(n_stops-1) along the curve.
A viewport is (cx, cy, width, height, W, H) in world units / pixels.

The paper's own example scenes are artwork that is not available here; the
generators below stand in for them with the sizes of its workloads
(151-4,632 curves, Tab. 2) and with the configurations measured by the
benchmark.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Scene", "uniform_scene", "sized_scene", "clustered_scene",
    "zoom_viewports", "serving_scenes", "polygon_ctrl", "circle_ctrl",
    "bernstein_point", "batch_scene", "serving_requests", "poisson_arrivals",
    "synthetic_densities", "serving_extent", "serving_domain",
    "TINY", "FMM", "PRECISION", "BATCH", "SERVING",
]


class Scene(dict):
    """A plain dict with keys ctrl, left, right and the discretisation."""

    @property
    def n_curves(self) -> int:
        return int(self["ctrl"].shape[0])


def _draw_curves(rng, n, n_stops, shape_fn):
    ctrl = np.empty((n, 4, 2))
    left = np.empty((n, n_stops, 3))
    right = np.empty((n, n_stops, 3))
    for c in range(n):  # draw order per curve: shape, left stops, right stops
        ctrl[c] = shape_fn(rng, c)
        left[c] = rng.uniform(0.0, 1.0, size=(n_stops, 3))
        right[c] = rng.uniform(0.0, 1.0, size=(n_stops, 3))
    return ctrl, left, right


def uniform_scene(n_curves=8, n_stops=2, seed=0, panels=4, gl=16, segs=80,
                  leaf_max=64):
    """Curves with control points uniform in [0,1]^2 (the tiny configuration)."""
    rng = np.random.default_rng(seed)
    ctrl, left, right = _draw_curves(
        rng, n_curves, n_stops, lambda r, c: r.uniform(0.0, 1.0, size=(4, 2)))
    return Scene(ctrl=ctrl, left=left, right=right, panels=panels, gl=gl,
                 segs=segs, leaf_max=leaf_max)


def _sized_shape(lmin, lmax, centre_fn):
    def shape(rng, c):
        ell = np.exp(rng.uniform(np.log(lmin), np.log(lmax)))
        raw = rng.uniform(0.0, 1.0, size=(4, 2))
        # Size is set on the control-polygon length, an upper bound of the
        # arc length; the curve is scaled about C0.
        poly = np.sum(np.hypot(*(raw[1:] - raw[:-1]).T))
        pts = raw[0] + (raw - raw[0]) * (ell / poly)
        centre = 0.5 * (pts.min(axis=0) + pts.max(axis=0))
        return pts - centre + centre_fn(rng, c)
    return shape


def sized_scene(n_curves=200, n_stops=3, seed=1, lmin=0.01, lmax=0.5,
                panels=16, gl=16, segs=80, leaf_max=64):
    """Curves of log-uniform size with bbox centres uniform in [0,1]^2."""
    rng = np.random.default_rng(seed)
    shape = _sized_shape(lmin, lmax, lambda r, c: r.uniform(0.0, 1.0, size=2))
    ctrl, left, right = _draw_curves(rng, n_curves, n_stops, shape)
    return Scene(ctrl=ctrl, left=left, right=right, panels=panels, gl=gl,
                 segs=segs, leaf_max=leaf_max)


def clustered_scene(n_blob_curves=2000, n_blobs=5, n_long=20, n_stops=3,
                    seed=2, sigma=0.05, lmin=0.005, lmax=0.1, panels=32,
                    gl=16, segs=80, leaf_max=64):
    """Curves clustered in Gaussian blobs plus long curves spanning [0,1]."""
    rng = np.random.default_rng(seed)
    blobs = rng.uniform(0.2, 0.8, size=(n_blobs, 2))
    shape = _sized_shape(
        lmin, lmax,
        lambda r, c: blobs[c % n_blobs] + r.normal(0.0, sigma, size=2))
    c1, l1, r1 = _draw_curves(rng, n_blob_curves, n_stops, shape)

    def long_shape(r, c):
        pts = r.uniform(0.0, 1.0, size=(4, 2))
        pts[0, 0] = 0.0
        pts[3, 0] = 1.0
        return pts
    c2, l2, r2 = _draw_curves(rng, n_long, n_stops, long_shape)
    return Scene(ctrl=np.concatenate([c1, c2]), left=np.concatenate([l1, l2]),
                 right=np.concatenate([r1, r2]), panels=panels, gl=gl,
                 segs=segs, leaf_max=leaf_max)


def bernstein_point(ctrl4, t):
    """Point of one cubic Bezier at parameter t (curve definition only)."""
    s = 1.0 - t
    return (s ** 3) * ctrl4[0] + 3 * t * s * s * ctrl4[1] + \
        3 * t * t * s * ctrl4[2] + (t ** 3) * ctrl4[3]


def zoom_viewports(ctrl, n=64, sides=(128, 256, 512, 1024, 2048),
                   zoom=(1.0, 1e6), seed=3):
    """Viewports of random side, log-uniform zoom, centred on curve points."""
    rng = np.random.default_rng(seed + 1000)
    vps = []
    for _ in range(n):
        side = int(rng.choice(sides))
        z = 10.0 ** rng.uniform(np.log10(zoom[0]), np.log10(zoom[1]))
        c = int(rng.integers(ctrl.shape[0]))
        t = rng.uniform(0.0, 1.0)
        cx, cy = bernstein_point(ctrl[c], t)
        vps.append((float(cx), float(cy), 1.0 / z, 1.0 / z, side, side))
    return vps


def batch_scene(cfg=None):
    """The 500-curve scene of the batched-render workload and its 64 zoomed
    viewports.

    Curves are drawn by sized_scene (lengths log-uniform in [0.01, 0.5]),
    not with control points uniform in [0,1]^2: at 500 curves the latter
    cross so densely that the collocation system has a reciprocal condition
    number near 1e-12, densities near 1e6 and pixel values far outside the
    colour range, which is no diffusion-curve image.
    """
    cfg = BATCH if cfg is None else cfg
    sc = sized_scene(n_curves=cfg["n_curves"], n_stops=cfg["n_stops"], seed=cfg["seed"],
                     panels=cfg["panels"], gl=cfg["gl"], segs=cfg["segs"])
    vps = zoom_viewports(sc["ctrl"], n=cfg["n_viewports"], seed=cfg["seed"])
    return sc, vps


def serving_extent(n_curves, per_unit_area=200):
    """Side of the square [0, a]^2 holding the bbox centres of a serving
    scene's curves: the unit square up to per_unit_area curves, growing so
    that larger scenes keep that many curves per unit area."""
    return max(1.0, float(np.sqrt(n_curves / per_unit_area)))


def serving_scenes(n_scenes=16, seed0=100, nmin=10, nmax=5000, per_unit_area=200,
                   lmin=0.01, lmax=0.5, **kw):
    """Resident scenes of log-uniform curve counts for the serving loop.

    Curves are drawn as in sized_scene (lengths log-uniform in [lmin, lmax]),
    with bbox centres uniform in [0, a]^2, a = serving_extent(n): a scene of
    n curves covers n / per_unit_area unit squares, like a larger canvas,
    instead of packing thousands of curves of length up to 0.5 into the unit
    square (where they would cross each other some 10^5 times)."""
    out = []
    for k in range(n_scenes):
        rng = np.random.default_rng(seed0 + k)
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        a = serving_extent(n, per_unit_area)
        rng = np.random.default_rng(seed0 + k)
        shape = _sized_shape(lmin, lmax, lambda r, c, a=a: r.uniform(0.0, a, size=2))
        ctrl, left, right = _draw_curves(rng, n, 3, shape)
        out.append(Scene(ctrl=ctrl, left=left, right=right, extent=a, **kw))
    return out


def serving_domain(sc):
    """Quadtree root of a serving scene: its square extent with a margin of
    one unit, so zoom-1 viewports centred on any curve point fit."""
    a = sc.get("extent", 1.0)
    return (-1.0, -1.0, a + 1.0, a + 1.0)


def serving_requests(scenes, n, seed=7, sides=(256, 512, 1024, 2048), zoom=(1.0, 1e6)):
    """Request stream of the serving workload: (scene index, viewport) with
    the scene uniform, the side uniform over `sides`, zoom log-uniform and
    the centre at a uniform parameter of a random curve of that scene."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        k = int(rng.integers(len(scenes)))
        ctrl = scenes[k]["ctrl"]
        side = int(rng.choice(sides))
        z = 10.0 ** rng.uniform(np.log10(zoom[0]), np.log10(zoom[1]))
        c = int(rng.integers(ctrl.shape[0]))
        cx, cy = bernstein_point(ctrl[c], rng.uniform(0.0, 1.0))
        out.append((k, (float(cx), float(cy), 1.0 / z, 1.0 / z, side, side)))
    return out


def synthetic_densities(n_nodes, phase=0.0):
    """Smooth synthetic nodal densities [3][n_nodes] given by the node index
    alone (nodes are numbered curve, panel, GL node): 0.5 cos(0.37 i + 1.3 c
    + phase) for channel c.  Inputs for render and operator parity where a
    dense solve is out of reach."""
    i = np.arange(n_nodes, dtype=float)
    return np.stack([0.5 * np.cos(0.37 * i + 1.3 * c + phase) for c in range(3)])


def poisson_arrivals(n, rate, seed=11):
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def polygon_ctrl(vertices):
    """Closed polygon as straight Beziers with evenly spaced control points.

    Evenly spaced control points make the parametrisation linear, so every
    chord is exact and the arc-length scale of each segment is one.
    """
    v = np.asarray(vertices, float)
    out = []
    for a, b in zip(v, np.roll(v, -1, axis=0)):
        out.append([a, a + (b - a) / 3.0, a + 2.0 * (b - a) / 3.0, b])
    return np.array(out)


def circle_ctrl(cx=0.5, cy=0.5, radius=0.3, n_arcs=4, ccw=True):
    """Closed near-circle made of n_arcs cubic Beziers (standard handles)."""
    k = 4.0 / 3.0 * np.tan(np.pi / (2 * n_arcs))
    out = []
    for i in range(n_arcs):
        a0 = 2 * np.pi * i / n_arcs
        a1 = 2 * np.pi * (i + 1) / n_arcs
        if not ccw:
            a0, a1 = -a0, -a1
        p0 = np.array([np.cos(a0), np.sin(a0)])
        p3 = np.array([np.cos(a1), np.sin(a1)])
        sgn = 1.0 if ccw else -1.0
        t0 = sgn * np.array([-np.sin(a0), np.cos(a0)])
        t3 = sgn * np.array([-np.sin(a1), np.cos(a1)])
        pts = np.array([p0, p0 + k * t0, p3 - k * t3, p3])
        out.append(np.array([cx, cy]) + radius * pts)
    return np.array(out)


# Named workloads (sizes of the configurations the benchmark and tests use).
TINY = dict(n_curves=8, n_stops=2, seed=0, panels=4, gl=16, segs=80,
            viewport=(0.5, 0.5, 1.0, 1.0, 256, 256))
FMM = dict(n_curves=200, n_stops=3, seed=1, panels=16, gl=16, segs=80,
           leaf_max=64, p=20, gmres_tol=1e-10,
           viewport=(0.5, 0.5, 1.0, 1.0, 2048, 2048))
PRECISION = dict(seed=2, panels=32, gl=16, segs=80,
                 viewport=(0.5, 0.5, 1.0, 1.0, 4096, 4096))
# The batch scene uses the sized generator: 500 curves with control points
# uniform in the unit square cross each other thousands of times and make
# the hybrid system numerically singular (see batch_scene).  The domain
# covers zoom-1 viewports centred anywhere on a curve.
BATCH = dict(n_curves=500, n_stops=2, seed=3, panels=4, gl=16, segs=80,
             n_viewports=64, domain=(-1.0, -1.0, 2.0, 2.0))
SERVING = dict(n_scenes=16, seed0=100, panels=16, gl=16, segs=80,
               n_requests=2000, n_warmup=100)
