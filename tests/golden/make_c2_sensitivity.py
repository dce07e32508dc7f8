"""Write tests/golden/c2_sensitivity.npz: how much the oracle's own pixel
values of the 200-curve workload move when every chord end point is
rounded differently by one unit in the last place (ulp).

Two independent FP64 implementations of the discretisation (App. A, B)
evaluate the Bezier curves and their arc-length inverses with different
operation orders, so their chord end points differ by about one ulp.  On
this scene one curve has a near-cusp whose densities reach 1e7 with charges
of both signs (sum |q| about 1e4 against a net charge near 1), and the
chord scale kappa = arc/chord of its 2e-4-long chords turns a one-ulp end
point change into a relative change of about 5e-13 of such charges.  The
result bounds how closely any independent implementation can agree with the
oracle on this workload, whatever its own accuracy.

Stored, per sampled pixel of c2_samples.npz (both measured by the oracle
alone, with end points moved by +-1 ulp independently, shared end points of
consecutive chords moved together, kappa recomputed from the moved ends):
  render   [n_draws, n_px, 3]  change of the pixel values with the stored
                               oracle densities (c2_sigma.npz) held fixed
  solve    [n_px, 3]           change when the dense LU solve is repeated on
                               the moved geometry as well (one draw; the
                               densities follow the ill-conditioned system)
Calls only the oracle and the seeded scene generator.  Needs ~25 GB of RAM
and about fifteen minutes on 8 cores:
    python tests/golden/make_c2_sensitivity.py
"""
import dataclasses
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "c2_sensitivity.npz")
ULP = 2.0 ** -52


def moved_ends(disc, rng):
    """The discretisation with every chord end point scaled by (1 +- ulp);
    the end of chord j and the start of chord j+1 of a panel are one point."""
    s = disc.segs
    ends = np.concatenate([disc.seg_p1.reshape(-1, s, 2),
                           disc.seg_p2.reshape(-1, s, 2)[:, -1:, :]], axis=1)
    ends = ends * (1.0 + rng.choice([-1.0, 1.0], size=ends.shape) * ULP)
    p1 = ends[:, :-1].reshape(-1, 2).copy()
    p2 = ends[:, 1:].reshape(-1, 2).copy()
    kappa = disc.seg_ell / np.hypot(*(p2 - p1).T)
    return dataclasses.replace(disc, seg_p1=p1, seg_p2=p2, seg_kappa=kappa)


def main():
    cfg = scenegen.FMM
    workers = int(os.environ.get("WORKERS", "8"))
    n_draws = int(os.environ.get("DRAWS", "2"))
    sc = scenegen.sized_scene(n_curves=cfg["n_curves"], n_stops=cfg["n_stops"],
                              seed=cfg["seed"])
    disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"],
                             workers=workers)
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    sigma = np.load(os.path.join(HERE, "c2_sigma.npz"))["sigma"]
    smp = np.load(os.path.join(HERE, "c2_samples.npz"))
    xs, ys = oracle.pixel_centres(cfg["viewport"])
    pts = np.stack([xs[smp["cols"]], ys[smp["rows"]]], axis=1)
    base = oracle.evaluate(disc, sigma, up - um, pts, workers=workers)
    assert np.array_equal(base, smp["vals"]), "stored samples are not this oracle's"
    rng = np.random.default_rng(2311)
    render = []
    for k in range(n_draws):
        moved = moved_ends(disc, rng)
        d = oracle.evaluate(moved, sigma, up - um, pts, workers=workers) - base
        render.append(np.abs(d))
        print(f"render draw {k}: max {np.abs(d).max():.3e}", flush=True)
    moved = moved_ends(disc, rng)
    t0 = time.time()
    sig2, mu2 = oracle.solve(moved, up, um, workers=workers)
    print(f"solve on moved geometry: {time.time() - t0:.1f} s; densities rel change "
          f"{np.abs(sig2 - sigma).max() / np.abs(sigma).max():.3e}", flush=True)
    solve = np.abs(oracle.evaluate(moved, sig2, mu2, pts, workers=workers) - base)
    print(f"end-to-end change: max {solve.max():.3e}", flush=True)
    np.savez_compressed(OUT, render=np.array(render), solve=solve, rows=smp["rows"],
                        cols=smp["cols"], ulp=ULP)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
