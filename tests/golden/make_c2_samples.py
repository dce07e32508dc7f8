"""Write tests/golden/c2_samples.npz: FP64 oracle pixel values of the
200-curve workload's 2048 x 2048 render of [0,1]^2 at sampled pixels (a
stride-64 grid plus pixels that hold chord midpoints), using the oracle
densities of c2_sigma.npz.  Calls only the oracle and the scene generator.

    python tests/golden/make_c2_samples.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    cfg = scenegen.FMM
    workers = int(os.environ.get("WORKERS", "8"))
    sc = scenegen.sized_scene(n_curves=cfg["n_curves"], n_stops=cfg["n_stops"],
                              seed=cfg["seed"])
    disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"],
                             workers=workers)
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    sigma = np.load(os.path.join(HERE, "c2_sigma.npz"))["sigma"]
    vp = cfg["viewport"]
    W, H = vp[4], vp[5]
    rng = np.random.default_rng(77)
    rows, cols = np.meshgrid(np.arange(17, H, 64), np.arange(40, W, 64), indexing="ij")
    pick = rng.choice(disc.S, size=512, replace=False)
    mid = 0.5 * (disc.seg_p1[pick] + disc.seg_p2[pick])
    xs, ys = oracle.pixel_centres(vp)
    nc = np.clip(np.floor((mid[:, 0] - xs[0]) / (xs[1] - xs[0]) + 0.5).astype(int), 0, W - 1)
    nr = np.clip(np.floor((ys[0] - mid[:, 1]) / (ys[0] - ys[1]) + 0.5).astype(int), 0, H - 1)
    r = np.concatenate([rows.ravel(), nr])
    c = np.concatenate([cols.ravel(), nc])
    pts = np.stack([xs[c], ys[r]], axis=1)
    vals = oracle.evaluate(disc, sigma, up - um, pts, workers=workers)
    np.savez_compressed(os.path.join(HERE, "c2_samples.npz"), rows=r, cols=c, vals=vals)
    print("wrote", len(r), "samples; value range", vals.min(), vals.max())


if __name__ == "__main__":
    main()
