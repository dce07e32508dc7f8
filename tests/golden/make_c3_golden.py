"""Write tests/golden/c3_golden.npz: FP64 oracle values for the precision
workload (2,000 curves in 5 Gaussian blobs plus 20 long curves, 32 panels x
16 GL nodes per curve, 80 segments per panel: N = 1,034,240 nodes,
S = 5,171,200 segments; 4096 x 4096 render of [0,1]^2).

A dense solve of this size is out of reach, so the densities are the
synthetic ones of scenegen.synthetic_densities (smooth in the node index),
with mu = u+ - u- from the scene's colours; the file holds

  rows, cols, vals   oracle pixel values at a 64 x 64 stride-64 grid plus
                     1,024 pixels holding chord midpoints
  node_idx, yG, yF   rows of the solve's operator at 256 sampled nodes:
                     yG = G_H x for x = synthetic_densities(N, phase=0.7),
                     yF = F_H mu (self-segment rule included)

Calls only the oracle and the seeded scene generator.  About 20 minutes on
8 cores:  python tests/golden/make_c3_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_golden.npz")


def main():
    cfg = scenegen.PRECISION
    workers = int(os.environ.get("WORKERS", "8"))
    sc = scenegen.clustered_scene(seed=cfg["seed"], panels=cfg["panels"], gl=cfg["gl"],
                                  segs=cfg["segs"])
    t0 = time.time()
    disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"], workers=workers)
    print(f"discretize: {time.time() - t0:.1f} s, N={disc.N}, S={disc.S}", flush=True)
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    mu = up - um
    sigma = scenegen.synthetic_densities(disc.N)
    vp = cfg["viewport"]
    W, H = vp[4], vp[5]
    rng = np.random.default_rng(33)
    rr, cc = np.meshgrid(np.arange(31, H, 64), np.arange(17, W, 64), indexing="ij")
    pick = rng.choice(disc.S, size=1024, replace=False)
    mid = 0.5 * (disc.seg_p1[pick] + disc.seg_p2[pick])
    xs, ys = oracle.pixel_centres(vp)
    nc = np.clip(np.floor((mid[:, 0] - xs[0]) / (xs[1] - xs[0]) + 0.5).astype(int), 0, W - 1)
    nr = np.clip(np.floor((ys[0] - mid[:, 1]) / (ys[0] - ys[1]) + 0.5).astype(int), 0, H - 1)
    rows = np.concatenate([rr.ravel(), nr])
    cols = np.concatenate([cc.ravel(), nc])
    pts = np.stack([xs[cols], ys[rows]], axis=1)
    t0 = time.time()
    vals = oracle.evaluate(disc, sigma, mu, pts, workers=workers)
    print(f"evaluate {len(pts)} px: {time.time() - t0:.1f} s; values in "
          f"[{vals.min():.3f}, {vals.max():.3f}]", flush=True)
    # operator rows at sampled nodes
    node_idx = np.sort(rng.choice(disc.N, size=256, replace=False))
    x = scenegen.synthetic_densities(disc.N, phase=0.7)
    xbar = disc.interpolate(x)     # [3][S]
    mubar = disc.interpolate(mu)
    yG = np.zeros((3, node_idx.size))
    yF = np.zeros((3, node_idx.size))
    t0 = time.time()
    for b in range(0, disc.S, 65536):
        cols_s = np.arange(b, min(disc.S, b + 65536))
        G, F = oracle.node_operator_rows(disc, node_idx, cols_s)
        yG += (G @ xbar[:, cols_s].T).T
        yF += (F @ mubar[:, cols_s].T).T
    print(f"operator rows: {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(OUT, rows=rows, cols=cols, vals=vals, node_idx=node_idx, yG=yG, yF=yF)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
