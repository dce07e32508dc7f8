"""Write tests/golden/c4_golden.npz: FP64 oracle data for the 500-curve
batched-render workload (curves of log-uniform length 0.01..0.5, 4 panels x
16 GL nodes per curve, 80 segments per panel, N = 32,000; 64 zoomed
viewports of 128..2048 pixels a side, zoom 1..1e6, centred on curve
points):

  sigma      oracle densities from the dense LU solve [3][N]
  vp         the 64 viewports (cx, cy, w, h, W, H)
  vid, rows, cols, vals
             sampled pixels (viewport, row, column) and their oracle
             values: per viewport an 8 x 8 stride grid plus the 8 x 8 block
             of pixels around the centre, which lies on a curve, so every
             zoom level has near-singular targets

Calls only the oracle and the seeded scene generator.  Needs ~20 GB of RAM
and some minutes on 8 cores:  python tests/golden/make_c4_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_golden.npz")


def sample_pixels(W, H):
    """8 x 8 stride grid plus the 8 x 8 block around the centre pixel."""
    gr = np.unique(np.linspace(0, H - 1, 8).round().astype(int))
    gc = np.unique(np.linspace(0, W - 1, 8).round().astype(int))
    rr, cc = np.meshgrid(gr, gc, indexing="ij")
    br = np.clip(np.arange(H // 2 - 4, H // 2 + 4), 0, H - 1)
    bc = np.clip(np.arange(W // 2 - 4, W // 2 + 4), 0, W - 1)
    r2, c2 = np.meshgrid(br, bc, indexing="ij")
    rows = np.concatenate([rr.ravel(), r2.ravel()])
    cols = np.concatenate([cc.ravel(), c2.ravel()])
    key = np.unique(rows.astype(np.int64) * W + cols)
    return key // W, key % W


def main():
    cfg = scenegen.BATCH
    workers = int(os.environ.get("WORKERS", "8"))
    sc, vps = scenegen.batch_scene(cfg)
    t0 = time.time()
    disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"],
                             workers=workers)
    print(f"discretize: {time.time() - t0:.1f} s, N={disc.N}, S={disc.S}", flush=True)
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    rep = {}
    t0 = time.time()
    sigma, mu = oracle.solve(disc, up, um, workers=workers, report=rep)
    print(f"solve: {time.time() - t0:.1f} s, rcond={rep.get('rcond')}", flush=True)
    vid, rows, cols, pts = [], [], [], []
    for v, vp in enumerate(vps):
        r, c = sample_pixels(vp[4], vp[5])
        xs, ys = oracle.pixel_centres(vp)
        vid.append(np.full(len(r), v))
        rows.append(r)
        cols.append(c)
        pts.append(np.stack([xs[c], ys[r]], axis=1))
    pts = np.concatenate(pts)
    t0 = time.time()
    vals = oracle.evaluate(disc, sigma, mu, pts, workers=workers)
    print(f"evaluate {len(pts)} px: {time.time() - t0:.1f} s", flush=True)
    print(f"|sigma| max {np.abs(sigma).max():.3e}, values in [{vals.min():.3f}, "
          f"{vals.max():.3f}]", flush=True)
    np.savez_compressed(OUT, sigma=sigma, vp=np.array(vps), vid=np.concatenate(vid),
                        rows=np.concatenate(rows), cols=np.concatenate(cols), vals=vals,
                        rcond=rep.get("rcond", np.nan))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
