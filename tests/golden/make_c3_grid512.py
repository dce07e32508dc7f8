"""Write tests/golden/c3_grid512.npz: FP64 oracle values of the precision
workload's 4096 x 4096 render on the 512 x 512 stride-8 subsample (pixel
rows and columns 4, 12, ..., 4092), with the synthetic densities of
scenegen.synthetic_densities and mu = u+ - u- from the scene's colours (no
dense solve exists at N = 1,034,240).

262,144 pixels x 5,171,200 segments = 1.36e12 closed-form pairs: hours on
8 cores.  The work is split into blocks of rows kept under $C3_GRID_TMP
(default /tmp/c3_grid512), so an interrupted run resumes where it stopped.
Calls only the oracle and the seeded scene generator:
    WORKERS=8 python tests/golden/make_c3_grid512.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_grid512.npz")
STRIDE, OFF, BLOCK = 8, 4, 8   # pixel stride, first pixel, grid rows per block


def main():
    cfg = scenegen.PRECISION
    workers = int(os.environ.get("WORKERS", "8"))
    tmp = os.environ.get("C3_GRID_TMP", "/tmp/c3_grid512")
    os.makedirs(tmp, exist_ok=True)
    sc = scenegen.clustered_scene(seed=cfg["seed"], panels=cfg["panels"], gl=cfg["gl"],
                                  segs=cfg["segs"])
    disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"],
                             workers=workers)
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    sigma = scenegen.synthetic_densities(disc.N)
    vp = cfg["viewport"]
    W, H = vp[4], vp[5]
    rows = np.arange(OFF, H, STRIDE)
    cols = np.arange(OFF, W, STRIDE)
    xs, ys = oracle.pixel_centres(vp)
    for b0 in range(0, len(rows), BLOCK):
        path = os.path.join(tmp, f"rows{b0:04d}.npy")
        if os.path.exists(path):
            continue
        t0 = time.time()
        rr, cc = np.meshgrid(rows[b0:b0 + BLOCK], cols, indexing="ij")
        pts = np.stack([xs[cc.ravel()], ys[rr.ravel()]], axis=1)
        vals = oracle.evaluate(disc, sigma, up - um, pts, workers=workers, pt_chunk=256)
        np.save(path + ".tmp.npy", vals.reshape(len(rr), len(cols), 3))
        os.replace(path + ".tmp.npy", path)
        print(f"grid rows {b0}..{b0 + len(rr) - 1}: {time.time() - t0:.1f} s", flush=True)
    vals = np.concatenate([np.load(os.path.join(tmp, f"rows{b0:04d}.npy"))
                           for b0 in range(0, len(rows), BLOCK)])
    np.savez_compressed(OUT, rows=rows, cols=cols, vals=vals)
    print("wrote", OUT, vals.shape, flush=True)


if __name__ == "__main__":
    main()
