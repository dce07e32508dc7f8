"""Write tests/golden/c3_grid512.npz: FP64 oracle values of the precision
workload's 4096 x 4096 render on the 512 x 512 stride-8 subsample (pixel
rows and columns 4, 12, ..., 4092), with the synthetic densities of
scenegen.synthetic_densities and mu = u+ - u- from the scene's colours (no
dense solve exists at N = 1,034,240).

262,144 pixels x 5,171,200 segments = 1.36e12 closed-form pairs: many
hours on 8 cores.  The work is split into blocks of 8 grid rows kept under
$C3_GRID_TMP (default /tmp/c3_grid512), taken in bit-reversed order so that
the blocks done so far spread over the whole image, and an interrupted run
resumes where it stopped.  With PARTIAL=1 the golden is written from the
blocks present (its `rows` array lists the grid rows it holds); otherwise
every block is computed first.  Calls only the oracle and the seeded scene
generator:
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
    vp = cfg["viewport"]
    rows = np.arange(OFF, vp[5], STRIDE)
    cols = np.arange(OFF, vp[4], STRIDE)
    if os.environ.get("PARTIAL") != "1":
        compute_blocks(cfg, workers, tmp, rows, cols)
    done = [b0 for b0 in range(0, len(rows), BLOCK)
            if os.path.exists(os.path.join(tmp, f"rows{b0:04d}.npy"))]
    vals = np.concatenate([np.load(os.path.join(tmp, f"rows{b0:04d}.npy")) for b0 in done])
    held = np.concatenate([rows[b0:b0 + BLOCK] for b0 in done])
    np.savez_compressed(OUT, rows=held, cols=cols, vals=vals)
    print("wrote", OUT, vals.shape, flush=True)


def compute_blocks(cfg, workers, tmp, rows, cols):
    sc = scenegen.clustered_scene(seed=cfg["seed"], panels=cfg["panels"], gl=cfg["gl"],
                                  segs=cfg["segs"])
    disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"],
                             workers=workers)
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    sigma = scenegen.synthetic_densities(disc.N)
    xs, ys = oracle.pixel_centres(cfg["viewport"])
    n_blocks = len(rows) // BLOCK
    bits = max(1, (n_blocks - 1).bit_length())
    order = sorted(range(n_blocks), key=lambda b: int(format(b, f"0{bits}b")[::-1], 2))
    for b in order:
        b0 = b * BLOCK
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


if __name__ == "__main__":
    main()
