"""Write tests/golden/c3_rows.npz: 4,096 sampled rows of the precision
workload's hybrid system (N = 1,034,240 nodes, S = 5,171,200 segments) from
the FP64 oracle, for checking the solve of that system, which is far beyond
a dense solve:

  node_idx [4096]   sampled collocation nodes
  yG [3, 4096]      rows of G_H x for x = scenegen.synthetic_densities(N, 0.7)
  yF [3, 4096]      rows of F_H mu, mu = u+ - u- from the scene's colours
  half_sum [3, 4096] (u+ + u-)/2 at those nodes, so b = half_sum - yF is the
                    right-hand side of Eq. db_mat_solve at the sampled rows
(self-segment rule of App. C.1, D.3, D.4 included).  Calls only the oracle
and the seeded scene generator.  About ten minutes on 8 cores:
    python tests/golden/make_c3_rows.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_rows.npz")
N_ROWS = 4096

_STATE = {}


def _rows_block(rows):
    disc, xbar, mubar = _STATE["disc"], _STATE["xbar"], _STATE["mubar"]
    yG = np.zeros((3, len(rows)))
    yF = np.zeros((3, len(rows)))
    for b in range(0, disc.S, 65536):
        cols = np.arange(b, min(disc.S, b + 65536))
        G, F = oracle.node_operator_rows(disc, rows, cols)
        yG += (G @ xbar[:, cols].T).T
        yF += (F @ mubar[:, cols].T).T
    return yG, yF


def main():
    cfg = scenegen.PRECISION
    workers = int(os.environ.get("WORKERS", "8"))
    sc = scenegen.clustered_scene(seed=cfg["seed"], panels=cfg["panels"], gl=cfg["gl"],
                                  segs=cfg["segs"])
    disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"],
                             workers=workers)
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    x = scenegen.synthetic_densities(disc.N, phase=0.7)
    rng = np.random.default_rng(44)
    node_idx = np.sort(rng.choice(disc.N, size=N_ROWS, replace=False))
    _STATE.update(disc=disc, xbar=disc.interpolate(x), mubar=disc.interpolate(up - um))
    t0 = time.time()
    blocks = np.array_split(node_idx, 8 * workers)
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_rows_block, blocks)
    yG = np.concatenate([p[0] for p in parts], axis=1)
    yF = np.concatenate([p[1] for p in parts], axis=1)
    print(f"{N_ROWS} rows in {time.time() - t0:.1f} s", flush=True)
    half = 0.5 * (up + um)[:, node_idx]
    np.savez_compressed(OUT, node_idx=node_idx, yG=yG, yF=yF, half_sum=half)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
