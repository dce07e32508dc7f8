"""Write tests/golden/c2_sigma.npz: FP64 oracle densities of the 200-curve
FMM workload (16 panels x 16 GL nodes per curve, 80 segments per panel,
N = 51,200), from the dense LU solve of the hybrid collocation system.

Calls only the oracle and the seeded scene generator.  Needs ~25 GB of RAM
and some minutes on 8 cores:  python tests/golden/make_c2_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_sigma.npz")


def main():
    cfg = scenegen.FMM
    workers = int(os.environ.get("WORKERS", "8"))
    sc = scenegen.sized_scene(n_curves=cfg["n_curves"], n_stops=cfg["n_stops"],
                              seed=cfg["seed"])
    t0 = time.time()
    disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"],
                             workers=workers)
    print(f"discretize: {time.time() - t0:.1f} s, N={disc.N}, S={disc.S}", flush=True)
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    rep = {}
    t0 = time.time()
    sigma, mu = oracle.solve(disc, up, um, workers=workers, report=rep)
    print(f"solve: {time.time() - t0:.1f} s, rcond={rep.get('rcond')}", flush=True)
    np.savez_compressed(OUT, sigma=sigma, node_xy=disc.node_xy,
                        rcond=rep.get("rcond", np.nan), seed=cfg["seed"],
                        n_curves=cfg["n_curves"], panels=cfg["panels"], gl=cfg["gl"],
                        segs=cfg["segs"])
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
