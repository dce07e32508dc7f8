"""Write tests/golden/c5_golden.npz: FP64 oracle values for sampled requests
of the serving workload (16 resident scenes of 10 to 5,000 curves, 16 panels
x 16 GL nodes per curve, 80 segments per panel; requests of 256 to 2048
pixels a side at zoom 1 to 1e6 centred on curve points).

The first request of each scene in the request stream is checked at 1,024
pixels: a 16 x 32 stride grid and 512 pixels along the chords that cross the
viewport (points spread along the crossing parts; the near field).  The
largest scenes are far beyond a dense solve, so the densities are the
synthetic ones of scenegen.synthetic_densities with mu = u+ - u- from the
scene's colours (the render of Alg. 4 is defined for any densities).

Stored: req [16] (index in the request stream), scene [16], vp [16, 6],
first [17] (offsets of each request's pixels), rows, cols [n], vals [n, 3].
Calls only the oracle and the seeded scene generator.  About ten minutes on
8 cores:  python tests/golden/make_c5_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_golden.npz")
N_GRID, N_NEAR = 512, 512


def sample(disc, vp, rng):
    cx, cy, w, h, W, H = vp
    gw, gh = 32, 16
    rows = ((np.arange(gh) + 0.5) * H / gh).astype(int)
    cols = ((np.arange(gw) + 0.5) * W / gw).astype(int)
    rr, cc = np.meshgrid(rows, cols, indexing="ij")
    rr, cc = rr.ravel(), cc.ravel()
    # chords crossing the viewport rectangle: clip p1 + t (p2 - p1) to it
    x0, x1, y0, y1 = cx - w / 2, cx + w / 2, cy - h / 2, cy + h / 2
    d = disc.seg_p2 - disc.seg_p1
    ta = np.zeros(disc.S)
    tb = np.ones(disc.S)
    ok = np.ones(disc.S, bool)
    for p, q in ((-d[:, 0], disc.seg_p1[:, 0] - x0), (d[:, 0], x1 - disc.seg_p1[:, 0]),
                 (-d[:, 1], disc.seg_p1[:, 1] - y0), (d[:, 1], y1 - disc.seg_p1[:, 1])):
        zero = p == 0
        ok &= ~(zero & (q < 0))
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(zero, 0.0, q / np.where(zero, 1.0, p))
        ta = np.where(~zero & (p < 0), np.maximum(ta, r), ta)
        tb = np.where(~zero & (p > 0), np.minimum(tb, r), tb)
    ok &= ta <= tb
    idx = np.nonzero(ok)[0]
    if len(idx):
        pick = rng.choice(idx, size=N_NEAR, replace=True)
        t = ta[pick] + (tb[pick] - ta[pick]) * rng.uniform(0.0, 1.0, size=N_NEAR)
        pts = disc.seg_p1[pick] + t[:, None] * d[pick]
        nc = np.clip(np.floor((pts[:, 0] - x0) / (w / W)).astype(int), 0, W - 1)
        nr = np.clip(np.floor((y1 - pts[:, 1]) / (h / H)).astype(int), 0, H - 1)
        rr = np.concatenate([rr, nr])
        cc = np.concatenate([cc, nc])
    return rr, cc


def main():
    cfg = scenegen.SERVING
    workers = int(os.environ.get("WORKERS", "8"))
    raw = scenegen.serving_scenes(n_scenes=cfg["n_scenes"], seed0=cfg["seed0"],
                                  panels=cfg["panels"], gl=cfg["gl"], segs=cfg["segs"])
    reqs = scenegen.serving_requests(raw, cfg["n_requests"] + cfg["n_warmup"], seed=7)
    chosen = {}
    for i, (k, vp) in enumerate(reqs):
        chosen.setdefault(k, i)
    rng = np.random.default_rng(55)
    out_req, out_scene, out_vp, first, R, Cc, V = [], [], [], [0], [], [], []
    for k in range(len(raw)):
        i = chosen[k]
        vp = reqs[i][1]
        sc = raw[k]
        t0 = time.time()
        disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"],
                                 workers=workers)
        up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
        sigma = scenegen.synthetic_densities(disc.N)
        rr, cc = sample(disc, vp, rng)
        xs, ys = oracle.pixel_centres(vp)
        pts = np.stack([xs[cc], ys[rr]], axis=1)
        vals = oracle.evaluate(disc, sigma, up - um, pts, workers=workers)
        print(f"scene {k} ({sc.n_curves} curves, S={disc.S}) request {i} {vp}: "
              f"{len(rr)} px in {time.time() - t0:.1f} s, values in "
              f"[{vals.min():.3f}, {vals.max():.3f}]", flush=True)
        out_req.append(i)
        out_scene.append(k)
        out_vp.append(vp)
        R.append(rr)
        Cc.append(cc)
        V.append(vals)
        first.append(first[-1] + len(rr))
    np.savez_compressed(OUT, req=np.array(out_req), scene=np.array(out_scene),
                        vp=np.array(out_vp), first=np.array(first),
                        rows=np.concatenate(R), cols=np.concatenate(Cc),
                        vals=np.concatenate(V))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
