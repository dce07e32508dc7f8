"""Anti-aliased render (Sec. 8): every pixel whose square meets a chord takes
the mean of the representation over its aa x aa sub-square centres, every
other pixel its centre value (the definition in oracle.render_aa).  The
pixels the library anti-aliases are counted against the oracle's edge mask
(an integer decision: exact), and the values are held to the FP64 bar
(1e-10) and the FP32 bar (1e-4) at every edge pixel and at sampled others."""
import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

TINY = scenegen.TINY


@pytest.fixture(scope="module")
def tiny(gpu_lib):
    sc = scenegen.uniform_scene(n_curves=TINY["n_curves"], n_stops=TINY["n_stops"],
                                seed=TINY["seed"])
    disc = oracle.discretize(sc["ctrl"], TINY["panels"], TINY["gl"], TINY["segs"])
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    sigma, mu = oracle.solve(disc, up, um)
    s = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=TINY["panels"],
                      gl=TINY["gl"], segs=TINY["segs"], leaf_max=16)
    s.set_densities(sigma)
    yield dict(s=s, disc=disc, sigma=sigma, mu=mu)
    s.close()


def _viewports(disc):
    q = disc.node_xy[200]
    return [(0.5, 0.5, 1.0, 1.0, 96, 80),                       # whole scene
            (float(q[0]) + 1e-3, float(q[1]), 8e-3, 6e-3, 40, 30)]  # zoomed on a curve


@pytest.mark.parametrize("aa", [2, 4])
def test_aa_matches_oracle(tiny, aa):
    import torch
    s, disc = tiny["s"], tiny["disc"]
    rng = np.random.default_rng(aa)
    for vp in _viewports(disc):
        W, H = vp[4], vp[5]
        mask = oracle.aa_edge_mask(disc, vp)
        img64, rep = s.render_aa(vp, aa=aa, out_dtype=torch.float64, method="fmm", p=28)
        img32, rep32 = s.render_aa(vp, aa=aa, method="fmm", precision="f32", p=12)
        plain = s.render(vp, out_dtype=torch.float64, method="fmm", p=28).cpu().numpy()
        assert rep["aa_pixels"] == int(mask.sum()) == rep32["aa_pixels"]
        er, ec = np.nonzero(mask)
        nr, nc = np.nonzero(~mask)
        pick = rng.choice(len(nr), size=min(48, len(nr)), replace=False)
        rows = np.concatenate([er, nr[pick]])
        cols = np.concatenate([ec, nc[pick]])
        want, edge = oracle.render_aa(disc, tiny["sigma"], tiny["mu"], vp, aa, rows, cols)
        assert np.array_equal(edge, mask[rows, cols])
        g64 = img64.cpu().numpy()
        e64 = np.abs(g64[rows, cols] - want).max()
        e32 = np.abs(img32.cpu().numpy()[rows, cols] - want).max()
        print(f"AA x{aa} {vp}: {rep}; FP64 {e64:.3e} FP32 {e32:.3e}", flush=True)
        assert e64 <= 1e-10
        assert e32 <= 1e-4
        # pixels that no chord meets keep the plain render's value, bit for bit
        assert np.array_equal(g64[~mask], plain[~mask])
        assert rep["aa_pixels"] > 0


def test_aa_rejects_bad_factor(gpu_lib, tiny):
    with pytest.raises(gpu_lib.DcError):
        tiny["s"].render_aa((0.5, 0.5, 1.0, 1.0, 8, 8), aa=1, method="fmm")
