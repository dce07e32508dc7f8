"""Batched render (many viewports of one scene in one set of launches).

Each image of a batch must equal the render of its viewport alone, bit for
bit: the viewports share launches, not arithmetic.  Parity with the FP64
oracle is checked on the tiny scene (sub-grids) and on the full 500-curve,
64-viewport workload (sampled pixels stored by tests/golden/make_c4_golden.py,
which calls only the oracle)."""
import os

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TINY = scenegen.TINY
C4 = scenegen.BATCH


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
    q = disc.node_xy[77]
    vps = [TINY["viewport"],
           (q[0] + 3e-3, q[1] - 1e-3, 1e-2, 1e-2, 64, 48),
           (q[0], q[1], 1e-5, 2e-5, 33, 17),
           (0.3, 0.6, 0.2, 0.1, 1, 1),
           (0.5, 0.5, 0.9, 0.9, 1, 50),
           (q[0] - 1e-7, q[1], 4e-7, 4e-7, 16, 16)]
    yield dict(s=s, disc=disc, sigma=sigma, mu=mu, vps=vps)
    s.close()


@pytest.mark.parametrize("prec,p", [("f64", 40), ("f32", 16)])
def test_batch_equals_alone_bitwise(tiny, prec, p):
    import torch
    dt = torch.float64 if prec == "f64" else torch.float32
    s, vps = tiny["s"], tiny["vps"]
    outs = s.render_batch(vps, out_dtype=dt, method="fmm", precision=prec, p=p)
    for v, img in zip(vps, outs):
        alone = s.render(v, out_dtype=dt, method="fmm", precision=prec, p=p)
        assert torch.equal(img, alone), v
    # a permuted batch gives the same images
    perm = [3, 0, 5, 2, 4, 1]
    outs2 = s.render_batch([vps[i] for i in perm], out_dtype=dt, method="fmm",
                           precision=prec, p=p)
    for j, i in enumerate(perm):
        assert torch.equal(outs2[j], outs[i])


def test_batch_matches_oracle(tiny):
    import torch
    s, vps = tiny["s"], tiny["vps"]
    outs64 = s.render_batch(vps, out_dtype=torch.float64, method="fmm", p=40)
    outs32 = s.render_batch(vps, out_dtype=torch.float32, method="fmm", precision="f32",
                            p=16)
    for v, g64, g32 in zip(vps, outs64, outs32):
        W, H = v[4], v[5]
        rows = np.unique(np.linspace(0, H - 1, min(H, 12)).round().astype(int))
        cols = np.unique(np.linspace(0, W - 1, min(W, 12)).round().astype(int))
        want = oracle.render(tiny["disc"], tiny["sigma"], tiny["mu"], v, rows=rows, cols=cols)
        e64 = np.abs(g64.cpu().numpy()[np.ix_(rows, cols)] - want).max()
        e32 = np.abs(g32.cpu().numpy()[np.ix_(rows, cols)] - want).max()
        print(f"viewport {v}: FP64 {e64:.3e} FP32 {e32:.3e}", flush=True)
        assert e64 <= 1e-10
        assert e32 <= 1e-4


def test_batch_rejects_bad_input(gpu_lib, tiny):
    import torch
    s = tiny["s"]
    with pytest.raises(gpu_lib.DcError):
        s.render_batch([(50.0, 50.0, 1.0, 1.0, 8, 8)], method="fmm")
    with pytest.raises(gpu_lib.DcError):
        s.render_batch([tiny["vps"][0]], method="direct")
    # a rejected batch leaves the scene usable
    img = s.render_batch([tiny["vps"][3]], out_dtype=torch.float64, method="fmm", p=40)[0]
    assert torch.isfinite(img).all()


@pytest.fixture(scope="module")
def c4(gpu_lib):
    g = np.load(os.path.join(HERE, "golden", "c4_golden.npz"))
    sc, vps = scenegen.batch_scene()
    np.testing.assert_array_equal(np.array(vps), g["vp"])
    s = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=C4["panels"],
                      gl=C4["gl"], segs=C4["segs"], leaf_max=16, domain=C4["domain"])
    print("C4 scene", s.info(), "pixels", sum(v[4] * v[5] for v in vps), flush=True)
    yield dict(s=s, vps=vps, g=g)
    s.close()


def _sampled_err(outs, g):
    err = np.zeros(len(outs))
    for v, img in enumerate(outs):
        m = g["vid"] == v
        got = img[g["rows"][m], g["cols"][m]].cpu().numpy()
        err[v] = np.abs(got - g["vals"][m]).max()
    return err


def test_c4_batch_with_oracle_densities(c4):
    import torch
    s, vps, g = c4["s"], c4["vps"], c4["g"]
    s.set_densities(g["sigma"])
    outs = s.render_batch(vps, method="fmm", precision="f32", p=16, tile_px=16)
    e32 = _sampled_err(outs, g)
    del outs
    outs = s.render_batch(vps, out_dtype=torch.float64, method="fmm", p=28, tile_px=16)
    e64 = _sampled_err(outs, g)
    print(f"C4 batch vs oracle: FP32 max {e32.max():.3e}  FP64 p=28 max {e64.max():.3e}",
          flush=True)
    # spot-check batch == alone on the largest and the most zoomed viewports
    big = int(np.argmax([v[4] for v in vps]))
    deep = int(np.argmin([v[2] for v in vps]))
    for i in {big, deep}:
        alone = s.render(vps[i], out_dtype=torch.float64, method="fmm", p=28, tile_px=16)
        assert torch.equal(alone, outs[i])
    # the FP64 bar (measured 1.2e-11 at p = 28, the library's direct sum
    # agreeing with the oracle to the same 1.2e-11)
    assert e64.max() <= 1e-10
    assert e32.max() <= 1e-4


def test_c4_solve_then_batch(c4):
    s, vps, g = c4["s"], c4["vps"], c4["g"]
    rep = s.solve(tol=1e-10, max_iter=1000, method="fmm", p=20)
    print("C4 FMM GMRES", rep, flush=True)
    assert rep["converged"]
    outs = s.render_batch(vps, method="fmm", precision="f32", p=16, tile_px=16)
    e32 = _sampled_err(outs, g)
    print(f"C4 end-to-end FP32 max {e32.max():.3e}", flush=True)
    assert e32.max() <= 1e-4
