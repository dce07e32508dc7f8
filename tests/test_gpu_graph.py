"""Render graphs (dc_render_graph_*): the launches of one batched render
captured into a HIP graph and replayed.  Every replay must equal the eager
render bit for bit (the same kernels on the same inputs), with eager work
and synchronisation between replays; a replay after the densities, or the
resident expansions' order, changed must be refused."""
import os

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TINY = scenegen.TINY
CFG = scenegen.FMM


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
    vps = [TINY["viewport"], (q[0] + 3e-3, q[1] - 1e-3, 1e-2, 1e-2, 64, 48)]
    yield dict(s=s, sigma=sigma, vps=vps, q=q)
    s.close()


@pytest.mark.parametrize("prec,p,tile", [("f32", 12, 8), ("f64", 24, 8), ("f32", 10, 16)])
def test_replays_equal_eager(gpu_lib, tiny, prec, p, tile):
    import torch
    s, vps = tiny["s"], tiny["vps"]
    dt = torch.float64 if prec == "f64" else torch.float32
    ev = dict(method="fmm", precision=prec, p=p, tile_px=tile)
    ref = [o.clone() for o in s.render_batch(vps, out_dtype=dt, **ev)]
    g = s.render_graph(vps, out_dtype=dt, **ev)
    try:
        other = (0.3, 0.4, 0.2, 0.2, 40, 40)
        for r in range(3):
            for o in g.outs:
                o.fill_(float("nan"))
            out = g.launch()
            torch.cuda.synchronize()
            for a, b in zip(out, ref):
                assert torch.equal(a, b), (prec, r)
            # eager work between replays (same options: the graph stays valid)
            s.render(other, out_dtype=dt, **ev)
            torch.cuda.synchronize()
    finally:
        g.close()


def test_stale_graph_is_refused(gpu_lib, tiny):
    import torch
    s, vps = tiny["s"], tiny["vps"]
    ev = dict(method="fmm", precision="f32", p=12, tile_px=8)
    ref = [o.clone() for o in s.render_batch(vps, **ev)]
    g = s.render_graph(vps, **ev)
    try:
        # another order rebuilds the resident expansions: the graph is stale
        s.render(vps[0], method="fmm", precision="f32", p=14, tile_px=8)
        with pytest.raises(gpu_lib.DcError):
            g.launch()
        s.render(vps[0], **ev)
        with pytest.raises(gpu_lib.DcError):
            g.launch()
        g.close()
        # a graph made again replays the same images
        g = s.render_graph(vps, **ev)
        out = g.launch()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(out, ref))
        # new densities invalidate it
        s.set_densities(tiny["sigma"] * 0.5)
        s.render(vps[0], **ev)
        with pytest.raises(gpu_lib.DcError):
            g.launch()
    finally:
        g.close()
        s.set_densities(tiny["sigma"])


def test_large_render_graph_uses_both_streams(gpu_lib):
    """2048^2 at 8-px tiles (72,900 tiles): the captured pass forks the
    queued heavy tiles onto the scene's second stream and joins them."""
    import torch
    g0 = np.load(os.path.join(HERE, "golden", "c2_sigma.npz"))
    sc = scenegen.sized_scene(n_curves=CFG["n_curves"], n_stops=CFG["n_stops"],
                              seed=CFG["seed"])
    s = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=CFG["panels"],
                      gl=CFG["gl"], segs=CFG["segs"], leaf_max=4)
    try:
        s.set_densities(g0["sigma"])
        ev = dict(method="fmm", precision="f32", p=12, tile_px=8)
        ref = s.render(CFG["viewport"], **ev).clone()
        g = s.render_graph([CFG["viewport"]], **ev)
        try:
            for r in range(3):
                g.outs[0].zero_()
                out = g.launch()[0]
                torch.cuda.synchronize()
                assert torch.equal(out, ref), r
                s.render((0.5, 0.5, 0.25, 0.25, 512, 512), **ev)
                torch.cuda.synchronize()
        finally:
            g.close()
    finally:
        s.close()
