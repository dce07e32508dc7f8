"""dc_render_noalloc: the allocation-free variant of dc_render (fixed device
scratch, every launch on the caller's stream) must give the images of
dc_render bit for bit, on consecutive calls whose second render is smaller
than the first (the fixed scratch keeps the first call's contents)."""
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
    sigma, _ = oracle.solve(disc, up, um)
    s = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=TINY["panels"],
                      gl=TINY["gl"], segs=TINY["segs"], leaf_max=8)
    s.set_densities(sigma)
    q = disc.node_xy[77]
    yield dict(s=s, q=q)
    s.close()


@pytest.mark.parametrize("prec,p,tile", [("f32", 12, 8), ("f64", 24, 8), ("f32", 16, 16)])
def test_noalloc_equals_render_on_two_calls(tiny, prec, p, tile):
    import torch
    s, q = tiny["s"], tiny["q"]
    dt = torch.float64 if prec == "f64" else torch.float32
    ev = dict(method="fmm", precision=prec, p=p, tile_px=tile)
    big = TINY["viewport"]                                   # 256 x 256
    small = (float(q[0]), float(q[1]), 3e-4, 2e-4, 40, 24)   # zoomed on a node
    for vp in (big, small):
        print("noalloc case", prec, p, tile, vp, flush=True)
        want = s.render(vp, out_dtype=dt, **ev)          # also prepares the scene
        got = torch.full_like(want, float("nan"))
        s.render_noalloc(vp, got, **ev)
        torch.cuda.synchronize()
        assert torch.equal(got, want), vp
    # once more on the large viewport after the small one
    want = s.render(big, out_dtype=dt, **ev)
    got = torch.full_like(want, float("nan"))
    s.render_noalloc(big, got, **ev)
    torch.cuda.synchronize()
    assert torch.equal(got, want)


def test_noalloc_refuses_what_it_cannot_do(gpu_lib, tiny):
    import torch
    s = tiny["s"]
    ev = dict(method="fmm", precision="f32", p=12, tile_px=8)
    s.render(TINY["viewport"], **ev)
    # a render whose scratch exceeds the fixed array
    vp = (0.5, 0.5, 1.0, 1.0, 4096, 4096)
    out = torch.empty((16, 16, 3), device="cuda")
    big_out = torch.empty((4096, 4096, 3), device="cuda")
    with pytest.raises(gpu_lib.DcError, match="DC_NOALLOC_SCRATCH_BYTES"):
        s.render_noalloc(vp, big_out, **ev)
    del big_out
    # an order the scene has not been prepared for
    with pytest.raises(gpu_lib.DcError, match="not prepared"):
        s.render_noalloc((0.5, 0.5, 1.0, 1.0, 16, 16), out, method="fmm", precision="f32",
                         p=9, tile_px=8)
    # the scene and the entry point still work afterwards
    want = s.render((0.5, 0.5, 1.0, 1.0, 16, 16), **ev)
    s.render_noalloc((0.5, 0.5, 1.0, 1.0, 16, 16), out, **ev)
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    assert np.isfinite(out.cpu().numpy()).all()
