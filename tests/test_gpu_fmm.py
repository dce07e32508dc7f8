"""GPU FMM path vs the FP64 oracle (direct sums and dense LU).

The tiny configuration is run with a small leaf capacity so that the tree is
deep and every interaction list of Alg. 8 (interaction, smaller and bigger
separated lists, neighbours) is exercised.  Tolerances: FMM truncation
decays geometrically with p; the FP64 path is held to 1e-10 at p = 40 and
the FP32 path to the 1e-4 bar on [0,1] colours."""
import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

CFG = scenegen.TINY
VP = CFG["viewport"]


@pytest.fixture(scope="module")
def ref():
    sc = scenegen.uniform_scene(n_curves=CFG["n_curves"], n_stops=CFG["n_stops"],
                                seed=CFG["seed"])
    disc = oracle.discretize(sc["ctrl"], CFG["panels"], CFG["gl"], CFG["segs"])
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    sigma, mu = oracle.solve(disc, up, um)
    A, fmu = oracle.assemble(disc, mu)
    # every 4th pixel of the 256^2 viewport plus a dense 32x32 block
    rows = np.unique(np.concatenate([np.arange(0, 256, 4), np.arange(100, 132)]))
    cols = np.unique(np.concatenate([np.arange(1, 256, 4), np.arange(60, 92)]))
    img = oracle.render(disc, sigma, mu, VP, rows=rows, cols=cols)
    return dict(sc=sc, disc=disc, sigma=sigma, mu=mu, A=A, fmu=fmu, rows=rows, cols=cols,
                img=img)


@pytest.fixture(scope="module", params=[8, 64], ids=["leaf8", "leaf64"])
def scene(request, gpu_lib, ref):
    sc = ref["sc"]
    s = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=CFG["panels"],
                      gl=CFG["gl"], segs=CFG["segs"], leaf_max=request.param)
    print("scene", s.info(), flush=True)
    yield s
    s.close()


def test_fmm_operator_converges_with_p(scene, ref):
    import torch
    rng = np.random.default_rng(3)
    x = rng.normal(size=(3, ref["disc"].N))
    yref = (ref["A"] @ x.T).T
    scale = np.abs(yref).max()
    xt = torch.tensor(x, device="cuda")
    errs = {}
    for p in (8, 16, 24, 32, 40):
        y = scene.apply_operator(xt, method="fmm", p=p).cpu().numpy()
        errs[p] = np.abs(y - yref).max() / scale
    print("relative operator error vs p", errs, flush=True)
    assert errs[16] < errs[8] and errs[32] < errs[16]
    assert errs[40] < 1e-11
    y32 = scene.apply_operator(xt, method="fmm", p=16, precision="f32").cpu().numpy()
    e32 = np.abs(y32 - yref).max() / scale
    print("FP32 operator error p=16", e32, flush=True)
    assert e32 < 1e-5


def test_fmm_double_layer_operator(scene, ref):
    import torch
    zero = torch.zeros((3, ref["disc"].N), dtype=torch.float64, device="cuda")
    y = scene.apply_operator(zero, c_mu=1, method="fmm", p=40).cpu().numpy()
    fmu = ref["fmu"].T
    assert np.abs(y - fmu).max() <= 1e-11 * max(1.0, np.abs(fmu).max())


def _sub(img, ref):
    return img[np.ix_(ref["rows"], ref["cols"])]


def test_fmm_render_fp64_with_oracle_densities(scene, ref):
    import torch
    scene.set_densities(ref["sigma"])
    errs = {}
    for p in (20, 40):
        img = scene.render(VP, out_dtype=torch.float64, method="fmm", p=p).cpu().numpy()
        errs[p] = np.abs(_sub(img, ref) - ref["img"]).max()
    print("render FP64 errors", errs, flush=True)
    assert errs[40] <= 1e-10


@pytest.mark.parametrize("tile", [4, 8, 16])
def test_fmm_render_fp32_with_oracle_densities(scene, ref, tile):
    import torch
    scene.set_densities(ref["sigma"])
    img = scene.render(VP, out_dtype=torch.float32, method="fmm", p=16, precision="f32",
                       tile_px=tile).cpu().numpy()
    err = np.abs(_sub(img, ref) - ref["img"]).max()
    print(f"render FP32 tile {tile} error {err:.3e}", flush=True)
    assert err <= 1e-4


def test_fmm_solve_and_render_end_to_end(scene, ref):
    import torch
    rep = scene.solve(tol=1e-13, max_iter=512, method="fmm", p=40)
    print("FMM GMRES", rep, flush=True)
    assert rep["converged"]
    img = scene.render(VP, out_dtype=torch.float64, method="fmm", p=40).cpu().numpy()
    err = np.abs(_sub(img, ref) - ref["img"]).max()
    print("end-to-end FP64 error", err, flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("zoom", [1e2, 1e4, 1e6])
def test_zoomed_viewports(scene, ref, zoom):
    """Deep zoom near a curve: the target tree descends far below the source
    leaves; 33 x 17 pixels so tiles are ragged at two edges."""
    import torch
    scene.set_densities(ref["sigma"])
    q = ref["disc"].node_xy[123] + np.array([0.37, -0.21]) / zoom
    vp = (q[0], q[1], 1.0 / zoom, 0.5 / zoom, 33, 17)
    want = oracle.render(ref["disc"], ref["sigma"], ref["mu"], vp)
    g64 = scene.render(vp, out_dtype=torch.float64, method="fmm", p=40).cpu().numpy()
    g32 = scene.render(vp, out_dtype=torch.float32, method="fmm", p=16,
                       precision="f32").cpu().numpy()
    e64, e32 = np.abs(g64 - want).max(), np.abs(g32 - want).max()
    print(f"zoom {zoom:g}: FP64 {e64:.3e} FP32 {e32:.3e}", flush=True)
    assert e64 <= 1e-10
    assert e32 <= 1e-4


def test_viewport_outside_root_is_rejected(gpu_lib, scene, ref):
    scene.set_densities(ref["sigma"])
    with pytest.raises(gpu_lib.DcError) as e:
        scene.render((50.0, 50.0, 1.0, 1.0, 8, 8), method="fmm")
    assert e.value.code == gpu_lib.DC_ERR_INVALID


def test_render_counts_are_consistent(scene, ref):
    scene.set_densities(ref["sigma"])
    c = scene.render_counts(VP, method="fmm", p=16, precision="f32")
    print("work counts", c, flush=True)
    # every pixel is evaluated from an incoming expansion exactly once
    assert c["l2p_targets"] == 256 * 256
    assert c["p2p_pairs"] > 0 and c["m2l_pairs"] > 0
    assert c["p2l_fp64_pairs"] <= c["p2l_pairs"]
    c64 = scene.render_counts(VP, method="fmm", p=16, precision="f64")
    # the FP64 path takes every incoming-from-source term in FP64; the tree
    # walk is the same
    assert c64["p2l_fp64_pairs"] == c64["p2l_pairs"] == c["p2l_pairs"]
    assert c64["m2l_pairs"] == c["m2l_pairs"]


def test_block_preconditioner_same_solution(gpu_lib, ref):
    """Right block-Jacobi preconditioning changes the iteration, not the
    solution of the hybrid system."""
    sc = ref["sc"]
    s = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=CFG["panels"],
                      gl=CFG["gl"], segs=CFG["segs"], leaf_max=16)
    r0 = s.solve(tol=1e-13, max_iter=512, method="fmm", p=40, precond="none")
    s0 = s.densities()
    r1 = s.solve(tol=1e-13, max_iter=512, method="fmm", p=40, precond="block")
    s1 = s.densities()
    print("iterations none/block", r0["iters"], r1["iters"], flush=True)
    assert r0["converged"] and r1["converged"]
    assert max(r1["iters"]) < max(r0["iters"])
    scale = np.abs(ref["sigma"]).max()
    assert np.abs(s1 - ref["sigma"]).max() <= 1e-8 * scale
    assert np.abs(s0 - s1).max() <= 1e-8 * scale
    s.close()


@pytest.mark.parametrize("precond", ["none", "block"])
def test_gmres_step_limits(gpu_lib, ref, precond):
    """GMRES capped at 1, 2, 3 and 8 Arnoldi steps (each step is queued
    before the host has read the previous one): every channel stops at the
    cap, unconverged, and the residual shrinks with the cap; the GMRES
    estimate agrees with the recomputed residual.  A tolerance the initial
    guess already meets takes no step."""
    sc = ref["sc"]
    s = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=CFG["panels"],
                      gl=CFG["gl"], segs=CFG["segs"], leaf_max=16)
    try:
        ev = dict(method="fmm", p=40, precond=precond)
        prev = None
        for m in (1, 2, 3, 8):
            r = s.solve(tol=1e-14, max_iter=m, **ev)
            print(f"{precond} max_iter {m}: iters {r['iters']}, estimate {r['rel_residual']}, "
                  f"recomputed {r['true_rel_residual']}", flush=True)
            assert not r["converged"] and r["iters"] == [m, m, m]
            est, true = np.array(r["rel_residual"]), np.array(r["true_rel_residual"])
            assert np.all(np.abs(est - true) <= 1e-6 + 1e-6 * true)
            if prev is not None:
                assert np.all(true <= prev * (1 + 1e-12))
            prev = true
        r = s.solve(tol=1e3, max_iter=50, **ev)
        assert r["converged"] and r["iters"] == [0, 0, 0]
    finally:
        s.close()
