"""GPU direct-sum path vs the FP64 oracle on the tiny configuration
(8 random cubic Beziers, 4 panels x 16 GL nodes, 80 segments per panel,
256 x 256 pixels over [0,1]^2).  Tolerances: FP64 path <= 1e-10 absolute on
pixel values (the bar stated for the FP64 path), operator entries at
rounding level."""
import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

CFG = scenegen.TINY


@pytest.fixture(scope="module")
def tiny():
    sc = scenegen.uniform_scene(n_curves=CFG["n_curves"], n_stops=CFG["n_stops"],
                                seed=CFG["seed"])
    disc = oracle.discretize(sc["ctrl"], CFG["panels"], CFG["gl"], CFG["segs"])
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    sigma, mu = oracle.solve(disc, up, um)
    return dict(sc=sc, disc=disc, up=up, um=um, sigma=sigma, mu=mu)


@pytest.fixture(scope="module")
def oracle_image(tiny):
    print("oracle render of the tiny viewport", flush=True)
    return oracle.render(tiny["disc"], tiny["sigma"], tiny["mu"], CFG["viewport"])


@pytest.fixture(scope="module")
def scene(gpu_lib, tiny):
    s = gpu_lib.Scene(tiny["sc"]["ctrl"], tiny["sc"]["left"], tiny["sc"]["right"],
                      panels=CFG["panels"], gl=CFG["gl"], segs=CFG["segs"])
    yield s
    s.close()


def test_nodes_match_oracle(scene, tiny):
    nodes = scene.nodes()
    np.testing.assert_allclose(nodes, tiny["disc"].node_xy, atol=1e-13, rtol=0)


def test_operator_matches_oracle_matrix(scene, tiny):
    import torch
    disc = tiny["disc"]
    rng = np.random.default_rng(5)
    x = rng.normal(size=(3, disc.N))
    A, fmu = oracle.assemble(disc, tiny["mu"])
    y = scene.apply_operator(torch.tensor(x, device="cuda"), method="direct").cpu().numpy()
    ref = (A @ x.T).T
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    zero = torch.zeros((3, disc.N), dtype=torch.float64, device="cuda")
    yf = scene.apply_operator(zero, c_mu=1, method="direct").cpu().numpy()
    # the double layer is an angle: near chord ends it is conditioned like 1/distance
    assert np.abs(yf - fmu.T).max() <= 1e-11 * max(1.0, np.abs(fmu).max())


def test_direct_solve_matches_lu(scene, tiny):
    rep = scene.solve(tol=1e-14, max_iter=512, method="direct")
    print("GMRES report", rep, flush=True)
    sig = scene.densities()
    ref = tiny["sigma"]
    err = np.abs(sig - ref).max() / np.abs(ref).max()
    assert max(rep["true_rel_residual"]) < 1e-12
    assert err < 1e-9, err


def test_direct_render_with_oracle_densities(scene, tiny, oracle_image):
    import torch
    scene.set_densities(tiny["sigma"])
    img = scene.render(CFG["viewport"], out_dtype=torch.float64, method="direct")
    err = np.abs(img.cpu().numpy() - oracle_image).max()
    print("render max err (oracle densities)", err, flush=True)
    assert err <= 1e-11


def test_direct_render_end_to_end(scene, tiny, oracle_image):
    import torch
    scene.solve(tol=1e-14, max_iter=512, method="direct")
    img = scene.render(CFG["viewport"], out_dtype=torch.float64, method="direct")
    err = np.abs(img.cpu().numpy() - oracle_image).max()
    print("render max err (GPU densities)", err, flush=True)
    assert err <= 1e-10
    img32 = scene.render(CFG["viewport"], out_dtype=torch.float32, method="direct")
    assert np.abs(img32.cpu().numpy() - oracle_image).max() <= 1e-6


def test_render_before_solve_is_rejected(gpu_lib, tiny):
    s = gpu_lib.Scene(tiny["sc"]["ctrl"], tiny["sc"]["left"], tiny["sc"]["right"],
                      panels=2, gl=8, segs=40)
    with pytest.raises(gpu_lib.DcError) as e:
        s.render((0.5, 0.5, 1.0, 1.0, 8, 8), method="direct")
    assert e.value.code == gpu_lib.DC_ERR_INVALID
    s.close()


def test_gmres_max_iter_reports_not_converged(gpu_lib, tiny):
    s = gpu_lib.Scene(tiny["sc"]["ctrl"], tiny["sc"]["left"], tiny["sc"]["right"],
                      panels=2, gl=8, segs=40)
    rep = s.solve(tol=1e-14, max_iter=2, method="direct")
    assert rep["rc"] == gpu_lib.DC_ERR_NOT_CONVERGED and not rep["converged"]
    assert rep["iters"] == [2, 2, 2]
    s.close()
