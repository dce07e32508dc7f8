"""Mixed Dirichlet/Neumann conditions on a closed curve (Sec. 5.4,
Eq. neumann_mat) through dc_solve_mixed: u = x^2 - y^2 inside the square
[0.2, 0.8]^2 (counter-clockwise), Dirichlet data on two edges and Neumann
data on the other two.  The solved densities and the rendered interior are
held to the FP64 oracle's dense solve of the same system (oracle.solve_mixed)
and the interior to the harmonic field itself."""
import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

V = np.array([[0.2, 0.2], [0.8, 0.2], [0.8, 0.8], [0.2, 0.8]])
P = 8


@pytest.fixture(scope="module")
def square(gpu_lib):
    ctrl = scenegen.polygon_ctrl(V)
    disc = oracle.discretize(ctrl, P, 16, 80)
    q = disc.node_xy
    edge = np.arange(disc.N) // (P * 16)
    n_out = np.array([[0.0, -1.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])[edge]
    u = q[:, 0] ** 2 - q[:, 1] ** 2
    psi = 2 * q[:, 0] * n_out[:, 0] - 2 * q[:, 1] * n_out[:, 1]
    neumann = (edge == 1) | (edge == 2)
    vals = np.stack([np.where(neumann, psi, u)] * 3) * np.array([[1.0], [2.0], [-1.0]])
    ps, us = oracle.solve_mixed(disc, neumann, vals)
    zeros = np.zeros((ctrl.shape[0], 2, 3))
    s = gpu_lib.Scene(ctrl, zeros, zeros, panels=P, gl=16, segs=80, leaf_max=16)
    yield dict(s=s, disc=disc, neumann=neumann, vals=vals, ps=ps, us=us)
    s.close()


@pytest.mark.parametrize("method,p", [("direct", 20), ("fmm", 28)])
def test_mixed_solve_matches_oracle(square, method, p):
    import torch
    s = square["s"]
    rep = s.solve_mixed(square["neumann"].astype(np.int32), square["vals"], tol=1e-13,
                        max_iter=600, method=method, p=p)
    print(f"mixed {method}:", rep, flush=True)
    assert rep["converged"]
    psi = s.densities()
    e_psi = np.abs(psi - square["ps"]).max() / np.abs(square["ps"]).max()
    vp = (0.5, 0.5, 0.5, 0.5, 40, 40)
    img = s.render(vp, out_dtype=torch.float64, method="fmm", p=28).cpu().numpy()
    xs, ys = oracle.pixel_centres(vp)
    X, Y = np.meshgrid(xs, ys)
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    want = oracle.evaluate(square["disc"], square["ps"], square["us"], pts).reshape(40, 40, 3)
    e_img = np.abs(img - want).max()
    exact = (X ** 2 - Y ** 2)[..., None] * np.array([1.0, 2.0, -1.0])
    e_exact = np.abs(img - exact).max()
    print(f"mixed {method}: psi rel {e_psi:.2e}, render vs oracle {e_img:.2e}, "
          f"vs x^2 - y^2 {e_exact:.2e}", flush=True)
    assert e_psi <= 1e-9
    assert e_img <= 1e-10
    assert e_exact <= 5e-6


def test_two_sided_data_return_after_a_mixed_solve(square):
    """The scene's colours are zero on both sides: once the two-sided solve
    runs again, mu = u+ - u- = 0 replaces the mixed solve's u and the field
    vanishes (with the mixed u still in place it would be x^2 - y^2)."""
    import torch
    s = square["s"]
    s.solve_mixed(square["neumann"].astype(np.int32), square["vals"], tol=1e-10,
                  method="direct")
    rep = s.solve(tol=1e-10, max_iter=500, method="direct", precond="none")
    assert rep["rc"] == 0
    img = s.render((0.5, 0.5, 0.5, 0.5, 16, 16), out_dtype=torch.float64, method="fmm", p=20)
    assert torch.abs(img).max().item() <= 1e-6


def test_mixed_solve_rejects_bad_input(gpu_lib, square):
    s = square["s"]
    bad = square["neumann"].astype(np.int32) * 2
    with pytest.raises(gpu_lib.DcError):
        s.solve_mixed(bad, square["vals"], method="direct")
