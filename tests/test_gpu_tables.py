"""Cached near-field tables of the solve (Sec. 6.4: operators precomputed
once and reused by every GMRES matvec).  The FP64 operator read from the
tables must agree with the one that walks the tree and evaluates the
closed forms (the same values summed in another order), on the 200-curve
workload at leaf capacities 4 and 64, and the solve must reach the same
densities; the oracle-checked operator tests (test_gpu_c3 and others) run
on the tables by default."""
import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu

CFG = scenegen.FMM


@pytest.fixture(scope="module")
def c2(gpu_lib):
    return scenegen.sized_scene(n_curves=CFG["n_curves"], n_stops=CFG["n_stops"],
                                seed=CFG["seed"])


@pytest.mark.parametrize("leaf", [4, 64])
def test_tables_match_on_the_fly_operator(gpu_lib, c2, leaf):
    """Forced tables at leaf 4 (a sparse near field, which the default skips)
    and default tables at leaf 64 against the on-the-fly operator."""
    import torch
    s = gpu_lib.Scene(c2["ctrl"], c2["left"], c2["right"], panels=CFG["panels"], gl=CFG["gl"],
                      segs=CFG["segs"], leaf_max=leaf)
    try:
        N = s.N
        x = torch.tensor(scenegen.synthetic_densities(N), device="cuda")
        ev = dict(method="fmm", precision="f64", p=20)
        y0 = s.apply_operator(x, c_mu=1, **ev).cpu().numpy()
        assert (s.info()["table_pairs"] > 0) == (leaf == 64)     # the default's choice
        s.set_solve_tables("always")
        y_tab = s.apply_operator(x, c_mu=1, **ev).cpu().numpy()
        info = s.info()
        assert info["table_pairs"] > 0 and info["table_bytes"] > 16 * info["table_pairs"] - 1
        if leaf == 64:
            assert np.array_equal(y0, y_tab)
        s.set_solve_tables("off")
        assert s.info()["table_pairs"] == 0
        y_fly = s.apply_operator(x, c_mu=1, **ev).cpu().numpy()
        assert s.info()["table_pairs"] == 0
        d = np.abs(y_tab - y_fly).max()
        print(f"leaf {leaf}: {info['table_pairs']:,} pairs, {info['table_bytes'] / 2**20:.0f} MiB; "
              f"tables vs on the fly {d:.2e} (max {np.abs(y_fly).max():.2e})", flush=True)
        assert d <= 1e-13 * np.abs(y_fly).max()
        s.set_solve_tables("always")
        y_again = s.apply_operator(x, c_mu=1, **ev).cpu().numpy()
        assert np.array_equal(y_again, y_tab)
    finally:
        s.close()


@pytest.mark.parametrize("leaf", [4, 16, 64])
def test_solve_with_and_without_tables(gpu_lib, c2, leaf):
    s = gpu_lib.Scene(c2["ctrl"], c2["left"], c2["right"], panels=CFG["panels"], gl=CFG["gl"],
                      segs=CFG["segs"], leaf_max=leaf)
    try:
        ev = dict(method="fmm", precision="f64", p=20)
        s.set_solve_tables("always")
        r_tab = s.solve(tol=1e-10, max_iter=1000, **ev)
        sig_tab = s.densities()
        s.set_solve_tables("off")
        r_fly = s.solve(tol=1e-10, max_iter=1000, **ev)
        sig_fly = s.densities()
        d = np.abs(sig_tab - sig_fly).max() / np.abs(sig_fly).max()
        print(f"leaf {leaf}: solve with tables {r_tab['seconds']:.3f} s "
              f"({max(r_tab['iters'])} steps), "
              f"without {r_fly['seconds']:.3f} s ({max(r_fly['iters'])} steps); densities "
              f"differ by {d:.2e} relative", flush=True)
        assert r_tab["converged"] and r_fly["converged"]
        assert abs(max(r_tab["iters"]) - max(r_fly["iters"])) <= 2
        assert d <= 1e-8
    finally:
        s.close()
