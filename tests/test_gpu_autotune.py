"""dc_autotune: the order and tile size it picks against the library's own
FP64 direct sum must hold against the FP64 oracle on pixels it never saw
(the stored oracle samples are held out from the tuner's samples)."""
import os

import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
CFG = scenegen.FMM
VP = CFG["viewport"]


@pytest.fixture(scope="module")
def c2(gpu_lib):
    s = np.load(os.path.join(GOLD, "c2_sigma.npz"))
    t = np.load(os.path.join(GOLD, "c2_samples.npz"))
    sc = scenegen.sized_scene(n_curves=CFG["n_curves"], n_stops=CFG["n_stops"],
                              seed=CFG["seed"])
    scn = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=CFG["panels"],
                        gl=CFG["gl"], segs=CFG["segs"], leaf_max=4)
    scn.set_densities(s["sigma"])
    yield dict(s=scn, rows=t["rows"], cols=t["cols"], vals=t["vals"])
    scn.close()


def test_autotune_fp32_holds_on_held_out_oracle_pixels(c2):
    s = c2["s"]
    rep = s.autotune([VP], target_err=5e-5, precision="f32", tiles=(8, 16), samples=2048)
    print("C2 autotune FP32", rep, flush=True)
    assert rep["met"] and rep["err"] <= 5e-5
    assert rep["eval"]["tile_px"] in (8, 16) and 8 <= rep["eval"]["p"] <= 24
    img = s.render(VP, **rep["eval"]).cpu().numpy()
    e = np.abs(img[c2["rows"], c2["cols"]] - c2["vals"]).max()
    print(f"C2 tuned FP32 render vs oracle (held out): {e:.3e}", flush=True)
    assert e <= 1e-4


def test_autotune_fp64_reaches_1e10(c2):
    import torch
    s = c2["s"]
    rep = s.autotune([VP], target_err=1e-10, precision="f64", p_min=20, p_max=40, p_step=4,
                     tiles=(8,), samples=1024, timing_reps=1)
    print("C2 autotune FP64", rep, flush=True)
    assert rep["met"] and rep["eval"]["p"] <= 32
    img = s.render(VP, out_dtype=torch.float64, **rep["eval"]).cpu().numpy()
    z = np.load(os.path.join(GOLD, "c2_sensitivity.npz"))
    e = np.abs(img[c2["rows"], c2["cols"]] - c2["vals"]).max()
    assert e <= 1e-10 + z["render"].max()


def test_autotune_zoomed_viewports(gpu_lib):
    """Eight of the batch workload's zoomed viewports (zoom 1 to 1e6) tuned
    together, checked against the stored oracle pixels of those viewports."""
    g = np.load(os.path.join(GOLD, "c4_golden.npz"))
    sc, vps = scenegen.batch_scene()
    C4 = scenegen.BATCH
    s = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=C4["panels"], gl=C4["gl"],
                      segs=C4["segs"], leaf_max=8, domain=C4["domain"])
    s.set_densities(g["sigma"])
    pick = list(range(0, 64, 8))
    sub = [vps[i] for i in pick]
    rep = s.autotune(sub, target_err=5e-5, precision="f32", tiles=(8, 16), samples=512)
    print("C4 autotune", rep, flush=True)
    assert rep["met"]
    outs = s.render_batch(sub, **rep["eval"])
    worst = 0.0
    for v, img in zip(pick, outs):
        m = g["vid"] == v
        got = img[g["rows"][m], g["cols"][m]].cpu().numpy()
        worst = max(worst, float(np.abs(got - g["vals"][m]).max()))
    print(f"C4 tuned render vs oracle (held out): {worst:.3e}", flush=True)
    assert worst <= 1e-4
    s.close()


def test_autotune_rejects_bad_options(gpu_lib, c2):
    s = c2["s"]
    with pytest.raises(gpu_lib.DcError):
        s.autotune([VP], p_min=10, p_max=8)
    with pytest.raises(gpu_lib.DcError):
        s.autotune([VP], tiles=(1,))
    with pytest.raises(gpu_lib.DcError):
        s.autotune([VP], target_err=0.0)
