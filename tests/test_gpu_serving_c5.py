"""Served images of the serving workload against the FP64 oracle.

The 16 resident scenes (10 to 5,000 curves, 16 panels x 16 GL nodes) hold
the synthetic densities of scenegen.synthetic_densities (the oracle cannot
solve the largest ones); each scene's expansion order and tile size are
chosen by dc_autotune on its checked viewport and the scene is registered
with the server under those options.  The first request of every scene in
the request stream is served in a mix with the following requests of the
stream and checked at 1,024 pixels against stored oracle values
(tests/golden/make_c5_golden.py, which calls only the oracle): the FP32 bar
1e-4."""
import os

import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CFG = scenegen.SERVING


@pytest.fixture(scope="module")
def c5(gpu_lib):
    g = np.load(os.path.join(HERE, "golden", "c5_golden.npz"))
    raw = scenegen.serving_scenes(n_scenes=CFG["n_scenes"], seed0=CFG["seed0"],
                                  panels=CFG["panels"], gl=CFG["gl"], segs=CFG["segs"])
    reqs = scenegen.serving_requests(raw, CFG["n_requests"] + CFG["n_warmup"], seed=7)
    scenes = []
    for k, sc in enumerate(raw):
        s = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=CFG["panels"],
                          gl=CFG["gl"], segs=CFG["segs"], leaf_max=32,
                          domain=scenegen.serving_domain(sc))
        s.set_densities(scenegen.synthetic_densities(s.N))
        scenes.append(s)
    yield dict(g=g, reqs=reqs, scenes=scenes)
    for s in scenes:
        s.close()


@pytest.mark.timeout(600)
def test_served_requests_match_oracle(gpu_lib, c5):
    import torch
    g, reqs, scenes = c5["g"], c5["reqs"], c5["scenes"]
    tuned = []
    for j, (i, k) in enumerate(zip(g["req"], g["scene"])):
        vp = reqs[int(i)][1]
        assert np.allclose(vp, g["vp"][j])
        rep = scenes[int(k)].autotune([vp], target_err=5e-5, precision="f32", tiles=(8, 16),
                                      samples=1024, timing_reps=2)
        print(f"scene {int(k)} tuned {rep['eval']} err {rep['err']:.2e} met {rep['met']}",
              flush=True)
        tuned.append(rep)
    srv = gpu_lib.Server(precision="f32", n_streams=4, max_batch=16, hbm_budget=16 << 30)
    try:
        for k, rep in zip(g["scene"], tuned):
            srv.add_scene(scenes[int(k)], **rep["eval"])
        # the checked requests in a mix with the stream's next requests
        last = int(g["req"].max())
        stream = list(range(0, last + 32))
        tickets = {i: srv.submit(scenes[reqs[i][0]], reqs[i][1]) for i in stream}
        worst = 0.0
        for j, i in enumerate(g["req"]):
            info = srv.wait(tickets[int(i)], timeout=300)
            assert info is not None and info["status"] == 0
            img = srv.fetch(tickets.pop(int(i))).cpu().numpy()
            a, b = int(g["first"][j]), int(g["first"][j + 1])
            err = float(np.abs(img[g["rows"][a:b], g["cols"][a:b]] - g["vals"][a:b]).max())
            print(f"request {int(i)} (scene {int(g['scene'][j])}, {reqs[int(i)][1][4]} px, "
                  f"zoom {1 / reqs[int(i)][1][2]:.3g}): max err vs oracle {err:.3e}", flush=True)
            worst = max(worst, err)
        for t in tickets.values():
            assert srv.wait(t, timeout=300)["status"] == 0
            srv.fetch(t)
    finally:
        srv.close()
    print(f"serving workload: worst served-image error vs oracle {worst:.3e}", flush=True)
    assert worst <= 1e-4
