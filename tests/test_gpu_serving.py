"""Serving loop: continuous batching over resident scenes.

Every result must be the same alone and in a mix of other requests (bit for
bit: a request is rendered by the same kernels with the same arithmetic
whatever else shares its batch), equal to dc_render of its viewport, and
within the FP32 bar of the FP64 oracle.  Admission by device footprint is
exercised with a budget that holds only a few images at once."""
import threading
import time

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

TINY = scenegen.TINY
EV = dict(precision="f32", p=12, tile_px=8)


@pytest.fixture(scope="module")
def scenes(gpu_lib):
    """Three small resident scenes; the first with oracle densities."""
    out = []
    sc = scenegen.uniform_scene(n_curves=TINY["n_curves"], n_stops=TINY["n_stops"],
                                seed=TINY["seed"])
    disc = oracle.discretize(sc["ctrl"], TINY["panels"], TINY["gl"], TINY["segs"])
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    sigma, mu = oracle.solve(disc, up, um)
    s0 = gpu_lib.Scene(sc["ctrl"], sc["left"], sc["right"], panels=TINY["panels"],
                       gl=TINY["gl"], segs=TINY["segs"], leaf_max=16)
    s0.set_densities(sigma)
    out.append(s0)
    for n, seed in ((30, 101), (60, 102)):
        sz = scenegen.sized_scene(n_curves=n, seed=seed, panels=4)
        s = gpu_lib.Scene(sz["ctrl"], sz["left"], sz["right"], panels=4, leaf_max=32)
        rep = s.solve(tol=1e-10, max_iter=500, method="fmm", p=20)
        assert rep["converged"]
        out.append(s)
    yield dict(scenes=out, disc=disc, sigma=sigma, mu=mu)
    for s in out:
        s.close()


def _random_viewports(rng, n, centres):
    vps = []
    for _ in range(n):
        side = int(rng.choice([16, 33, 64, 128, 256]))
        z = 10.0 ** rng.uniform(0, 5)
        c = centres[rng.integers(len(centres))]
        vps.append((float(c[0]), float(c[1]), 1.0 / z, 1.0 / z, side, side))
    return vps


def test_alone_equals_in_mix(gpu_lib, scenes):
    import torch
    ss = scenes["scenes"]
    rng = np.random.default_rng(5)
    centres = scenes["disc"].node_xy[::7]
    probe = (float(centres[3][0]), float(centres[3][1]), 1e-3, 1e-3, 64, 64)
    srv = gpu_lib.Server(**EV, n_streams=4, max_batch=8)
    try:
        for s in ss:
            srv.add_scene(s)
        t = srv.submit(ss[0], probe)
        assert srv.wait(t, timeout=60) is not None
        alone = srv.fetch(t)
        # the mix: 40 requests over all scenes with the probe in the middle
        mix = [(ss[int(rng.integers(3))], vp) for vp in _random_viewports(rng, 40, centres)]
        mix.insert(17, (ss[0], probe))
        tickets = [srv.submit(s, vp) for s, vp in mix]
        infos = [srv.wait(t, timeout=120) for t in tickets]
        assert all(i is not None and i["status"] == 0 for i in infos)
        imgs = [srv.fetch(t) for t in tickets]
        st = srv.stats()
        print("server stats", st, "batch sizes", sorted({i["batch_size"] for i in infos}),
              flush=True)
        assert torch.equal(imgs[17], alone)
        # batches held several requests, and several batches overlapped
        assert max(i["batch_size"] for i in infos) > 1
        # every result equals a plain dc_render of its viewport
        for (s, vp), img in zip(mix, imgs):
            ref = s.render(vp, method="fmm", **EV)
            assert torch.equal(img, ref), vp
    finally:
        srv.close()
    # parity of the probe with the FP64 oracle
    rows = np.arange(0, 64, 9)
    cols = np.arange(3, 64, 9)
    want = oracle.render(scenes["disc"], scenes["sigma"], scenes["mu"], probe, rows=rows,
                         cols=cols)
    err = np.abs(alone.cpu().numpy()[np.ix_(rows, cols)] - want).max()
    print(f"probe vs oracle {err:.3e}", flush=True)
    assert err <= 1e-4


def test_admission_by_footprint(gpu_lib, scenes):
    """A budget of a few images: requests wait for memory instead of failing,
    and the arena never holds more than the budget."""
    import torch
    ss = scenes["scenes"]
    budget = 6 << 20     # 6 MiB: a 256^2 FP32 image is 768 KiB plus scratch
    srv = gpu_lib.Server(**EV, n_streams=2, max_batch=4, hbm_budget=budget)
    try:
        for s in ss:
            srv.add_scene(s)
        with pytest.raises(gpu_lib.DcError) as e:
            srv.submit(ss[0], (0.5, 0.5, 1.0, 1.0, 2048, 2048))   # 48 MiB alone
        assert e.value.code == gpu_lib.DC_ERR_OOM
        vp = [(0.5, 0.5, 1.0, 1.0, 256, 256), (0.4, 0.6, 0.3, 0.3, 256, 256)]
        # all submitted before any fetch: 16 images do not fit, so later
        # requests must wait for fetched images to free the arena
        tickets = [(srv.submit(ss[k % 3], vp[k % 2]), k) for k in range(16)]
        # nothing is fetched yet: images accumulate until the arena is full
        # and the oldest queued request has to wait
        deadline = time.time() + 60
        while srv.stats()["admission_waits"] == 0 and time.time() < deadline:
            time.sleep(0.01)
        st0 = srv.stats()
        print("server stats (arena full)", st0, flush=True)
        assert st0["admission_waits"] >= 1 and st0["completed"] < 16
        for t, k in tickets:
            info = srv.wait(t, timeout=120)
            assert info is not None and info["status"] == 0
            img = srv.fetch(t)
            assert torch.equal(img, ss[k % 3].render(vp[k % 2], method="fmm", **EV))
        st = srv.stats()
        print("server stats (one client)", st, flush=True)
        assert st["bytes_peak"] <= budget and st["bytes_in_use"] == 0
        results = {}

        def client(k):
            # submit, wait, fetch: images leave the arena as they are fetched
            s = ss[k % 3]
            t = srv.submit(s, vp[k % 2])
            info = srv.wait(t, timeout=120)
            results[k] = (info, srv.fetch(t), s, vp[k % 2])

        th = [threading.Thread(target=client, args=(k,)) for k in range(16)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        st = srv.stats()
        print("server stats (16 client threads)", st, flush=True)
        assert st["completed"] == 32 and st["fetched"] == 32
        assert st["bytes_peak"] <= budget and st["bytes_in_use"] == 0
        for info, img, s, v in results.values():
            assert info["status"] == 0
            assert torch.equal(img, s.render(v, method="fmm", **EV))
    finally:
        srv.close()


def test_fetched_images_survive_the_next_batch(gpu_lib, scenes):
    """Large images through a small arena: a fetched image's region is
    handed to the next batch as soon as fetch returns, so the copy out of
    it must have finished by then.  Every image fetched into device memory
    while later batches run equals a plain dc_render of its viewport."""
    import torch
    ss = scenes["scenes"]
    srv = gpu_lib.Server(**EV, n_streams=4, max_batch=2, hbm_budget=160 << 20)
    try:
        for s in ss:
            srv.add_scene(s)
        vps = [(0.5, 0.5, 1.0, 1.0, 1024, 1024), (0.45, 0.55, 0.5, 0.5, 1024, 1024),
               (0.6, 0.4, 0.25, 0.25, 1024, 1024)]
        reqs = [(ss[k % 3], vps[(k // 3) % 3]) for k in range(24)]
        tickets = [srv.submit(s, vp) for s, vp in reqs]
        imgs = []
        for t in tickets:
            info = srv.wait(t, timeout=120)
            assert info is not None and info["status"] == 0
            imgs.append(srv.fetch(t))
        st = srv.stats()
        print("server stats", st, flush=True)
        assert st["admission_waits"] >= 1
        refs = {}
        for (s, vp), img in zip(reqs, imgs):
            key = (id(s), vp)
            if key not in refs:
                refs[key] = s.render(vp, method="fmm", **EV)
            assert torch.equal(img, refs[key]), vp
    finally:
        srv.close()


def test_registered_scene_is_read_only(gpu_lib, scenes):
    s = scenes["scenes"][1]
    srv = gpu_lib.Server(**EV, n_streams=1)
    try:
        srv.add_scene(s)
        with pytest.raises(gpu_lib.DcError):
            s.solve(tol=1e-6, max_iter=10, method="fmm", p=12)
        with pytest.raises(gpu_lib.DcError):
            s.render((0.5, 0.5, 1.0, 1.0, 8, 8), method="fmm", precision="f64", p=20)
        t = srv.submit(s, (0.5, 0.5, 1.0, 1.0, 32, 32))
        assert srv.wait(t, timeout=60)["status"] == 0
        srv.fetch(t)
    finally:
        srv.close()
    # unregistered again: solving is allowed
    rep = s.solve(tol=1e-10, max_iter=500, method="fmm", p=20)
    assert rep["converged"]
