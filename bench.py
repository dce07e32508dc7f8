#!/usr/bin/env python3
"""Benchmark: RGB pixels/s of the FP32 FMM render (and the plain FP64 FMM
render) of the 200-curve workload at 2048 x 2048, with max error against the
FP64 oracle on sampled pixels, the roofline figure of the dominant kernel
and the oracle timed on the host cores.

A step is one render of the viewport (per-viewport target tree, downward
pass and leaf evaluation; the densities are solved once before timing, as a
scene is solved once and rendered many times).

    python bench.py [--gpus 1] [--steps 10] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import scenegen  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden", "c2_sigma.npz")
GOLDEN_C4 = os.path.join(ROOT, "tests", "golden", "c4_golden.npz")
METRIC = "RGB pixels/s at max err <=1e-4 vs FP64 oracle; FP32-batched vs plain FP64 FMM"
PEAK_FP32 = 157.3e12   # MI355X FP32 vector (packed) TFLOP/s
PEAK_FP64 = 78.6e12
# Algorithmic flop-equivalents per unit of work (log = 20, atan2 = 30 flops).
FLOP_P2P = 117.0


def measured_traffic(kernel, config, key="hbm_bytes_per_launch"):
    """A per-launch figure of `kernel` (HBM bytes, or VALU wave instructions)
    from the committed rocprofv3 counter summary, or None when it covers
    another kernel or configuration, or the kernel source has changed since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_tile_c2_2048_traffic.txt")
    src = os.path.join(ROOT, "paper_2311_14312_amd", "csrc", "fmm.hip")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("kernel") != kernel or kv.get("config") != config or \
            kv.get("source_sha256") != sha or key not in kv:
        return None
    return float(kv[key])


def valu_issue(kernel, config, kernel_ms):
    """The pass's VALU wave instructions (SQ_INSTS_VALU, committed counter
    summary) per second against the issue peak, 256 CUs x 4 SIMDs x
    2.4 GHz / 4 cycles per wave64 instruction: how close the ALU-bound pass
    runs to instruction issue, independent of the flop weights."""
    n = measured_traffic(kernel, config, "valu_wave_instructions_per_launch")
    if n is None:
        return None
    peak = 256 * 4 * 2.4e9 / 4
    rate = n / (kernel_ms * 1e-3)
    return {"wave_instructions": n, "achieved_per_s": rate, "peak_per_s": peak,
            "frac": rate / peak}


def flops_l2p(p):
    return 6 * p + 12 * (p + 1)


def flops_m2p(p):
    return 6 * p + 12 * (p + 1) + 10 + 20


def leaf_flops(c, p):
    return (c["p2p_pairs"] * FLOP_P2P + c["m2p_pairs"] * flops_m2p(p)
            + c["l2p_targets"] * flops_l2p(p))


def p64_of(args):
    """FP64 order of the side workloads: 28 reaches the FP64 bar on them
    (measured against the oracle and the device's direct sum)."""
    return args.p64 if args.p64 > 0 else 28


def sample_pixels(W, H, segs_p1, segs_p2, rng, n_near=4096, stride=16):
    rows, cols = np.meshgrid(np.arange(stride // 2, H, stride),
                             np.arange(stride // 2, W, stride), indexing="ij")
    pick = rng.choice(segs_p1.shape[0], size=n_near, replace=False)
    mid = 0.5 * (segs_p1[pick] + segs_p2[pick])
    nc = np.clip(np.floor(mid[:, 0] * W).astype(int), 0, W - 1)
    nr = np.clip(np.floor((1.0 - mid[:, 1]) * H).astype(int), 0, H - 1)
    r = np.concatenate([rows.ravel(), nr])
    c = np.concatenate([cols.ravel(), nc])
    return r, c


def cpu_model():
    """Host CPU model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, sc, workers):
    """Oracle on the host cores: discretisation, then the direct-sum render
    of a bounded pixel sample (timed) with the golden oracle densities.
    One worker process per core, each with one BLAS thread (set before the
    workers are forked), so `workers` is the number of threads used."""
    import oracle
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        return _cpu_baseline(oracle, cfg, sc, workers)


def _cpu_baseline(oracle, cfg, sc, workers):
    t0 = time.time()
    disc = oracle.discretize(sc["ctrl"], cfg["panels"], cfg["gl"], cfg["segs"], workers=workers)
    t_disc = time.time() - t0
    up, um = oracle.boundary_values(disc, sc["left"], sc["right"])
    mu = up - um
    have_golden = os.path.exists(GOLDEN)
    if have_golden:
        sigma = np.load(GOLDEN)["sigma"]
    else:
        sigma = np.ones((3, disc.N))
    vp = cfg["viewport"]
    rng = np.random.default_rng(2024)
    rows, cols = sample_pixels(vp[4], vp[5], disc.seg_p1, disc.seg_p2, rng)
    xs, ys = oracle.pixel_centres(vp)
    pts = np.stack([xs[cols], ys[rows]], axis=1)
    t0 = time.time()
    vals = oracle.evaluate(disc, sigma, mu, pts, workers=workers)
    t_eval = time.time() - t0
    return dict(rows=rows, cols=cols, vals=vals if have_golden else None,
                value=len(pts) / t_eval, seconds=t_eval, n=len(pts), S=disc.S,
                t_disc=t_disc, golden=have_golden)


def batch_bench(args, torch, dcfmm):
    """The 500-curve scene with 64 zoomed viewports (128..2048 px a side,
    zoom 1..1e6): one batched FP32 render of all viewports vs the same
    viewports rendered one at a time (FP32, and the plain FP64 FMM).  Order
    and leaf capacity are autotuned against the stored oracle samples."""
    cfg = scenegen.BATCH
    sc, vps = scenegen.batch_scene(cfg)
    gold = np.load(GOLDEN_C4) if os.path.exists(GOLDEN_C4) else None
    px = sum(v[4] * v[5] for v in vps)
    outs = [torch.empty((v[5], v[4], 3), device="cuda", dtype=torch.float32) for v in vps]

    def err(imgs):
        if gold is None:
            return None
        e = 0.0
        for v, img in enumerate(imgs):
            m = gold["vid"] == v
            got = img[gold["rows"][m], gold["cols"][m]].cpu().numpy()
            e = max(e, float(np.abs(got - gold["vals"][m]).max()))
        return e

    def time_it(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    tune, best, scenes = [], None, {}
    for leaf in [int(v) for v in args.batch_leaves.split(",")]:
        scn = dcfmm.Scene(sc["ctrl"], sc["left"], sc["right"], panels=cfg["panels"],
                          gl=cfg["gl"], segs=cfg["segs"], leaf_max=leaf,
                          domain=cfg["domain"])
        if gold is not None:
            scn.set_densities(gold["sigma"])
            rep = None
        else:
            rep = scn.solve(tol=1e-10, max_iter=1000, method="fmm", p=20)
        scenes[leaf] = (scn, rep)
        # order and tile size from dc_autotune over all 64 viewports (its own
        # sampled pixels against the device's FP64 direct sum); the stored
        # oracle pixels stay held out for the reported error
        tr = scn.autotune(vps, target_err=5e-5, precision="f32", p_min=8, p_max=24, p_step=2,
                          tiles=(8, 16), samples=256, timing_reps=2)
        ev = tr["eval"]
        ms = time_it(lambda: scn.render_batch(vps, outs=outs, **ev), 3, 1)
        tune.append({"leaf": leaf, "tile": ev["tile_px"], "p": ev["p"], "ms": ms,
                     "tuner_err": tr["err"], "tuner_samples": tr["n_samples"]})
        print("batch autotune", tune[-1], flush=True)
        if best is None or ms < best["ms"]:
            best = dict(tune[-1])
    scn, rep = scenes[best["leaf"]]
    ev32 = dict(method="fmm", precision="f32", p=best["p"], tile_px=best["tile"])
    ms_batch = time_it(lambda: scn.render_batch(vps, outs=outs, **ev32), args.steps,
                       args.warmup)
    e_batch = err(outs)

    def one_by_one(ev, bufs):
        for v, o in zip(vps, bufs):
            scn.render(v, out=o, **ev)

    ms_seq = time_it(lambda: one_by_one(ev32, outs), max(1, args.steps // 2), 1)
    del outs
    outs64 = [torch.empty((v[5], v[4], 3), device="cuda", dtype=torch.float64) for v in vps]
    ev64 = dict(method="fmm", precision="f64", p=p64_of(args), tile_px=best["tile"])
    ms64 = time_it(lambda: one_by_one(ev64, outs64), max(1, args.steps // 4), 1)
    e64 = err(outs64)
    del outs64
    for s_, _ in scenes.values():
        s_.close()
    return {
        "workload": "500 cubic Beziers (lengths log-uniform 0.01-0.5), 4 panels x 16 GL nodes (32,000 nodes), "
                    "64 viewports, side U{128..2048} px, zoom 10^U(0,6), on curve points",
        "pixels": px,
        "value": px / (ms_batch * 1e-3), "unit": "RGB pixels/s", "ms_per_batch": ms_batch,
        "p": best["p"], "tile_px": best["tile"], "leaf_max": best["leaf"],
        "max_err_vs_oracle": e_batch,
        "err_sample": None if gold is None else f"{len(gold['vals'])} oracle pixels "
                                                "(8x8 grid + 8x8 centre block per viewport)",
        "one_at_a_time_fp32": {"value": px / (ms_seq * 1e-3), "ms": ms_seq},
        "one_at_a_time_fp64": {"value": px / (ms64 * 1e-3), "ms": ms64, "p": p64_of(args),
                               "max_err_vs_oracle": e64},
        "densities": "oracle (stored)" if gold is not None else "GPU FMM GMRES",
        "autotune": tune,
    }


def precision_bench(args, torch, dcfmm):
    """The precision workload: 2,000 blob curves plus 20 long curves, 32
    panels x 16 GL nodes (N = 1,034,240), 4096 x 4096 render, FP32 path vs
    plain FP64 FMM, max and RMS error against stored oracle values at 5,120
    sampled pixels (synthetic densities: no dense solve exists at this
    size)."""
    cfg = scenegen.PRECISION
    gold_path = os.path.join(ROOT, "tests", "golden", "c3_golden.npz")
    gold = np.load(gold_path) if os.path.exists(gold_path) else None
    sc = scenegen.clustered_scene(seed=cfg["seed"], panels=cfg["panels"], gl=cfg["gl"],
                                  segs=cfg["segs"])
    t0 = time.time()
    scn = dcfmm.Scene(sc["ctrl"], sc["left"], sc["right"], panels=cfg["panels"], gl=cfg["gl"],
                      segs=cfg["segs"], leaf_max=args.precision_leaf)
    t_create = time.time() - t0
    scn.set_densities(scenegen.synthetic_densities(scn.N))
    vp = cfg["viewport"]
    W, H = vp[4], vp[5]

    def timed(ev, dtype, steps):
        out = torch.empty((H, W, 3), device="cuda", dtype=dtype)
        scn.render(vp, out=out, **ev)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            scn.render(vp, out=out, **ev)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps, out

    def errs(img):
        if gold is None:
            return None, None
        d = img.cpu().numpy()[gold["rows"], gold["cols"]] - gold["vals"]
        return float(np.abs(d).max()), float(np.sqrt(np.mean(d * d)))

    res = {}
    tune = None
    if args.precision_p32 > 0:
        p32 = args.precision_p32
    else:
        # the FP32 order the same way as the headline's: the smallest order
        # in {8, 10, ..., 24} within 5e-5 of the library's own FP64 direct
        # sum at 2,048 sampled pixels (not the oracle's)
        tr = scn.autotune([vp], target_err=5e-5, precision="f32", p_min=8, p_max=24, p_step=2,
                          tiles=(8,), samples=2048, timing_reps=2)
        p32 = tr["eval"]["p"]
        tune = {"p": p32, "tuner_err": tr["err"], "tuner_samples": tr["n_samples"],
                "met": tr["met"]}
        print("precision autotune", tune, flush=True)
    for name, ev, dtype in (
            ("fp32", dict(method="fmm", precision="f32", p=p32, tile_px=8),
             torch.float32),
            ("fp64", dict(method="fmm", precision="f64", p=p64_of(args), tile_px=8),
             torch.float64)):
        ms, img = timed(ev, dtype, 3)
        mx, rms = errs(img)
        del img
        res[name] = {"value": W * H / (ms * 1e-3), "unit": "RGB pixels/s", "ms": ms,
                     "p": ev["p"], "max_err_vs_oracle": mx, "rms_err_vs_oracle": rms}
        print("precision", name, res[name], flush=True)
    info = scn.info()
    scn.close()
    return {
        "workload": "2,000 curves in 5 Gaussian blobs (sigma 0.05, lengths 0.005-0.1) + 20 "
                    "long curves, 32 panels x 16 GL nodes (1,034,240 nodes, 5,171,200 "
                    "segments), 4096x4096 render of [0,1]^2, synthetic densities",
        "leaf_max": args.precision_leaf, "tile_px": 8, "scene_create_s": t_create,
        "autotune": tune,
        "n_pieces": info["n_pieces"], "n_cells": info["n_cells"],
        "err_sample": None if gold is None else f"{len(gold['vals'])} oracle pixels (64x64 "
                                                "stride-64 grid + 1,024 near-chord)",
        **res,
        "speedup_fp32_vs_fp64": res["fp64"]["ms"] / res["fp32"]["ms"],
    }


def serving_bench(args, torch, dcfmm):
    """16 resident scenes of 10..5000 curves; requests of 256..2048 px a side
    at zoom 1..1e6 on curve points.  Capacity is measured with a burst of
    requests; then Poisson arrivals at 0.5x, 1x and 2x capacity, each
    n_warmup + n_requests requests, report p50/p99 latency (submit to
    observed completion) and pixels/s."""
    import threading
    cfg = scenegen.SERVING
    t0 = time.time()
    raw = scenegen.serving_scenes(n_scenes=cfg["n_scenes"], seed0=cfg["seed0"],
                                  panels=cfg["panels"], gl=cfg["gl"], segs=cfg["segs"])
    n_req, n_warm = cfg["n_requests"], cfg["n_warmup"]
    reqs = scenegen.serving_requests(raw, n_req + n_warm, seed=7)
    first_req = {}
    for i, (k, vp) in enumerate(reqs):
        first_req.setdefault(k, i)
    scenes, solve, tuned = [], [], []
    for k, sc in enumerate(raw):
        s = dcfmm.Scene(sc["ctrl"], sc["left"], sc["right"], panels=cfg["panels"],
                        gl=cfg["gl"], segs=cfg["segs"], leaf_max=32,
                        domain=scenegen.serving_domain(sc))
        rep = s.solve(tol=1e-6, max_iter=1000, method="fmm", p=16, raise_on_fail=False)
        # render options of the scene: dc_autotune on its first request of
        # the stream (FP32, target 5e-5 against the device's FP64 direct sum)
        if args.serve_p > 0:
            ev = dict(method="fmm", precision="f32", p=args.serve_p, tile_px=args.serve_tile)
            tr = None
        else:
            tr = s.autotune([reqs[first_req[k]][1]], target_err=5e-5, precision="f32",
                            tiles=(8, 16), samples=1024, timing_reps=2)
            ev = tr["eval"]
        tuned.append(ev)
        solve.append({"curves": int(sc["ctrl"].shape[0]), "N": s.info()["N"],
                      "iters": max(rep["iters"]), "s": round(rep["seconds"], 3),
                      "rel_residual": max(rep["true_rel_residual"]),
                      "converged": bool(rep["converged"]),
                      "p": ev["p"], "tile_px": ev["tile_px"],
                      "tune_err": None if tr is None else tr["err"]})
        print("serving scene", k, solve[-1], flush=True)
        scenes.append(s)
    t_setup = time.time() - t0
    srv = dcfmm.Server(precision="f32", n_streams=4, max_batch=32, max_batch_pixels=1 << 25,
                       hbm_budget=32 << 30)
    for s, ev in zip(scenes, tuned):
        srv.add_scene(s, **ev)
    sink = torch.empty(2048 * 2048 * 3, device="cuda", dtype=torch.float32)

    def fetch(t, vp):
        srv.fetch(t, out=sink[:vp[4] * vp[5] * 3].view(vp[5], vp[4], 3))

    # capacity: everything submitted at once
    t_b = time.time()
    tickets = [srv.submit(scenes[k], vp) for k, vp in reqs[:400]]
    for t, (k, vp) in zip(tickets, reqs[:400]):
        srv.wait(t)
        fetch(t, vp)
    dt = time.time() - t_b
    cap = 400 / dt
    cap_px = sum(vp[4] * vp[5] for _, vp in reqs[:400]) / dt
    print(f"serving capacity {cap:.0f} req/s, {cap_px:.3e} px/s", flush=True)
    runs = []
    for mult in (0.5, 1.0, 2.0):
        rate = mult * cap
        arr = scenegen.poisson_arrivals(len(reqs), rate, seed=11)
        tick = [None] * len(reqs)
        lock = threading.Condition()

        def submitter():
            start = time.perf_counter()
            for i, (k, vp) in enumerate(reqs):
                d = arr[i] - (time.perf_counter() - start)
                if d > 0:
                    time.sleep(d)
                t = srv.submit(scenes[k], vp)
                with lock:
                    tick[i] = t
                    lock.notify()

        th = threading.Thread(target=submitter)
        th.start()
        infos = []
        for i, (k, vp) in enumerate(reqs):
            with lock:
                while tick[i] is None:
                    lock.wait()
            infos.append(srv.wait(tick[i]))
            fetch(tick[i], vp)
        th.join()
        meas = infos[n_warm:]
        lat = np.array([x["t_done"] - x["t_submit"] for x in meas]) * 1e3
        span = max(x["t_done"] for x in meas) - min(x["t_submit"] for x in meas)
        px = sum(vp[4] * vp[5] for _, vp in reqs[n_warm:])
        runs.append({"load": mult, "rate_req_s": rate, "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                     "pixels_per_s": px / span,
                     "mean_batch": float(np.mean([x["batch_size"] for x in meas]))})
        print("serving", runs[-1], flush=True)
    st = srv.stats()
    srv.close()
    check = serving_oracle_check(dcfmm, scenes, tuned, reqs)
    for s in scenes:
        s.close()
    return {
        "workload": "16 resident scenes (10-5000 curves, log-uniform, 200 curves per unit "
                    "area; 16 panels x 16 GL nodes), requests 256-2048 px a side, zoom "
                    "10^U(0,6), Poisson arrivals",
        "options": "per scene, dc_autotune on its first request (FP32, target 5e-5)"
                   if args.serve_p <= 0 else f"fixed p {args.serve_p}, tile {args.serve_tile}",
        "precision": "f32", "oracle_check": check,
        "capacity_req_s": cap, "capacity_pixels_per_s": cap_px,
        "requests_per_run": n_req, "warmup_per_run": n_warm, "runs": runs,
        "server": {"n_streams": 4, "max_batch": 32, "hbm_budget_GiB": 32,
                   "batches": st["batches"], "max_in_flight": st["max_in_flight"],
                   "bytes_peak": st["bytes_peak"], "admission_waits": st["admission_waits"]},
        "setup_s": t_setup, "scenes": solve,
    }


def refine_bench(scene, cfg, solve_rep, torch):
    """Adaptive subdivision (Sec. 7) on the solved 200-curve scene: an 8x
    zoom around the panel with the largest Legendre tail, one round of
    Alg. 7 cutting the quarter of the panels in view with the largest tails
    (eps1 = 4 pixels of a 2048-px render of the zoom), re-solved globally
    and locally from the same warm start; the analogue of the paper's
    initial solve / global re-solve / local re-solve timing table."""
    tails = scene.panel_tails()
    pc, lo, hi = scene.panels()
    g = cfg["gl"]
    nodes = scene.nodes().reshape(-1, g, 2)
    top = int(np.argmax(tails))
    cx, cy = nodes[top].mean(axis=0)
    side = 1.0 / 8.0
    view = (float(cx), float(cy), side, side)
    inview = (np.abs(nodes[..., 0] - cx) <= side / 2).any(axis=1) & \
        (np.abs(nodes[..., 1] - cy) <= side / 2).any(axis=1)
    eps2 = float(np.quantile(tails[inview], 0.75))
    eps1 = 4.0 * side / 2048
    ev = dict(method="fmm", precision="f64", p=cfg["p"])
    out = {"viewport": view, "eps2": eps2, "eps1": eps1, "panels": int(len(pc)),
           "panels_in_view": int(inview.sum()),
           "initial_solve_s": solve_rep["seconds"], "initial_iters": max(solve_rep["iters"])}
    imgs = {}
    zoom = (view[0], view[1], side, side, 512, 512)
    for name, local in (("global", False), ("local", True)):
        torch.cuda.synchronize()
        ref_, rep_, res = scene.refine(eps2, eps1=eps1, viewport=view, local=local,
                                       tol=cfg["gmres_tol"], max_iter=1000, **ev)
        out[name] = {k: rep_[k] for k in ("seconds", "label_seconds", "solve_seconds",
                                          "iters", "panels_cut", "curves_resolved",
                                          "rel_residual", "converged")}
        imgs[name] = ref_.render(zoom, out_dtype=torch.float64, **ev).cpu().numpy()
        ref_.close()
        print("refine", name, out[name], flush=True)
    out["zoom_field_local_vs_global"] = float(np.abs(imgs["local"] - imgs["global"]).max())
    return out


def serving_oracle_check(dcfmm, scenes, tuned, reqs):
    """The first request of every serving scene, served with the scene's
    options but with synthetic densities (the oracle cannot solve the large
    scenes), against stored oracle values at 1,024 pixels per request."""
    path = os.path.join(ROOT, "tests", "golden", "c5_golden.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    srv = dcfmm.Server(precision="f32", n_streams=4, max_batch=16, hbm_budget=16 << 30)
    errs, rms = [], []
    try:
        for k, s in enumerate(scenes):
            s.set_densities(scenegen.synthetic_densities(s.N))
            srv.add_scene(s, **tuned[k])
        tickets = [srv.submit(scenes[int(k)], reqs[int(i)][1])
                   for i, k in zip(g["req"], g["scene"])]
        for j, t in enumerate(tickets):
            srv.wait(t)
            img = srv.fetch(t).cpu().numpy()
            a, b = int(g["first"][j]), int(g["first"][j + 1])
            d = img[g["rows"][a:b], g["cols"][a:b]] - g["vals"][a:b]
            errs.append(float(np.abs(d).max()))
            rms.append(float(np.sqrt(np.mean(d * d))))
    finally:
        srv.close()
    return {"requests": len(errs), "pixels_per_request": int(np.diff(g["first"]).max()),
            "max_err_vs_oracle": max(errs), "rms_err_vs_oracle": float(np.sqrt(np.mean(
                np.square(rms)))), "per_request_max": errs,
            "densities": "synthetic (scenegen.synthetic_densities); served with the timed "
                         "per-scene options"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--p64", type=int, default=0,
                    help="expansion order of the FP64 path (0: dc_autotune to 1e-10)")
    ap.add_argument("--p32", type=int, default=0,
                    help="fixed FP32 order (skips the autotuner; first tile size)")
    ap.add_argument("--tiles", default="8,16")
    ap.add_argument("--leaves", default="4,8,16")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-viewport batch")
    ap.add_argument("--batch-leaves", default="4,8")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving loop")
    ap.add_argument("--no-refine", action="store_true",
                    help="skip the adaptive subdivision timing")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 1M-node 4096^2 precision workload")
    ap.add_argument("--precision-leaf", type=int, default=8)
    ap.add_argument("--precision-p32", type=int, default=0,
                    help="FP32 order of the precision workload (0: dc_autotune)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB three times (reference "
                         "for hardware byte counters)")
    ap.add_argument("--serve-p", type=int, default=0,
                    help="fixed serving order (0: per-scene dc_autotune)")
    ap.add_argument("--serve-tile", type=int, default=16)
    # the host share of one GPU on the measurement boxes is 16 cores,
    # whatever os.cpu_count() reports there
    ap.add_argument("--workers", type=int,
                    default=min(16, len(os.sched_getaffinity(0)) or 1))
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the render shards by viewport; see the design notes)", file=sys.stderr)
        sys.exit(2)

    cfg = scenegen.FMM
    sc = scenegen.sized_scene(n_curves=cfg["n_curves"], n_stops=cfg["n_stops"],
                              seed=cfg["seed"])
    vp = cfg["viewport"]
    W, H = vp[4], vp[5]
    # The oracle runs first, before anything touches the GPU (its worker
    # processes are forked).
    cpu = None
    if not args.no_cpu:
        print("cpu baseline: oracle discretisation + sampled direct-sum render", flush=True)
        cpu = cpu_baseline(cfg, sc, args.workers)
        print(f"cpu baseline: {cpu['n']} px in {cpu['seconds']:.1f} s", flush=True)

    import torch
    from paper_2311_14312_amd import dcfmm
    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:
        n = args.calibrate_copy << 18   # float32 elements
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy calibration: 3 x {args.calibrate_copy} MiB device-to-device", flush=True)
        del src, dst

    def make_scene(leaf):
        t0 = time.time()
        sc_ = dcfmm.Scene(sc["ctrl"], sc["left"], sc["right"], panels=cfg["panels"],
                          gl=cfg["gl"], segs=cfg["segs"], leaf_max=leaf)
        t_create = time.time() - t0
        rep_ = sc_.solve(tol=cfg["gmres_tol"], max_iter=1000, method="fmm", p=cfg["p"])
        print(f"leaf {leaf}: scene {sc_.info()} create {t_create:.2f} s, solve {rep_}",
              flush=True)
        return sc_, rep_, t_create

    def timed(scene, ev, steps, warmup, dtype):
        out = torch.empty((H, W, 3), device="cuda", dtype=dtype)
        for _ in range(warmup):
            scene.render(vp, out=out, **ev)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(steps):
            scene.render(vp, out=out, **ev)
        stop.record()
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps, out

    def sample_err(img):
        if cpu is None or cpu["vals"] is None:
            return None
        return float(np.abs(img[cpu["rows"], cpu["cols"]] - cpu["vals"]).max())

    # Autotune: the leaf capacity (a scene property) by time; for each, the
    # library's dc_autotune picks the expansion order and tile size against
    # its own FP64 direct sum at sampled pixels (target 5e-5, half the bar).
    # The oracle pixels that give max_err_vs_oracle are not seen by the tuner.
    leaves = [int(v) for v in args.leaves.split(",")]
    tiles = tuple(int(v) for v in args.tiles.split(","))
    tune = []
    best = None
    scenes = {}
    for leaf in leaves:
        scn, rep, t_create = make_scene(leaf)
        scenes[leaf] = (scn, rep, t_create)
        if args.p32 > 0:
            # a fixed order and the first tile size (profiling runs: only the
            # timed configuration's kernels are launched)
            ev = dict(method="fmm", precision="f32", p=args.p32, tile_px=tiles[0])
            ms, _ = timed(scn, ev, 5, 2, torch.float32)
            tune.append({"leaf": leaf, "tile": tiles[0], "p": args.p32, "ms": ms,
                         "tuner_err": None, "fixed": True})
        else:
            tr = scn.autotune([vp], target_err=5e-5, precision="f32", p_min=8, p_max=24,
                              p_step=2, tiles=tiles, samples=2048, timing_reps=5)
            ev = tr["eval"]
            ms, _ = timed(scn, ev, 5, 2, torch.float32)
            tune.append({"leaf": leaf, "tile": ev["tile_px"], "p": ev["p"], "ms": ms,
                         "tuner_err": tr["err"], "tuner_samples": tr["n_samples"],
                         "per_tile": {"tiles": tr["tiles"], "p": tr["tile_p"],
                                      "ms": tr["tile_ms"]}})
        print("autotune", tune[-1], flush=True)
        if best is None or ms < best["ms"]:
            best = dict(tune[-1])
        if best["leaf"] != leaf:
            scn.close()
            del scenes[leaf]
    scene, rep, t_create = scenes[best["leaf"]]
    p32, tile, leaf = best["p"], best["tile"], best["leaf"]
    # the FP64 comparator's order: dc_autotune against the same direct sum
    # with the FP64 bar (1e-10) as target
    if args.p64 > 0:
        tr64 = {"err": None}
        p64 = args.p64
    else:
        tr64 = scene.autotune([vp], target_err=1e-10, precision="f64", p_min=20, p_max=40,
                              p_step=4, tiles=(tile,), samples=1024, timing_reps=1)
        p64 = tr64["eval"]["p"]
    print(f"FP64 order {p64} (tuner error {tr64['err']})", flush=True)

    ev32 = dict(method="fmm", precision="f32", p=p32, tile_px=tile)
    ev64 = dict(method="fmm", precision="f64", p=p64, tile_px=tile)
    ms32, img32 = timed(scene, ev32, args.steps, args.warmup, torch.float32)
    img32 = img32.cpu().numpy()
    ms64, img64 = timed(scene, ev64, max(1, args.steps // 2), 1, torch.float64)
    img64 = img64.cpu().numpy()
    print(f"FP32 {ms32:.3f} ms/step, FP64 {ms64:.3f} ms/step", flush=True)

    # The same FP32 render replayed from a captured HIP graph (same kernels,
    # same work; no per-call planning or launch work on the host).
    graph = scene.render_graph([vp], **ev32)
    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record()
    for _ in range(args.steps):
        graph.launch()
    g1.record()
    torch.cuda.synchronize()
    ms_graph = g0.elapsed_time(g1) / args.steps
    graph_err = sample_err(graph.outs[0].cpu().numpy())
    graph.close()
    print(f"FP32 graph replay {ms_graph:.3f} ms/step", flush=True)

    # Dominant kernel: per-phase HIP-event timing on the render stream.
    scene.set_timing(True)
    for _ in range(args.steps):
        scene.render(vp, **ev32)
    tm = scene.get_timing()
    scene.set_timing(False)
    counts = scene.render_counts(vp, **ev32)
    leaf_ms = tm["leaf_ms"] / max(1, tm["calls"])
    fl = leaf_flops(counts, p32)
    achieved = fl / (leaf_ms * 1e-3)
    scene.set_timing(True)
    for _ in range(max(1, args.steps // 2)):
        scene.render(vp, **ev64)
    tm64 = scene.get_timing()
    scene.set_timing(False)
    counts64 = scene.render_counts(vp, **ev64)
    leaf64_ms = tm64["leaf_ms"] / max(1, tm64["calls"])
    achieved64 = leaf_flops(counts64, p64) / (leaf64_ms * 1e-3)

    px = W * H
    err32, err64 = sample_err(img32), sample_err(img64)
    kernel_name = ("k_tile<float, 64, 1, 1, false> + k_tile_big<float, false, 1>" if tile <= 8
                   else "k_tile<float, 128, 2, 1, false>")
    line = {
        "metric": METRIC,
        "value": px / (ms32 * 1e-3),
        "unit": "RGB pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "200 random cubic Beziers (lengths log-uniform 0.01-0.5), "
                               "16 panels x 16 GL nodes (51,200 nodes), 80 segments/panel, "
                               "3 colour stops/side; 2048x2048 render of [0,1]^2",
                   "p_fp32": p32, "p_fp64": p64, "tile_px": tile,
                   "leaf_max": leaf, "gmres_tol": cfg["gmres_tol"], "autotune": tune},
        "max_err_vs_oracle": err32,
        "err_sample": (f"{cpu['n']} pixels (128x128 stride-16 grid + 4096 near-chord)"
                       if cpu else None),
        "fp64_fmm": {"value": px / (ms64 * 1e-3), "unit": "RGB pixels/s", "ms_per_step": ms64,
                     "max_err_vs_oracle": err64, "p": p64,
                     "tuner_err_vs_direct_sum": tr64["err"],
                     "roofline": {"bound": "alu", "achieved": achieved64 / 1e12,
                                  "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                                  "frac": achieved64 / PEAK_FP64}},
        "speedup_fp32_vs_fp64": ms64 / ms32,
        "graph_replay": {"value": px / (ms_graph * 1e-3), "unit": "RGB pixels/s",
                         "ms_per_step": ms_graph, "max_err_vs_oracle": graph_err},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": measured_traffic(kernel_name, f"leaf {leaf}, tile {tile}, p {p32}"),
                     "traffic_unit": "bytes/launch",
                     "kernel": kernel_name,
                     "kernel_ms": leaf_ms,
                     "flop_eq_per_launch": fl,
                     "valu_issue": valu_issue(kernel_name, f"leaf {leaf}, tile {tile}, p {p32}",
                                              leaf_ms)},
        "phases_ms": {k: v / max(1, tm["calls"]) for k, v in tm.items() if k.endswith("_ms")},
        "work": counts,
        "solve": {"seconds": rep["seconds"], "iters": rep["iters"], "precond": "block",
                  "true_rel_residual": rep["true_rel_residual"], "p": cfg["p"],
                  "scene_create_s": t_create},
        "cpu_baseline": None if cpu is None else {
            "value": cpu["value"], "unit": "RGB pixels/s", "cores": args.workers,
            "kind": "oracle",
            "sample": f"{cpu['n']} sampled pixels of the 2048x2048 viewport x {cpu['S']} "
                      f"segments, FP64 NumPy direct sum ({cpu['seconds']:.1f} s); value is "
                      f"the rate on that sample",
            "cpu_model": cpu_model(), "host_cpu_count": os.cpu_count(),
            "threads": f"{args.workers} worker processes x 1 BLAS thread",
            "pairs_per_s": cpu["value"] * cpu["S"],
            "full_frame_s_extrapolated": W * H / cpu["value"]},
    }
    if not args.no_refine:
        line["refine"] = refine_bench(scene, cfg, rep, torch)
    for scn, _, _ in scenes.values():
        scn.close()
    if not args.no_batch:
        line["batch"] = batch_bench(args, torch, dcfmm)
    if not args.no_precision:
        line["precision"] = precision_bench(args, torch, dcfmm)
    if not args.no_serving:
        line["serving"] = serving_bench(args, torch, dcfmm)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
