"""Python binding of libdcfmm.so (argument marshalling only).

Every computation runs in the HIP library; PyTorch supplies device memory
and the current stream.  Importing this module fails loudly if the library
has not been built (``python -m paper_2311_14312_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcfmm.so")

DC_OK, DC_ERR_INVALID, DC_ERR_OOM, DC_ERR_NOT_CONVERGED, DC_ERR_HIP = 0, -1, -2, -3, -4
DC_ERR_TIMEOUT = -5
PREC_F64, PREC_F32 = 0, 1
METHOD_FMM, METHOD_DIRECT = 0, 1
OUT_F32, OUT_F64 = 0, 1
P_MAX = 63


class SceneOpts(C.Structure):
    _fields_ = [("panels_per_curve", C.c_int), ("gl_per_panel", C.c_int),
                ("segs_per_panel", C.c_int), ("leaf_max", C.c_int),
                ("max_depth", C.c_int), ("domain", C.c_double * 4)]


class EvalOpts(C.Structure):
    _fields_ = [("method", C.c_int), ("precision", C.c_int), ("p", C.c_int),
                ("tile_px", C.c_int), ("near_fp64", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("matvec", EvalOpts),
                ("precond", C.c_int)]


class Viewport(C.Structure):
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("width", C.c_double),
                ("height", C.c_double), ("W", C.c_int), ("H", C.c_int)]


class SolveReport(C.Structure):
    _fields_ = [("iters", C.c_int * 3), ("rel_residual", C.c_double * 3),
                ("true_rel_residual", C.c_double * 3), ("seconds", C.c_double),
                ("converged", C.c_int)]


class SceneInfo(C.Structure):
    _fields_ = [("n_curves", C.c_int), ("N", C.c_int), ("S", C.c_int),
                ("n_pieces", C.c_int), ("n_cells", C.c_int), ("n_leaves", C.c_int),
                ("depth", C.c_int), ("root", C.c_double * 3), ("solved", C.c_int),
                ("table_pairs", C.c_longlong), ("table_bytes", C.c_longlong)]


class WorkCounts(C.Structure):
    _fields_ = [("p2p_pairs", C.c_ulonglong), ("p2p_fp64_pairs", C.c_ulonglong),
                ("m2p_pairs", C.c_ulonglong), ("l2p_targets", C.c_ulonglong),
                ("m2l_pairs", C.c_ulonglong), ("p2l_pairs", C.c_ulonglong),
                ("p2l_fp64_pairs", C.c_ulonglong), ("l2l_boxes", C.c_ulonglong), ("leaf_boxes", C.c_ulonglong),
                ("pieces", C.c_ulonglong), ("source_cells", C.c_ulonglong),
                ("levels", C.c_int), ("p", C.c_int)]


class RenderGraph:
    """Launches of one batched render captured into a HIP graph
    (dc_render_graph_*): launch() renders the same viewports into the same
    output tensors (self.outs) again."""

    def __init__(self, scene, viewports, outs=None, out_dtype=None, **ev):
        import torch
        n = len(viewports)
        vps = (Viewport * n)()
        for i, (cx, cy, w, h, W, H) in enumerate(viewports):
            vps[i] = Viewport(float(cx), float(cy), float(w), float(h), int(W), int(H))
        if outs is None:
            outs = [torch.empty((int(v[5]), int(v[4]), 3), device="cuda",
                                dtype=out_dtype or torch.float32) for v in viewports]
        assert len(outs) == n and len({o.dtype for o in outs}) == 1
        for o, v in zip(outs, viewports):
            assert o.is_cuda and o.is_contiguous() and tuple(o.shape) == (v[5], v[4], 3)
        code = {torch.float32: OUT_F32, torch.float64: OUT_F64}[outs[0].dtype]
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        o = eval_opts(**ev)
        h = C.c_void_p()
        _check(_lib.dc_render_graph_create(scene._h, vps, n, C.byref(o), code, ptrs, C.byref(h)))
        self._h = h
        self.scene = scene
        self.outs = outs

    def launch(self):
        _check(_lib.dc_render_graph_launch(self._h, _stream()))
        return self.outs

    def close(self):
        if getattr(self, "_h", None):
            _lib.dc_render_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class TuneOpts(C.Structure):
    _fields_ = [("target_err", C.c_double), ("precision", C.c_int), ("p_min", C.c_int),
                ("p_max", C.c_int), ("p_step", C.c_int), ("tiles", C.c_int * 4),
                ("n_tiles", C.c_int), ("samples", C.c_int), ("near_fp64", C.c_double),
                ("timing_reps", C.c_int)]


class TuneReport(C.Structure):
    _fields_ = [("chosen", EvalOpts), ("err", C.c_double), ("ms", C.c_double),
                ("n_samples", C.c_int), ("met", C.c_int), ("tile_p", C.c_int * 4),
                ("tile_err", C.c_double * 4), ("tile_ms", C.c_double * 4)]


class AaReport(C.Structure):
    _fields_ = [("aa_pixels", C.c_longlong), ("blocks", C.c_int), ("samples", C.c_longlong)]


class RefineOpts(C.Structure):
    _fields_ = [("eps2", C.c_double), ("eps1", C.c_double), ("viewport", C.c_double * 4),
                ("ratio", C.c_double), ("max_rounds", C.c_int), ("local", C.c_int),
                ("solve", SolveOpts)]


class RefineReport(C.Structure):
    _fields_ = [("rounds", C.c_int), ("panels_cut", C.c_int), ("n_panels", C.c_int),
                ("curves_resolved", C.c_int), ("iters", C.c_int), ("converged", C.c_int),
                ("rel_residual", C.c_double), ("seconds", C.c_double),
                ("label_seconds", C.c_double), ("solve_seconds", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("eval", EvalOpts), ("out_dtype", C.c_int), ("n_streams", C.c_int),
                ("max_batch", C.c_int), ("max_batch_pixels", C.c_longlong),
                ("hbm_budget", C.c_longlong)]


class RequestInfo(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("batch", C.c_longlong), ("batch_size", C.c_int), ("status", C.c_int),
                ("bytes", C.c_longlong)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_longlong), ("completed", C.c_longlong),
                ("fetched", C.c_longlong), ("batches", C.c_longlong),
                ("max_in_flight", C.c_longlong), ("bytes_in_use", C.c_longlong),
                ("bytes_peak", C.c_longlong), ("admission_waits", C.c_longlong)]


class DcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dcfmm error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2311_14312_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, I, D, V = C.c_void_p, C.c_int, C.c_double, C.c_void_p
    dp = C.POINTER(C.c_double)
    sig = {
        "dc_default_scene_opts": (None, [C.POINTER(SceneOpts)]),
        "dc_default_eval_opts": (None, [C.POINTER(EvalOpts)]),
        "dc_scene_create": (I, [dp, I, dp, dp, I, C.POINTER(SceneOpts), C.POINTER(P)]),
        "dc_scene_create_panels": (I, [dp, I, dp, dp, I, C.POINTER(C.c_int), dp, dp, I,
                                       C.POINTER(SceneOpts), C.POINTER(P)]),
        "dc_scene_panels": (I, [P, C.POINTER(C.c_int), C.POINTER(C.c_int), dp, dp]),
        "dc_panel_tails": (I, [P, dp, V]),
        "dc_default_refine_opts": (None, [C.POINTER(RefineOpts)]),
        "dc_refine": (I, [P, C.POINTER(RefineOpts), C.POINTER(P), C.POINTER(RefineReport),
                          C.POINTER(C.c_ubyte), V]),
        "dc_set_solve_tables": (I, [P, I]),
        "dc_scene_destroy": (None, [P]),
        "dc_scene_get_info": (I, [P, C.POINTER(SceneInfo)]),
        "dc_get_nodes": (I, [P, dp]),
        "dc_set_boundary": (I, [P, dp, dp]),
        "dc_solve_densities": (I, [P, C.POINTER(SolveOpts), C.POINTER(SolveReport), V]),
        "dc_get_densities": (I, [P, dp]),
        "dc_solve_mixed": (I, [P, C.POINTER(C.c_int), dp, C.POINTER(SolveOpts),
                               C.POINTER(SolveReport), V]),
        "dc_set_densities": (I, [P, dp]),
        "dc_apply_operator": (I, [P, V, V, I, C.POINTER(EvalOpts), V]),
        "dc_render": (I, [P, C.POINTER(Viewport), C.POINTER(EvalOpts), I, V, V]),
        "dc_render_noalloc": (I, [P, C.POINTER(Viewport), C.POINTER(EvalOpts), I, V, V]),
        "dc_render_aa": (I, [P, C.POINTER(Viewport), C.POINTER(EvalOpts), I, I, V,
                             C.POINTER(AaReport), V]),
        "dc_render_batch": (I, [P, C.POINTER(Viewport), I, C.POINTER(EvalOpts), I,
                                C.POINTER(V), V]),
        "dc_eval_points": (I, [P, V, I, C.POINTER(EvalOpts), I, V, V]),
        "dc_default_tune_opts": (None, [C.POINTER(TuneOpts)]),
        "dc_autotune": (I, [P, C.POINTER(Viewport), I, C.POINTER(TuneOpts),
                            C.POINTER(TuneReport), V]),
        "dc_render_counts": (I, [P, C.POINTER(Viewport), C.POINTER(EvalOpts),
                                 C.POINTER(WorkCounts), V]),
        "dc_render_graph_create": (I, [P, C.POINTER(Viewport), I, C.POINTER(EvalOpts), I,
                                       C.POINTER(V), C.POINTER(P)]),
        "dc_render_graph_launch": (I, [P, V]),
        "dc_render_graph_destroy": (None, [P]),
        "dc_set_timing": (I, [P, I]),
        "dc_get_timing": (I, [P, dp]),
        "dc_default_server_opts": (None, [C.POINTER(ServerOpts)]),
        "dc_server_create": (I, [C.POINTER(ServerOpts), C.POINTER(P)]),
        "dc_server_add_scene": (I, [P, P]),
        "dc_server_add_scene_opts": (I, [P, P, C.POINTER(EvalOpts)]),
        "dc_server_submit": (I, [P, P, C.POINTER(Viewport), C.POINTER(C.c_longlong)]),
        "dc_server_wait": (I, [P, C.c_longlong, C.c_double, C.POINTER(RequestInfo)]),
        "dc_server_fetch": (I, [P, C.c_longlong, V, I]),
        "dc_server_get_stats": (I, [P, C.POINTER(ServerStats)]),
        "dc_server_destroy": (None, [P]),
        "dc_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _check(rc, allow=()):
    if rc != DC_OK and rc not in allow:
        raise DcError(rc, _lib.dc_last_error().decode())
    return rc


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def eval_opts(method="fmm", precision="f64", p=20, tile_px=8, near_fp64=1e-3):
    e = EvalOpts()
    _lib.dc_default_eval_opts(C.byref(e))
    e.method = {"fmm": METHOD_FMM, "direct": METHOD_DIRECT}[method]
    e.precision = {"f64": PREC_F64, "f32": PREC_F32}[precision]
    e.p = int(p)
    e.tile_px = int(tile_px)
    e.near_fp64 = float(near_fp64)
    return e


class Scene:
    """A resident scene: geometry, quadtree and densities on the device."""

    def __init__(self, ctrl, left, right, panels=16, gl=16, segs=80, leaf_max=64,
                 max_depth=40, domain=None, panel_list=None):
        """panels equal panels per curve, or panel_list = (curve, lo, hi):
        panels of any lengths (dc_scene_create_panels)."""
        o = SceneOpts()
        _lib.dc_default_scene_opts(C.byref(o))
        o.panels_per_curve, o.gl_per_panel, o.segs_per_panel = panels, gl, segs
        o.leaf_max, o.max_depth = leaf_max, max_depth
        if domain is not None:
            for k in range(4):
                o.domain[k] = float(domain[k])
        self._ctrl = _f64(ctrl)
        left, right = _f64(left), _f64(right)
        n = self._ctrl.shape[0]
        if self._ctrl.shape != (n, 4, 2) or left.shape[0] != n or left.shape != right.shape \
                or left.ndim != 3 or left.shape[2] != 3:
            raise ValueError("expected ctrl [n,4,2] and left/right [n,stops,3]")
        h = C.c_void_p()
        if panel_list is None:
            _check(_lib.dc_scene_create(_ptr(self._ctrl), n, _ptr(left), _ptr(right),
                                        left.shape[1], C.byref(o), C.byref(h)))
        else:
            pc = np.ascontiguousarray(panel_list[0], dtype=np.int32)
            lo, hi = _f64(panel_list[1]), _f64(panel_list[2])
            if lo.shape != pc.shape or hi.shape != pc.shape or pc.ndim != 1:
                raise ValueError("panel_list: three arrays [n_panels]")
            _check(_lib.dc_scene_create_panels(
                _ptr(self._ctrl), n, _ptr(left), _ptr(right), left.shape[1],
                pc.ctypes.data_as(C.POINTER(C.c_int)), _ptr(lo), _ptr(hi), len(pc),
                C.byref(o), C.byref(h)))
        self._h = h

    @classmethod
    def _wrap(cls, handle):
        sc = cls.__new__(cls)
        sc._h = handle
        return sc

    def panels(self):
        """The panel list (curve [n], lo [n], hi [n]) of dc_scene_panels."""
        n = C.c_int()
        _check(_lib.dc_scene_panels(self._h, C.byref(n), None, None, None))
        pc = np.empty(n.value, np.int32)
        lo, hi = np.empty(n.value), np.empty(n.value)
        _check(_lib.dc_scene_panels(self._h, C.byref(n), pc.ctypes.data_as(C.POINTER(C.c_int)),
                                    _ptr(lo), _ptr(hi)))
        return pc, lo, hi

    def set_solve_tables(self, mode="auto"):
        """dc_set_solve_tables: "auto" (default), "always" or "off"."""
        _check(_lib.dc_set_solve_tables(self._h, {"off": 0, "auto": 1, "always": 2}[mode]))

    def panel_tails(self):
        """dc_panel_tails: the highest Legendre coefficient of every panel."""
        n = len(self.panels()[0])
        out = np.empty(n)
        _check(_lib.dc_panel_tails(self._h, _ptr(out), _stream()))
        return out

    def refine(self, eps2, eps1=0.0, viewport=None, ratio=0.9, max_rounds=1, local=True,
               tol=1e-10, max_iter=500, precond="block", raise_on_fail=False, **ev):
        """dc_refine: returns (refined Scene or None, report dict, re-solved
        curve flags of the last round [n_curves])."""
        o = RefineOpts()
        _lib.dc_default_refine_opts(C.byref(o))
        o.eps2, o.eps1, o.ratio = float(eps2), float(eps1), float(ratio)
        if viewport is not None:
            for k in range(4):
                o.viewport[k] = float(viewport[k])
        o.max_rounds, o.local = int(max_rounds), 1 if local else 0
        o.solve.tol, o.solve.max_iter, o.solve.matvec = tol, max_iter, eval_opts(**ev)
        o.solve.precond = {"none": 0, "block": 1}[precond]
        rep = RefineReport()
        res = np.zeros(self.info()["n_curves"], np.uint8)
        h = C.c_void_p()
        allow = () if raise_on_fail else (DC_ERR_NOT_CONVERGED,)
        rc = _check(_lib.dc_refine(self._h, C.byref(o), C.byref(h), C.byref(rep),
                                   res.ctypes.data_as(C.POINTER(C.c_ubyte)), _stream()), allow)
        out = Scene._wrap(h) if h.value else None
        d = {k: getattr(rep, k) for k, _ in RefineReport._fields_}
        d["rc"] = rc
        return out, d, res.astype(bool)

    @classmethod
    def from_dict(cls, sc, **kw):
        args = dict(panels=sc.get("panels", 16), gl=sc.get("gl", 16),
                    segs=sc.get("segs", 80), leaf_max=sc.get("leaf_max", 64))
        args.update(kw)
        return cls(sc["ctrl"], sc["left"], sc["right"], **args)

    def close(self):
        if getattr(self, "_h", None):
            _lib.dc_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = SceneInfo()
        _check(_lib.dc_scene_get_info(self._h, C.byref(i)))
        return {k: (list(getattr(i, k)) if k == "root" else getattr(i, k))
                for k, _ in SceneInfo._fields_}

    @property
    def N(self):
        return self.info()["N"]

    def nodes(self):
        out = np.empty((self.N, 2))
        _check(_lib.dc_get_nodes(self._h, _ptr(out)))
        return out

    def set_boundary(self, u_plus, u_minus):
        up, um = _f64(u_plus), _f64(u_minus)
        if up.shape != (3, self.N) or um.shape != (3, self.N):
            raise ValueError("boundary values must be [3, N]")
        _check(_lib.dc_set_boundary(self._h, _ptr(up), _ptr(um)))

    def solve(self, tol=1e-10, max_iter=1000, raise_on_fail=False, precond="block", **ev):
        o = SolveOpts()
        o.tol, o.max_iter, o.matvec = tol, max_iter, eval_opts(**ev)
        o.precond = {"none": 0, "block": 1}[precond]
        rep = SolveReport()
        allow = () if raise_on_fail else (DC_ERR_NOT_CONVERGED,)
        rc = _check(_lib.dc_solve_densities(self._h, C.byref(o), C.byref(rep), _stream()),
                    allow)
        return {"iters": list(rep.iters), "rel_residual": list(rep.rel_residual),
                "true_rel_residual": list(rep.true_rel_residual),
                "seconds": rep.seconds, "converged": bool(rep.converged), "rc": rc}

    def solve_mixed(self, neumann, values, tol=1e-10, max_iter=1000, raise_on_fail=False,
                    **ev):
        """dc_solve_mixed: neumann [N] flags, values [3, N] (u* or psi*)."""
        fl = np.ascontiguousarray(neumann, dtype=np.int32)
        vals = _f64(values)
        if fl.shape != (self.N,) or vals.shape != (3, self.N):
            raise ValueError("expected neumann [N] and values [3, N]")
        o = SolveOpts()
        o.tol, o.max_iter, o.matvec = tol, max_iter, eval_opts(**ev)
        o.precond = 0
        rep = SolveReport()
        allow = () if raise_on_fail else (DC_ERR_NOT_CONVERGED,)
        rc = _check(_lib.dc_solve_mixed(self._h, fl.ctypes.data_as(C.POINTER(C.c_int)),
                                        _ptr(vals), C.byref(o), C.byref(rep), _stream()),
                    allow)
        return {"iters": list(rep.iters), "rel_residual": list(rep.rel_residual),
                "true_rel_residual": list(rep.true_rel_residual),
                "seconds": rep.seconds, "converged": bool(rep.converged), "rc": rc}

    def densities(self):
        out = np.empty((3, self.N))
        _check(_lib.dc_get_densities(self._h, _ptr(out)))
        return out

    def set_densities(self, sigma):
        s = _f64(sigma)
        if s.shape != (3, self.N):
            raise ValueError("densities must be [3, N]")
        _check(_lib.dc_set_densities(self._h, _ptr(s)))

    def apply_operator(self, x, y=None, c_mu=0, **ev):
        """y = G_H x + c_mu F_H mu at the nodes; x, y torch cuda float64 [3, N]."""
        import torch
        assert x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()
        assert tuple(x.shape) == (3, self.N)
        if y is None:
            y = torch.empty_like(x)
        o = eval_opts(**ev)
        _check(_lib.dc_apply_operator(self._h, C.c_void_p(x.data_ptr()),
                                      C.c_void_p(y.data_ptr()), int(c_mu), C.byref(o),
                                      _stream()))
        return y

    def render(self, viewport, out=None, out_dtype=None, **ev):
        """Image [H, W, 3] of viewport (cx, cy, width, height, W, H)."""
        import torch
        cx, cy, w, h, W, H = viewport
        vp = Viewport(float(cx), float(cy), float(w), float(h), int(W), int(H))
        if out is None:
            out = torch.empty((int(H), int(W), 3), device="cuda",
                              dtype=out_dtype or torch.float32)
        assert out.is_cuda and out.is_contiguous() and tuple(out.shape) == (H, W, 3)
        code = {torch.float32: OUT_F32, torch.float64: OUT_F64}[out.dtype]
        o = eval_opts(**ev)
        _check(_lib.dc_render(self._h, C.byref(vp), C.byref(o), code,
                              C.c_void_p(out.data_ptr()), _stream()))
        return out

    def render_noalloc(self, viewport, out, **ev):
        """dc_render_noalloc: render into the caller's tensor `out` with the
        library's fixed device scratch (nothing is allocated)."""
        import torch
        cx, cy, w, h, W, H = viewport
        vp = Viewport(float(cx), float(cy), float(w), float(h), int(W), int(H))
        assert out.is_cuda and out.is_contiguous() and tuple(out.shape) == (H, W, 3)
        code = {torch.float32: OUT_F32, torch.float64: OUT_F64}[out.dtype]
        o = eval_opts(**ev)
        _check(_lib.dc_render_noalloc(self._h, C.byref(vp), C.byref(o), code,
                                      C.c_void_p(out.data_ptr()), _stream()))
        return out

    def render_aa(self, viewport, aa=4, out=None, out_dtype=None, **ev):
        """dc_render_aa: anti-aliased image [H, W, 3] and its report."""
        import torch
        cx, cy, w, h, W, H = viewport
        vp = Viewport(float(cx), float(cy), float(w), float(h), int(W), int(H))
        if out is None:
            out = torch.empty((int(H), int(W), 3), device="cuda",
                              dtype=out_dtype or torch.float32)
        assert out.is_cuda and out.is_contiguous() and tuple(out.shape) == (H, W, 3)
        code = {torch.float32: OUT_F32, torch.float64: OUT_F64}[out.dtype]
        o = eval_opts(**ev)
        r = AaReport()
        _check(_lib.dc_render_aa(self._h, C.byref(vp), C.byref(o), int(aa), code,
                                 C.c_void_p(out.data_ptr()), C.byref(r), _stream()))
        return out, {k: getattr(r, k) for k, _ in AaReport._fields_}

    def render_batch(self, viewports, outs=None, out_dtype=None, **ev):
        """Images of several viewports of this scene in one batched render."""
        import torch
        n = len(viewports)
        vps = (Viewport * n)()
        for i, (cx, cy, w, h, W, H) in enumerate(viewports):
            vps[i] = Viewport(float(cx), float(cy), float(w), float(h), int(W), int(H))
        if outs is None:
            outs = [torch.empty((int(v[5]), int(v[4]), 3), device="cuda",
                                dtype=out_dtype or torch.float32) for v in viewports]
        assert len(outs) == n and len({o.dtype for o in outs}) == 1
        for o, v in zip(outs, viewports):
            assert o.is_cuda and o.is_contiguous() and tuple(o.shape) == (v[5], v[4], 3)
        code = {torch.float32: OUT_F32, torch.float64: OUT_F64}[outs[0].dtype]
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        o = eval_opts(**ev)
        _check(_lib.dc_render_batch(self._h, vps, n, C.byref(o), code, ptrs, _stream()))
        return outs

    def render_graph(self, viewports, outs=None, out_dtype=None, **ev):
        """A RenderGraph that replays render_batch(viewports, outs) (see
        dc_render_graph_create)."""
        return RenderGraph(self, viewports, outs, out_dtype, **ev)

    def eval_points(self, xy, out_dtype=None, **ev):
        """Representation at points xy (torch cuda float64 [n, 2]) -> [n, 3]."""
        import torch
        assert xy.is_cuda and xy.dtype == torch.float64 and xy.is_contiguous()
        n = xy.shape[0]
        out = torch.empty((n, 3), device="cuda", dtype=out_dtype or torch.float64)
        code = {torch.float32: OUT_F32, torch.float64: OUT_F64}[out.dtype]
        o = eval_opts(**ev)
        _check(_lib.dc_eval_points(self._h, C.c_void_p(xy.data_ptr()), n, C.byref(o), code,
                                   C.c_void_p(out.data_ptr()), _stream()))
        return out


    def autotune(self, viewports, target_err=None, precision="f32", p_min=None, p_max=None,
                 p_step=None, tiles=None, samples=None, near_fp64=None, timing_reps=None):
        """dc_autotune over the viewports; returns a dict with `eval` (the
        chosen options as keyword arguments of render) and the report."""
        n = len(viewports)
        vps = (Viewport * n)()
        for i, (cx, cy, w, h, W, H) in enumerate(viewports):
            vps[i] = Viewport(float(cx), float(cy), float(w), float(h), int(W), int(H))
        t = TuneOpts()
        _lib.dc_default_tune_opts(C.byref(t))
        t.precision = {"f64": PREC_F64, "f32": PREC_F32}[precision]
        for name, val in (("target_err", target_err), ("p_min", p_min), ("p_max", p_max),
                          ("p_step", p_step), ("samples", samples), ("near_fp64", near_fp64),
                          ("timing_reps", timing_reps)):
            if val is not None:
                setattr(t, name, val)
        if tiles is not None:
            t.n_tiles = len(tiles)
            for k, v in enumerate(tiles):
                t.tiles[k] = int(v)
        r = TuneReport()
        _check(_lib.dc_autotune(self._h, vps, n, C.byref(t), C.byref(r), _stream()))
        c = r.chosen
        ev = dict(method="fmm", precision={PREC_F64: "f64", PREC_F32: "f32"}[c.precision],
                  p=c.p, tile_px=c.tile_px, near_fp64=c.near_fp64)
        k = t.n_tiles
        return {"eval": ev, "err": r.err, "ms": r.ms, "n_samples": r.n_samples,
                "met": bool(r.met), "tiles": [t.tiles[i] for i in range(k)],
                "tile_p": list(r.tile_p)[:k], "tile_err": list(r.tile_err)[:k],
                "tile_ms": list(r.tile_ms)[:k]}

    def render_counts(self, viewport, **ev):
        """Device-counted work of one FMM render of viewport (synchronous)."""
        cx, cy, w, h, W, H = viewport
        vp = Viewport(float(cx), float(cy), float(w), float(h), int(W), int(H))
        o = eval_opts(**ev)
        wc = WorkCounts()
        _check(_lib.dc_render_counts(self._h, C.byref(vp), C.byref(o), C.byref(wc),
                                     _stream()))
        return {k: getattr(wc, k) for k, _ in WorkCounts._fields_}

    def set_timing(self, enable=True):
        _check(_lib.dc_set_timing(self._h, int(bool(enable))))

    def get_timing(self):
        """Summed per-phase render times (ms) since the last call, and calls."""
        ms = np.zeros(5)
        _check(_lib.dc_get_timing(self._h, _ptr(ms)))
        return {"upward_ms": ms[0], "downward_ms": ms[1], "leaf_ms": ms[2],
                "total_ms": ms[3], "calls": int(ms[4])}


def exported_symbols():
    """Names of the dc_* functions the loaded library exports."""
    return sorted(n for n in dir(_lib) if n.startswith("dc_"))


class Server:
    """Continuous-batching render server over resident scenes (the C-ABI
    dc_server_*: a native worker thread batches, admits by device footprint
    and launches on several streams)."""

    def __init__(self, precision="f32", p=12, tile_px=8, near_fp64=1e-3, out_dtype=None,
                 n_streams=4, max_batch=64, max_batch_pixels=1 << 26, hbm_budget=8 << 30):
        import torch
        o = ServerOpts()
        _lib.dc_default_server_opts(C.byref(o))
        o.eval = eval_opts(method="fmm", precision=precision, p=p, tile_px=tile_px,
                           near_fp64=near_fp64)
        self.dtype = out_dtype or torch.float32
        o.out_dtype = {torch.float32: OUT_F32, torch.float64: OUT_F64}[self.dtype]
        o.n_streams, o.max_batch = int(n_streams), int(max_batch)
        o.max_batch_pixels, o.hbm_budget = int(max_batch_pixels), int(hbm_budget)
        h = C.c_void_p()
        _check(_lib.dc_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._shapes = {}
        self._scenes = []

    def add_scene(self, scene, **ev):
        """Register a scene; keyword render options (those of render, e.g.
        the `eval` dict of Scene.autotune) give it options of its own."""
        if ev:
            o = eval_opts(**ev)
            _check(_lib.dc_server_add_scene_opts(self._h, scene._h, C.byref(o)))
        else:
            _check(_lib.dc_server_add_scene(self._h, scene._h))
        self._scenes.append(scene)

    def submit(self, scene, viewport):
        cx, cy, w, h, W, H = viewport
        vp = Viewport(float(cx), float(cy), float(w), float(h), int(W), int(H))
        t = C.c_longlong()
        _check(_lib.dc_server_submit(self._h, scene._h, C.byref(vp), C.byref(t)))
        self._shapes[t.value] = (int(H), int(W), 3)
        return t.value

    def wait(self, ticket, timeout=-1.0):
        """Request info dict once done; None on timeout."""
        info = RequestInfo()
        rc = _check(_lib.dc_server_wait(self._h, int(ticket), float(timeout), C.byref(info)),
                    allow=(DC_ERR_TIMEOUT,))
        if rc == DC_ERR_TIMEOUT:
            return None
        return {k: getattr(info, k) for k, _ in RequestInfo._fields_}

    def fetch(self, ticket, out=None):
        """Copy the finished image into out (a CUDA tensor, new if None)."""
        import torch
        shape = self._shapes.pop(ticket)
        if out is None:
            out = torch.empty(shape, device="cuda", dtype=self.dtype)
        assert out.is_cuda and out.is_contiguous() and tuple(out.shape) == shape
        assert out.dtype == self.dtype
        _check(_lib.dc_server_fetch(self._h, int(ticket), C.c_void_p(out.data_ptr()), 1))
        return out

    def stats(self):
        st = ServerStats()
        _check(_lib.dc_server_get_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.dc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
