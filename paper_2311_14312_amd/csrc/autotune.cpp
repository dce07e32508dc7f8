// Choice of the render options of a scene (expansion order and tile size)
// against an accuracy target, measured on the device: the FMM image is
// compared at sampled pixels with the FP64 direct sum over every chord
// segment (Alg. 4 without the FMM, the same discrete representation on the
// same geometry), so the error measured is the FMM's own (truncation and
// arithmetic), and the fastest tile size meeting the target is kept.
#include <algorithm>
#include <cmath>
#include <set>
#include <utility>
#include <vector>

#include "autotune.h"

namespace dc {

namespace {

__global__ void k_gather_px(const void* __restrict__ img, int out_f64, int W,
                            const int* __restrict__ rc, int n, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t o = ((size_t)rc[2 * i] * W + rc[2 * i + 1]) * 3;
    for (int ch = 0; ch < 3; ++ch)
        out[3 * i + ch] = out_f64 ? static_cast<const double*>(img)[o + ch]
                                  : (double)static_cast<const float*>(img)[o + ch];
}

// Parameter interval [ta, tb] of the chord p0 + t (p1 - p0), t in [0, 1],
// inside the rectangle [x0, x1] x [y0, y1] (Liang-Barsky clipping); false
// when the chord misses it.
bool clip_chord(double px, double py, double dx, double dy, double x0, double x1, double y0,
                double y1, double& ta, double& tb) {
    ta = 0.0;
    tb = 1.0;
    const double p[4] = {-dx, dx, -dy, dy};
    const double q[4] = {px - x0, x1 - px, py - y0, y1 - py};
    for (int k = 0; k < 4; ++k) {
        if (p[k] == 0.0) {
            if (q[k] < 0.0) return false;
            continue;
        }
        const double r = q[k] / p[k];
        if (p[k] < 0.0) ta = std::max(ta, r);
        else tb = std::min(tb, r);
        if (ta > tb) return false;
    }
    return true;
}

}  // namespace

void tune_sample_pixels(const Geometry& G, const dc_viewport& vp, int want,
                        std::vector<int>& rows, std::vector<int>& cols) {
    std::set<std::pair<int, int>> px;
    // a stride grid over the viewport
    const int n_grid = std::max(1, want / 2);
    const double aspect = (double)vp.W / vp.H;
    const int gw = std::max(1, std::min(vp.W, (int)std::lround(std::sqrt(n_grid * aspect))));
    const int gh = std::max(1, std::min(vp.H, n_grid / gw));
    for (int j = 0; j < gh; ++j)
        for (int i = 0; i < gw; ++i)
            px.insert({(int)((j + 0.5) * vp.H / gh), (int)((i + 0.5) * vp.W / gw)});
    // pixels along the chords that cross the viewport: the near field,
    // where the FP32 path switches to FP64 closed forms
    const double pw = vp.width / vp.W, ph = vp.height / vp.H;
    const double x0 = vp.cx - 0.5 * vp.width, x1 = vp.cx + 0.5 * vp.width;
    const double y0 = vp.cy - 0.5 * vp.height, y1 = vp.cy + 0.5 * vp.height;
    std::vector<std::pair<int, std::pair<double, double>>> cand;
    for (int j = 0; j < G.S; ++j) {
        double ta, tb;
        const double dx = G.seg_x1[j] - G.seg_x0[j], dy = G.seg_y1[j] - G.seg_y0[j];
        if (clip_chord(G.seg_x0[j], G.seg_y0[j], dx, dy, x0, x1, y0, y1, ta, tb))
            cand.push_back({j, {ta, tb}});
    }
    const int n_near = want - n_grid;
    if (!cand.empty() && n_near > 0) {
        const size_t step = std::max<size_t>(1, cand.size() / (size_t)n_near);
        const int per = std::max(1, (int)((n_near + cand.size() - 1) / cand.size()));
        for (size_t c = 0; c < cand.size(); c += step) {
            const int j = cand[c].first;
            const double ta = cand[c].second.first, tb = cand[c].second.second;
            const double dx = G.seg_x1[j] - G.seg_x0[j], dy = G.seg_y1[j] - G.seg_y0[j];
            for (int m = 0; m < per; ++m) {
                const double t = ta + (tb - ta) * (m + 0.5) / per;
                const double x = G.seg_x0[j] + t * dx, y = G.seg_y0[j] + t * dy;
                const int col = std::min(vp.W - 1, std::max(0, (int)std::floor((x - x0) / pw)));
                const int row = std::min(vp.H - 1, std::max(0, (int)std::floor((y1 - y) / ph)));
                px.insert({row, col});
            }
        }
    }
    rows.clear();
    cols.clear();
    for (const auto& rc : px) {
        rows.push_back(rc.first);
        cols.push_back(rc.second);
    }
}

void autotune_scene(dc_scene_s& s, const dc_viewport* vps, int n, const dc_tune_opts& t,
                    const double* seg_w, dc_tune_report& rep, hipStream_t st) {
    const bool f64 = t.precision == DC_PREC_F64;
    const int out_dtype = f64 ? DC_OUT_F64 : DC_OUT_F32;
    const size_t esz = f64 ? 8 : 4;
    // sampled pixels of every viewport and their FP64 direct-sum values
    std::vector<std::vector<int>> rows(n), cols(n);
    std::vector<double> pts;
    std::vector<int> rc;
    std::vector<int> first(n + 1, 0);
    for (int v = 0; v < n; ++v) {
        tune_sample_pixels(s.geo, vps[v], t.samples, rows[v], cols[v]);
        first[v + 1] = first[v] + (int)rows[v].size();
        for (size_t k = 0; k < rows[v].size(); ++k) {
            pts.push_back(pixel_x(vps[v].cx, vps[v].width, vps[v].W, cols[v][k]));
            pts.push_back(pixel_y(vps[v].cy, vps[v].height, vps[v].H, rows[v][k]));
            rc.push_back(rows[v][k]);
            rc.push_back(cols[v][k]);
        }
    }
    const int ns = first[n];
    DevBuf<double> d_pts, d_ref, d_got;
    DevBuf<int> d_rc;
    d_pts.upload(pts);
    d_rc.upload(rc);
    d_ref.alloc((size_t)3 * ns);
    d_got.alloc((size_t)3 * ns);
    launch_direct_targets(nullptr, d_pts.p, ns, s.segs(), seg_w, 1, d_ref.p, st);
    std::vector<double> ref(3 * (size_t)ns), got(3 * (size_t)ns);
    DC_HIP(hipMemcpyAsync(ref.data(), d_ref.p, ref.size() * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    DC_HIP(hipStreamSynchronize(st));
    // images of the candidate renders
    std::vector<DevBuf<char>> imgs(n);
    std::vector<void*> outs(n);
    for (int v = 0; v < n; ++v) {
        imgs[v].alloc((size_t)vps[v].W * vps[v].H * 3 * esz);
        outs[v] = imgs[v].p;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DC_HIP(hipEventCreate(&e0));
    DC_HIP(hipEventCreate(&e1));
    auto cleanup = [&] {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    };
    try {
        auto measure = [&](const dc_eval_opts& o) {
            fmm_render_batch(s, vps, n, o, out_dtype, outs.data(), st);
            for (int v = 0; v < n; ++v) {
                const int m = first[v + 1] - first[v];
                if (m == 0) continue;
                hipLaunchKernelGGL(k_gather_px, dim3((m + 255) / 256), dim3(256), 0, st,
                                   outs[v], f64 ? 1 : 0, vps[v].W, d_rc.p + 2 * first[v], m,
                                   d_got.p + 3 * (size_t)first[v]);
                DC_HIP(hipGetLastError());
            }
            DC_HIP(hipMemcpyAsync(got.data(), d_got.p, got.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, st));
            DC_HIP(hipStreamSynchronize(st));
            double e = 0.0;
            for (size_t i = 0; i < got.size(); ++i) {
                const double d = std::fabs(got[i] - ref[i]);
                e = std::isfinite(d) ? std::max(e, d) : INFINITY;
            }
            return e;
        };
        rep = dc_tune_report{};
        rep.n_samples = ns;
        bool have = false, any_met = false;
        for (int ti = 0; ti < t.n_tiles; ++ti) {
            dc_eval_opts o{};
            dc_default_eval_opts(&o);
            o.method = DC_METHOD_FMM;
            o.precision = t.precision;
            o.tile_px = t.tiles[ti];
            o.near_fp64 = t.near_fp64;
            int p_ok = -1;
            double e_ok = INFINITY;
            for (int p = t.p_min; p <= t.p_max; p += t.p_step) {
                o.p = p;
                const double e = measure(o);
                e_ok = e;
                p_ok = p;
                if (e <= t.target_err) break;
            }
            o.p = p_ok;
            const bool met = e_ok <= t.target_err;
            // time the chosen order for this tile size
            fmm_render_batch(s, vps, n, o, out_dtype, outs.data(), st);
            DC_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < t.timing_reps; ++r)
                fmm_render_batch(s, vps, n, o, out_dtype, outs.data(), st);
            DC_HIP(hipEventRecord(e1, st));
            DC_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            DC_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double per = (double)ms / t.timing_reps;
            rep.tile_p[ti] = p_ok;
            rep.tile_err[ti] = e_ok;
            rep.tile_ms[ti] = per;
            // keep the fastest tile size that meets the target (or, while
            // none does, the most accurate one)
            const bool better = met ? (!any_met || per < rep.ms)
                                    : (!any_met && (!have || e_ok < rep.err));
            if (better) {
                rep.chosen = o;
                rep.err = e_ok;
                rep.ms = per;
                rep.met = met ? 1 : 0;
                have = true;
                any_met = any_met || met;
            }
        }
        // leave the scene prepared for the chosen options
        fmm_prepare(s, rep.chosen, st);
        DC_HIP(hipStreamSynchronize(st));
    } catch (...) {
        (void)hipStreamSynchronize(st);
        cleanup();
        throw;
    }
    cleanup();
}

}  // namespace dc
