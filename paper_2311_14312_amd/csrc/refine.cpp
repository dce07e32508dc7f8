// Adaptive subdivision with local re-solve (Sec. 7): Alg. 5 (which panels
// to cut), Alg. 6 (warm start, re-solving curves, local GMRES) and the loop
// of Alg. 7, over the scene kernels.  The quadtree and the FMM state of a
// refined scene are built afresh (make_scene) rather than updated in place
// (Sec. 7.1.2, 7.1.3): on the device a full rebuild of the upward pass costs
// less than one GMRES step, and the operators are evaluated, not stored.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "aa.h"
#include "refine.h"
#include "solve.h"

using namespace dc;

namespace {

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// wp[i] = (2g-1)/2 w_i P_{g-1}(x_i), so that a_{g-1} = sum_i wp[i] sigma_i.
std::vector<double> tail_weights(int g) {
    std::vector<double> x, w;
    gauss_legendre(g, x, w);
    std::vector<double> wp(g);
    for (int i = 0; i < g; ++i) {
        // Bonnet's recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}
        double p0 = 1.0, p1 = x[i];
        if (g == 1) p1 = 1.0;
        for (int n = 1; n < g - 1; ++n) {
            const double p2 = ((2.0 * n + 1.0) * x[i] * p1 - n * p0) / (n + 1.0);
            p0 = p1;
            p1 = p2;
        }
        wp[i] = 0.5 * (2.0 * g - 1.0) * w[i] * p1;
    }
    return wp;
}

// lag[h][i][m]: Lagrange basis polynomial m of the g roots at child node i
// of half h, which sits at (x_i + 1)/2 - 1 (h = 0) or (x_i + 1)/2 (h = 1)
// of the parent's [-1, 1] (Eq. legendre_poly in its Lagrange form).
std::vector<double> child_lagrange(int g) {
    std::vector<double> x, w;
    gauss_legendre(g, x, w);
    std::vector<double> lag((size_t)2 * g * g);
    for (int h = 0; h < 2; ++h)
        for (int i = 0; i < g; ++i) {
            const double at = 0.5 * (x[i] + 1.0) - (h == 0 ? 1.0 : 0.0);
            for (int m = 0; m < g; ++m) {
                double v = 1.0;
                for (int j = 0; j < g; ++j)
                    if (j != m) v *= (at - x[j]) / (x[m] - x[j]);
                lag[((size_t)h * g + i) * g + m] = v;
            }
        }
    return lag;
}

std::vector<double> panel_tails(dc_scene s, hipStream_t st) {
    const Geometry& G = s->geo;
    DevBuf<double> wp, tails;
    wp.upload(tail_weights(G.g));
    tails.alloc(G.n_panels());
    launch_panel_tails(G.n_panels(), G.g, G.N, wp.p, s->d_sigma.p, tails.p, st);
    std::vector<double> out(G.n_panels());
    DC_HIP(hipMemcpyAsync(out.data(), tails.p, out.size() * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    DC_HIP(hipStreamSynchronize(st));
    return out;
}

// Alg. 5 on one scene: the panels to cut.
std::vector<int> select_panels(const Geometry& G, const std::vector<double>& tails,
                               const dc_refine_opts& o) {
    const bool whole = !(o.viewport[2] > 0.0 && o.viewport[3] > 0.0);
    const double xa = o.viewport[0] - 0.5 * o.viewport[2], xb = o.viewport[0] + 0.5 * o.viewport[2];
    const double ya = o.viewport[1] - 0.5 * o.viewport[3], yb = o.viewport[1] + 0.5 * o.viewport[3];
    std::vector<int> chosen;
    for (int k = 0; k < G.n_panels(); ++k) {
        const double len = G.curve_len[G.panel_curve[k]] * (G.panel_hi[k] - G.panel_lo[k]);
        if (!(tails[k] > o.eps2) || len < o.eps1) continue;
        bool in = whole;
        for (int j = k * G.s; !in && j < (k + 1) * G.s; ++j)
            in = segment_meets_box(G.seg_x0[j], G.seg_y0[j], G.seg_x1[j], G.seg_y1[j], xa, xb, ya,
                                   yb);
        if (in) chosen.push_back(k);
    }
    return chosen;
}

// Re-solving curves (Sec. 7.1.4) of the refined scene ns: the cut curves
// and every curve whose potential range under a unit density on a cut curve
// exceeds ratio times the cut curve's own; three cut curves per operator
// application (one per colour channel).
std::vector<unsigned char> label_curves(dc_scene ns, const std::vector<int>& cut_curves,
                                        const dc_refine_opts& o, hipStream_t st) {
    const Geometry& G = ns->geo;
    const int nc = G.n_curves, N = G.N;
    std::vector<unsigned char> res(nc, 0);
    std::vector<int> node0(nc + 1, 0);
    for (int k = 0; k < G.n_panels(); ++k) node0[G.panel_curve[k] + 1] += G.g;
    for (int c = 0; c < nc; ++c) node0[c + 1] += node0[c];
    DevBuf<int> d_node0;
    d_node0.upload(node0);
    DevBuf<double> x, y, range;
    x.alloc(3 * (size_t)N);
    y.alloc(3 * (size_t)N);
    range.alloc(3 * (size_t)nc);
    std::vector<double> h(3 * (size_t)nc);
    for (size_t a = 0; a < cut_curves.size(); a += 3) {
        int cs[3] = {-1, -1, -1};
        for (int q = 0; q < 3 && a + q < cut_curves.size(); ++q) cs[q] = cut_curves[a + q];
        launch_curve_indicator(N, G.g, ns->panel_curve.p, cs, x.p, st);
        apply_operator(ns, x.p, nullptr, y.p, o.solve.matvec, st);
        launch_curve_ranges(nc, N, d_node0.p, y.p, range.p, st);
        DC_HIP(hipMemcpyAsync(h.data(), range.p, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                              st));
        DC_HIP(hipStreamSynchronize(st));
        for (int q = 0; q < 3; ++q) {
            if (cs[q] < 0) continue;
            const double* r = h.data() + (size_t)q * nc;
            res[cs[q]] = 1;
            for (int b = 0; b < nc; ++b)
                if (r[b] > o.ratio * r[cs[q]]) res[b] = 1;
        }
    }
    return res;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

void dc_default_refine_opts(dc_refine_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->eps2 = 1.0;
    o->eps1 = 0.0;
    o->ratio = 0.9;
    o->max_rounds = 1;
    o->local = 1;
    o->solve.tol = 1e-10;
    o->solve.max_iter = 500;
    o->solve.precond = DC_PRECOND_BLOCK;
    dc_default_eval_opts(&o->solve.matvec);
}

int dc_panel_tails(dc_scene s, double* tails_host, void* stream) {
    return guarded([&] {
        DC_REQUIRE(s && tails_host, "null argument");
        DC_REQUIRE(s->solved, "scene has no densities");
        const std::vector<double> t = panel_tails(s, as_stream(stream));
        std::copy(t.begin(), t.end(), tails_host);
    });
}

int dc_refine(dc_scene s, const dc_refine_opts* o, dc_scene* out, dc_refine_report* rep,
              unsigned char* resolved_host, void* stream) {
    int rc = DC_OK;
    int g = guarded([&] {
        DC_REQUIRE(s && o && out && rep, "null argument");
        *out = nullptr;
        std::memset(rep, 0, sizeof(*rep));
        check_not_served(s);
        check_eval(&o->solve.matvec);
        DC_REQUIRE(o->solve.tol > 0 && o->solve.max_iter >= 1, "bad GMRES options");
        DC_REQUIRE(o->solve.precond == DC_PRECOND_NONE || o->solve.precond == DC_PRECOND_BLOCK,
                   "bad preconditioner");
        DC_REQUIRE(std::isfinite(o->eps2) && std::isfinite(o->eps1) && std::isfinite(o->ratio) &&
                       o->ratio >= 0.0 && o->max_rounds >= 0,
                   "bad refinement options");
        for (double v : o->viewport) DC_REQUIRE(std::isfinite(v), "bad refinement viewport");
        DC_REQUIRE(s->solved && !s->mu_from_mixed, "dc_refine needs densities of a two-sided solve");
        DC_REQUIRE(s->boundary_from_stops, "dc_refine needs a scene whose colours are stops");
        const hipStream_t st = as_stream(stream);
        const auto t_all = std::chrono::steady_clock::now();
        rep->converged = 1;
        const int gq = s->geo.g;
        DevBuf<double> d_lag;
        d_lag.upload(child_lagrange(gq));
        std::unique_ptr<dc_scene_s> owned;
        dc_scene cur = s;
        std::vector<unsigned char> res;
        for (int round = 0; round < o->max_rounds; ++round) {
            const Geometry& G = cur->geo;
            const std::vector<int> chosen = select_panels(G, panel_tails(cur, st), *o);
            if (chosen.empty()) break;
            // the new panel list: every chosen panel replaced by its halves
            std::vector<int> pc, parent, half;
            std::vector<double> lo, hi;
            std::vector<int> cut_curves;
            size_t q = 0;
            for (int k = 0; k < G.n_panels(); ++k) {
                const bool cut = q < chosen.size() && chosen[q] == k;
                if (!cut) {
                    pc.push_back(G.panel_curve[k]);
                    lo.push_back(G.panel_lo[k]);
                    hi.push_back(G.panel_hi[k]);
                    parent.push_back(k);
                    half.push_back(-1);
                    continue;
                }
                ++q;
                const double mid = 0.5 * (G.panel_lo[k] + G.panel_hi[k]);
                for (int h = 0; h < 2; ++h) {
                    pc.push_back(G.panel_curve[k]);
                    lo.push_back(h == 0 ? G.panel_lo[k] : mid);
                    hi.push_back(h == 0 ? mid : G.panel_hi[k]);
                    parent.push_back(k);
                    half.push_back(h);
                }
                if (cut_curves.empty() || cut_curves.back() != G.panel_curve[k])
                    cut_curves.push_back(G.panel_curve[k]);
            }
            std::unique_ptr<dc_scene_s> ns =
                make_scene(cur->ctrl.data(), G.n_curves, cur->left_rgb.data(),
                           cur->right_rgb.data(), cur->n_stops, &cur->opts, pc.data(), lo.data(),
                           hi.data(), (int)pc.size());
            const int Nn = ns->geo.N;
            // warm start: the old densities at the new nodes
            DevBuf<int> d_parent, d_half;
            d_parent.upload(parent);
            d_half.upload(half);
            DevBuf<double> x0;
            x0.alloc(3 * (size_t)Nn);
            launch_warm_start((int)pc.size(), gq, G.N, d_parent.p, d_half.p, d_lag.p,
                              cur->d_sigma.p, x0.p, st);
            // re-solving curves
            const auto t_label = std::chrono::steady_clock::now();
            if (o->local) {
                res = label_curves(ns.get(), cut_curves, *o, st);
            } else {
                res.assign(G.n_curves, 1);
            }
            rep->label_seconds += seconds_since(t_label);
            int n_res = 0;
            for (unsigned char v : res) n_res += v;
            DevBuf<unsigned char> d_res, cmask;
            LocalSolve ls{nullptr, x0.p};
            if (n_res < G.n_curves) {
                d_res.upload(res);
                cmask.alloc(Nn);
                launch_constrained_nodes(Nn, gq, ns->panel_curve.p, d_res.p, cmask.p, st);
                ls.cmask = cmask.p;
            }
            const auto t_solve = std::chrono::steady_clock::now();
            dc_solve_report srep{};
            const int src = gmres_solve(ns.get(), o->solve, srep, st, nullptr, &ls);
            rep->solve_seconds += seconds_since(t_solve);
            if (src != DC_OK) {
                rc = src;
                rep->converged = 0;
            }
            rep->rounds += 1;
            rep->panels_cut += (int)chosen.size();
            rep->curves_resolved += n_res;
            rep->iters += std::max(srep.iters[0], std::max(srep.iters[1], srep.iters[2]));
            for (int c = 0; c < 3; ++c)
                rep->rel_residual = std::max(rep->rel_residual, srep.true_rel_residual[c]);
            owned = std::move(ns);
            cur = owned.get();
        }
        rep->n_panels = cur->geo.n_panels();
        if (resolved_host && !res.empty()) std::copy(res.begin(), res.end(), resolved_host);
        rep->seconds = seconds_since(t_all);
        *out = owned.release();
        if (rc != DC_OK) set_last_error("a re-solve did not reach the tolerance");
    });
    return g != DC_OK ? g : rc;
}

}  // extern "C"
