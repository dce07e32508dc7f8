// C ABI entry points (include/dcfmm.h): scene lifecycle, the GMRES solve of
// Alg. 3 and the render of Alg. 4, dispatching to the direct-sum or FMM
// kernels.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>

#include "aa.h"
#include "autotune.h"
#include "scene.h"
#include "solve.h"

using namespace dc;

namespace {
thread_local std::string g_last_error;
}  // namespace

void dc::set_last_error(const std::string& msg) { g_last_error = msg; }

namespace dc {

void check_eval(const dc_eval_opts* o) {
    DC_REQUIRE(o != nullptr, "null eval options");
    DC_REQUIRE(o->method == DC_METHOD_FMM || o->method == DC_METHOD_DIRECT, "bad method");
    DC_REQUIRE(o->precision == DC_PREC_F64 || o->precision == DC_PREC_F32, "bad precision");
    DC_REQUIRE(o->p >= 1 && o->p <= DC_P_MAX, "expansion order p must be in 1..DC_P_MAX");
    DC_REQUIRE(o->tile_px >= 2 && o->tile_px <= 16, "tile_px must be in 2..16");
    DC_REQUIRE(std::isfinite(o->near_fp64) && o->near_fp64 >= 0.0, "bad near_fp64");
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// A scene registered with a server keeps its densities and upward pass
// fixed: the server's streams read them at any time.
void check_not_served(dc_scene s) {
    DC_REQUIRE(s->served.load() == 0,
               "the scene is registered with a server (destroy the server first)");
}
void check_served_opts(dc_scene s, const dc_eval_opts* o) {
    if (s->served.load() == 0 || o->method != DC_METHOD_FMM) return;
    const FmmState& f = *s->fmm;
    DC_REQUIRE(f.up_p == o->p && f.up_prec == (o->precision == DC_PREC_F32 ? 4 : 8),
               "the scene is registered with a server for another order or precision");
}

void upload_boundary(dc_scene s) {
    const int N = s->geo.N;
    s->d_uplus.upload(s->uplus);
    s->d_uminus.upload(s->uminus);
    std::vector<double> mu(3 * (size_t)N);
    for (size_t i = 0; i < mu.size(); ++i) mu[i] = s->uplus[i] - s->uminus[i];
    s->d_mu.upload(mu);
    s->mu_from_mixed = false;
    s->solved = false;
    s->seg_w_valid = false;
    if (s->fmm) fmm_invalidate(*s->fmm);
}

// Segment weights (kappa sigma_bar, kappa mu_bar) of the resident densities.
void ensure_seg_weights(dc_scene s, hipStream_t st) {
    if (s->seg_w_valid) return;
    s->seg_w.alloc((size_t)6 * s->geo.S);
    launch_chord_weights(s->geo.S, nullptr, s->geo.s, s->geo.g, s->geo.N, s->Pi.p,
                         s->seg_kappa.p, s->d_sigma.p, s->d_mu.p, s->seg_w.p, nullptr, st);
    s->seg_w_valid = true;
}

// y = G_H x + c_mu F_H mu at the nodes (x or mu may be null).
void apply_operator(dc_scene s, const double* x, const double* mu, double* y,
                    const dc_eval_opts& o, hipStream_t st) {
    if (o.method == DC_METHOD_DIRECT) {
        DevBuf<double> w;
        w.alloc((size_t)6 * s->geo.S);
        launch_chord_weights(s->geo.S, nullptr, s->geo.s, s->geo.g, s->geo.N, s->Pi.p,
                             s->seg_kappa.p, x, mu, w.p, nullptr, st);
        launch_direct_nodes(s->nodes(), s->segs(), s->seg_ell.p, s->seg_kappa.p, w.p, y, st);
        DC_HIP(hipStreamSynchronize(st));  // w is released on return
    } else {
        fmm_apply_nodes(*s, x, mu, y, o, st);
    }
}

// Inverted diagonal blocks of the preconditioner (computed once per scene):
// runs of consecutive panels of one curve of at most 512 nodes, i.e. one
// block per curve unless the curve has more panels than fit.
void ensure_block_inverse(dc_scene s, hipStream_t st) {
    if (s->dinv_valid) return;
    const Geometry& G = s->geo;
    const int g = G.g, cap = std::max(1, 512 / g), np = G.n_panels();
    std::vector<int> panel_blk(np), node0, nn;
    std::vector<long long> doff;
    long long off = 0;
    int maxp = 0;
    for (int k = 0; k < np;) {
        int e = k + 1;
        while (e < np && e - k < cap && G.panel_curve[e] == G.panel_curve[k]) ++e;
        for (int q = k; q < e; ++q) panel_blk[q] = (int)node0.size();
        const long long n = (long long)(e - k) * g;
        node0.push_back(k * g);
        nn.push_back((int)n);
        doff.push_back(off);
        off += n * n;
        maxp = std::max(maxp, e - k);
        k = e;
    }
    s->blk_panel.upload(panel_blk);
    s->blk_node0.upload(node0);
    s->blk_n.upload(nn);
    s->blk_doff.upload(doff);
    s->blk_count = (int)node0.size();
    s->blk_max_panels = maxp;
    s->dinv.alloc((size_t)off);
    DevBuf<int> perm, flag;
    perm.alloc((size_t)G.N);
    flag.alloc(1);
    const int zero = 0;
    DC_HIP(hipMemcpy(flag.p, &zero, sizeof(int), hipMemcpyHostToDevice));
    launch_curve_blocks(s->nodes(), g, G.s, s->segs(), s->seg_ell.p, s->seg_kappa.p, s->Pi.p,
                        s->blocks(), s->dinv.p, st);
    launch_invert_blocks(s->blocks(), s->dinv.p, perm.p, flag.p, st);
    int singular = 0;
    DC_HIP(hipMemcpyAsync(&singular, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
    DC_HIP(hipStreamSynchronize(st));
    DC_REQUIRE(!singular, "a curve's diagonal block is singular; solve without preconditioner");
    s->dinv_valid = true;
}

// Alg. 3 with GMRES (Sec. 6.5.1): three channels share every matvec; with
// right preconditioning the Krylov space is built for A M^-1.  With mixed
// conditions (Eq. neumann_mat) the unknown x holds psi on Dirichlet nodes
// and u on Neumann nodes, A x = G_H x_d + F_H x_n - x_n / 2 and
// b = u*_d / 2 - G_H psi*_n - F_H u*_d (d, n: the parts on Dirichlet and
// Neumann nodes, zero elsewhere); no preconditioner.  With a local re-solve
// (Eq. local_resolve_mat) the rows of the constrained nodes become the
// identity and their right-hand side the fixed values: the Krylov vectors
// stay zero there, so GMRES runs on (G_H)_rr with b_r - (G_H)_rc sigma_c.
// A given initial guess replaces x0 = 1 (the warm start of Sec. 7.1.1).
// The two events of the Arnoldi steps' copies to the host (see gmres_solve).
struct StepEvents {
    hipEvent_t e[2] = {nullptr, nullptr};
    StepEvents() {
        for (auto& x : e) DC_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    }
    StepEvents(const StepEvents&) = delete;
    StepEvents& operator=(const StepEvents&) = delete;
    ~StepEvents() {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

int gmres_solve(dc_scene s, const dc_solve_opts& o, dc_solve_report& rep, hipStream_t st,
                const MixedBC* mixed, const LocalSolve* local) {
    const int N = s->geo.N;
    const size_t n3 = 3 * (size_t)N;
    const int m = std::max(1, std::min(o.max_iter, N));
    DevBuf<double> b, x, w, tmp, V, dev_h, dots_part;
    b.alloc(n3);
    x.alloc(n3);
    w.alloc(n3);
    tmp.alloc(n3);
    V.alloc((size_t)(m + 1) * n3);
    const int kcap = m + 1;
    // h1 [3][kcap], h2 [3][kcap] and the norms of w [3], one after another:
    // one copy to the host per Arnoldi step
    dev_h.alloc((size_t)6 * kcap + 8);
    dots_part.alloc((size_t)3 * kcap * block_dots_split(N));
    double* h1 = dev_h.p;
    double* h2 = dev_h.p + 3 * kcap;
    double* hn = dev_h.p + 6 * kcap;
    // two host slots: the host reads one step's values while the next
    // step's copy lands in the other
    const size_t slot = 6 * (size_t)kcap + 8;
    PinnedHost<double> host(2 * slot);
    StepEvents ev;
    const bool pre = o.precond == DC_PRECOND_BLOCK && mixed == nullptr;
    DevBuf<double> z;
    if (pre) {
        ensure_block_inverse(s, st);
        z.alloc(n3);
    }
    DevBuf<double> part_d, part_n;
    if (mixed) {
        part_d.alloc(n3);
        part_n.alloc(n3);
    }
    // y = A v
    const unsigned char* cmask = local ? local->cmask : nullptr;
    auto apply_A = [&](const double* v, double* y) {
        if (!mixed) {
            apply_operator(s, v, nullptr, y, o.matvec, st);
            if (cmask) launch_select(N, cmask, v, y, y, st);
            return;
        }
        launch_mask_split(N, mixed->neumann, v, part_d.p, part_n.p, st);
        apply_operator(s, part_d.p, part_n.p, y, o.matvec, st);
        launch_axpby((int)n3, 1.0, y, -0.5, part_n.p, y, st);
    };

    if (!mixed) {
        // b = (u+ + u-)/2 - F_H mu
        apply_operator(s, nullptr, s->d_mu.p, tmp.p, o.matvec, st);
        launch_axpby((int)n3, 0.5, s->d_uplus.p, 0.5, s->d_uminus.p, b.p, st);
        launch_axpby((int)n3, 1.0, b.p, -1.0, tmp.p, b.p, st);
        if (cmask) launch_select(N, cmask, local->x0, b.p, b.p, st);
    } else {
        // known u on Dirichlet nodes (part_d), known psi on Neumann nodes (part_n)
        launch_mask_split(N, mixed->neumann, mixed->values, part_d.p, part_n.p, st);
        apply_operator(s, part_n.p, part_d.p, tmp.p, o.matvec, st);
        launch_axpby((int)n3, 0.5, part_d.p, -1.0, tmp.p, b.p, st);
    }
    // x0 = 1 (or the given guess), r0 = b - A x0
    if (local && local->x0)
        DC_HIP(hipMemcpyAsync(x.p, local->x0, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
        launch_fill((int)n3, 1.0, x.p, st);
    apply_A(x.p, tmp.p);
    launch_axpby((int)n3, 1.0, b.p, -1.0, tmp.p, w.p, st);

    auto norms = [&](const double* vec, double out[3]) {
        launch_block_dots(vec, 1, vec, N, hn, dots_part.p, st);
        DC_HIP(hipMemcpyAsync(host.p, hn, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
        DC_HIP(hipStreamSynchronize(st));
        for (int c = 0; c < 3; ++c) out[c] = std::sqrt(std::max(host.p[c], 0.0));
    };
    double bnorm[3], beta[3];
    norms(b.p, bnorm);
    norms(w.p, beta);

    // Hessenberg columns, Givens rotations and the rotated rhs, per channel.
    // (R: column k holds rows 0..k once step k is done, and only those are
    // read; left uninitialised, since zeroing 3 kcap^2 values took ~6 ms a
    // solve at kcap = 1,001)
    std::unique_ptr<double[]> Rmem(new double[3 * (size_t)kcap * kcap]);
    double* R[3] = {Rmem.get(), Rmem.get() + (size_t)kcap * kcap,
                    Rmem.get() + 2 * (size_t)kcap * kcap};
    std::vector<std::vector<double>> cs(3, std::vector<double>(kcap)), sn(3, std::vector<double>(kcap));
    std::vector<std::vector<double>> gv(3, std::vector<double>(kcap + 1, 0.0));
    bool active[3];
    double alpha[3];
    for (int c = 0; c < 3; ++c) {
        gv[c][0] = beta[c];
        rep.iters[c] = 0;
        const double bn = bnorm[c] > 0 ? bnorm[c] : 1.0;
        rep.rel_residual[c] = beta[c] / bn;
        active[c] = rep.rel_residual[c] > o.tol && beta[c] > 0;
        alpha[c] = beta[c] > 0 ? 1.0 / beta[c] : 0.0;
    }
    launch_scale3(w.p, alpha, V.p, N, st);

    // Arnoldi step k: w = A M^-1 V_k orthogonalised against V_0..V_k, its
    // Hessenberg column and norm copied to host slot k % 2 (event k % 2),
    // and V_{k+1} = w / ||w|| per channel, scaled on the device.  Steps are
    // queued one ahead of the host: step k + 1 runs while the host applies
    // step k's Givens rotations.  A channel that has converged keeps being
    // extended; its later columns are not used.
    auto enqueue_step = [&](int k) {
        double* vk = V.p + (size_t)k * n3;
        if (pre) {
            launch_block_apply(N, s->geo.g, s->blocks(), s->dinv.p, vk, z.p, st);
            if (cmask) launch_select(N, cmask, vk, z.p, z.p, st);
            apply_A(z.p, w.p);
        } else {
            apply_A(vk, w.p);
        }
        // classical Gram-Schmidt, twice (CGS2), against V[0..k]
        launch_block_dots(V.p, k + 1, w.p, N, h1, dots_part.p, st);
        launch_block_update(V.p, k + 1, h1, k + 1, w.p, N, st);
        launch_block_dots(V.p, k + 1, w.p, N, h2, dots_part.p, st);
        launch_block_update(V.p, k + 1, h2, k + 1, w.p, N, st);
        launch_block_dots(w.p, 1, w.p, N, hn, dots_part.p, st);
        // h1 and h2 (3 (k + 1) values each, at the starts of their slots)
        // and the norms, in one copy to pinned memory
        DC_HIP(hipMemcpyAsync(host.p + (k % 2) * slot, dev_h.p,
                              (6 * (size_t)kcap + 3) * sizeof(double), hipMemcpyDeviceToHost,
                              st));
        DC_HIP(hipEventRecord(ev.e[k % 2], st));
        launch_scale3_by_norm(w.p, hn, V.p + (size_t)(k + 1) * n3, N, st);
    };
    if (active[0] || active[1] || active[2]) enqueue_step(0);
    for (int k = 0; k < m && (active[0] || active[1] || active[2]); ++k) {
        if (k + 1 < m) enqueue_step(k + 1);
        DC_HIP(hipEventSynchronize(ev.e[k % 2]));
        const double* hs = host.p + (k % 2) * slot;
        for (int c = 0; c < 3; ++c) {
            if (!active[c]) continue;
            double* col = &R[c][(size_t)k * kcap];
            for (int j = 0; j <= k; ++j)
                col[j] = hs[(size_t)c * (k + 1) + j] + hs[3 * (size_t)kcap + (size_t)c * (k + 1) + j];
            const double hk1 = std::sqrt(std::max(hs[6 * (size_t)kcap + c], 0.0));
            for (int j = 0; j < k; ++j) {
                const double a = cs[c][j] * col[j] + sn[c][j] * col[j + 1];
                col[j + 1] = -sn[c][j] * col[j] + cs[c][j] * col[j + 1];
                col[j] = a;
            }
            const double r = std::hypot(col[k], hk1);
            cs[c][k] = r > 0 ? col[k] / r : 1.0;
            sn[c][k] = r > 0 ? hk1 / r : 0.0;
            col[k] = r;
            gv[c][k + 1] = -sn[c][k] * gv[c][k];
            gv[c][k] = cs[c][k] * gv[c][k];
            rep.iters[c] = k + 1;
            const double bn = bnorm[c] > 0 ? bnorm[c] : 1.0;
            rep.rel_residual[c] = std::fabs(gv[c][k + 1]) / bn;
            if (rep.rel_residual[c] <= o.tol || hk1 == 0.0) active[c] = false;
        }
    }
    // Back substitution R y = g per channel; x += V y.
    std::vector<double> y(3 * (size_t)kcap, 0.0);
    for (int c = 0; c < 3; ++c) {
        const int kk = rep.iters[c];
        for (int i = kk - 1; i >= 0; --i) {
            double acc = gv[c][i];
            for (int j = i + 1; j < kk; ++j) acc -= R[c][(size_t)j * kcap + i] * y[(size_t)c * kcap + j];
            const double d = R[c][(size_t)i * kcap + i];
            y[(size_t)c * kcap + i] = d != 0 ? acc / d : 0.0;
        }
    }
    int kmax = std::max(rep.iters[0], std::max(rep.iters[1], rep.iters[2]));
    if (kmax > 0) {
        DevBuf<double> dy;
        dy.upload(y);
        if (pre) {
            // x += M^-1 (V y)
            launch_fill((int)n3, 0.0, tmp.p, st);
            launch_combine(V.p, kmax, dy.p, kcap, tmp.p, N, st);
            launch_block_apply(N, s->geo.g, s->blocks(), s->dinv.p, tmp.p, z.p, st);
            if (cmask) launch_select(N, cmask, tmp.p, z.p, z.p, st);
            launch_axpby((int)n3, 1.0, x.p, 1.0, z.p, x.p, st);
        } else {
            launch_combine(V.p, kmax, dy.p, kcap, x.p, N, st);
        }
        DC_HIP(hipStreamSynchronize(st));
    }
    // True residual.
    apply_A(x.p, tmp.p);
    launch_axpby((int)n3, 1.0, b.p, -1.0, tmp.p, w.p, st);
    double rn[3];
    norms(w.p, rn);
    rep.converged = 1;
    for (int c = 0; c < 3; ++c) {
        rep.true_rel_residual[c] = rn[c] / (bnorm[c] > 0 ? bnorm[c] : 1.0);
        if (rep.rel_residual[c] > o.tol) rep.converged = 0;
    }
    s->d_sigma.alloc(n3);
    if (!mixed) {
        DC_HIP(hipMemcpyAsync(s->d_sigma.p, x.p, n3 * sizeof(double), hipMemcpyDeviceToDevice,
                              st));
    } else {
        // psi = x on Dirichlet nodes, psi* on Neumann nodes; u = u* on
        // Dirichlet nodes, x on Neumann nodes (the double-layer density)
        s->d_mu.alloc(n3);
        launch_mask_merge(N, mixed->neumann, x.p, mixed->values, s->d_sigma.p, s->d_mu.p, st);
    }
    DC_HIP(hipStreamSynchronize(st));
    s->solved = true;
    s->seg_w_valid = false;
    if (s->fmm) fmm_invalidate(*s->fmm);
    return rep.converged ? DC_OK : DC_ERR_NOT_CONVERGED;
}

std::unique_ptr<dc_scene_s> make_scene(const double* ctrl, int n_curves, const double* left_rgb,
                                       const double* right_rgb, int n_stops,
                                       const dc_scene_opts* opts, const int* panel_curve,
                                       const double* panel_lo, const double* panel_hi,
                                       int n_panels) {
    auto s = std::make_unique<dc_scene_s>();
    s->opts = *opts;
    if (panel_curve == nullptr)
        discretize(ctrl, n_curves, opts->panels_per_curve, opts->gl_per_panel,
                   opts->segs_per_panel, s->geo);
    else
        discretize_panels(ctrl, n_curves, panel_curve, panel_lo, panel_hi, n_panels,
                          opts->gl_per_panel, opts->segs_per_panel, s->geo);
    boundary_from_stops(s->geo, left_rgb, right_rgb, n_stops, s->uplus, s->uminus);
    s->ctrl.assign(ctrl, ctrl + (size_t)n_curves * 8);
    s->left_rgb.assign(left_rgb, left_rgb + (size_t)n_curves * n_stops * 3);
    s->right_rgb.assign(right_rgb, right_rgb + (size_t)n_curves * n_stops * 3);
    s->n_stops = n_stops;
    s->boundary_from_stops = true;
    build_tree(s->geo, opts->leaf_max, opts->max_depth, opts->domain, s->tree);
    const Geometry& G = s->geo;
    std::vector<double> tx(G.S), ty(G.S), len(G.S);
    for (int j = 0; j < G.S; ++j) {
        const double ax = G.seg_x1[j] - G.seg_x0[j], ay = G.seg_y1[j] - G.seg_y0[j];
        len[j] = std::hypot(ax, ay);
        tx[j] = ax / len[j];
        ty[j] = ay / len[j];
    }
    s->seg_x0.upload(G.seg_x0);
    s->seg_y0.upload(G.seg_y0);
    s->seg_tx.upload(tx);
    s->seg_ty.upload(ty);
    s->seg_len.upload(len);
    s->seg_ell.upload(G.seg_ell);
    s->seg_kappa.upload(G.seg_kappa);
    s->node_x.upload(G.node_x);
    s->node_y.upload(G.node_y);
    s->node_tstar.upload(G.node_tstar);
    s->node_self.upload(G.node_self);
    s->Pi.upload(G.Pi);
    s->panel_curve.upload(G.panel_curve);
    upload_boundary(s.get());
    s->fmm = fmm_create(*s);
    return s;
}

}  // namespace dc

extern "C" {

void dc_default_scene_opts(dc_scene_opts* o) {
    if (!o) return;
    o->panels_per_curve = 16;
    o->gl_per_panel = 16;
    o->segs_per_panel = 80;
    o->leaf_max = 64;
    o->max_depth = 40;
    o->domain[0] = -0.45;
    o->domain[1] = -0.45;
    o->domain[2] = 1.45;
    o->domain[3] = 1.45;
}

void dc_default_eval_opts(dc_eval_opts* e) {
    if (!e) return;
    e->method = DC_METHOD_FMM;
    e->precision = DC_PREC_F64;
    e->p = 20;
    e->tile_px = 8;
    e->near_fp64 = 1e-3;
}

int dc_scene_create(const double* ctrl, int n_curves, const double* left_rgb,
                    const double* right_rgb, int n_stops, const dc_scene_opts* opts,
                    dc_scene* out) {
    return guarded([&] {
        DC_REQUIRE(ctrl && left_rgb && right_rgb && opts && out, "null argument");
        *out = nullptr;
        *out = make_scene(ctrl, n_curves, left_rgb, right_rgb, n_stops, opts, nullptr, nullptr,
                          nullptr, 0)
                   .release();
    });
}

int dc_scene_create_panels(const double* ctrl, int n_curves, const double* left_rgb,
                           const double* right_rgb, int n_stops, const int* panel_curve,
                           const double* panel_lo, const double* panel_hi, int n_panels,
                           const dc_scene_opts* opts, dc_scene* out) {
    return guarded([&] {
        DC_REQUIRE(ctrl && left_rgb && right_rgb && panel_curve && panel_lo && panel_hi && opts &&
                       out,
                   "null argument");
        *out = nullptr;
        *out = make_scene(ctrl, n_curves, left_rgb, right_rgb, n_stops, opts, panel_curve,
                          panel_lo, panel_hi, n_panels)
                   .release();
    });
}

int dc_scene_panels(dc_scene s, int* n_panels, int* panel_curve, double* panel_lo,
                    double* panel_hi) {
    return guarded([&] {
        DC_REQUIRE(s && n_panels, "null argument");
        const Geometry& G = s->geo;
        *n_panels = G.n_panels();
        for (int k = 0; k < G.n_panels(); ++k) {
            if (panel_curve) panel_curve[k] = G.panel_curve[k];
            if (panel_lo) panel_lo[k] = G.panel_lo[k];
            if (panel_hi) panel_hi[k] = G.panel_hi[k];
        }
    });
}

void dc_scene_destroy(dc_scene s) {
    if (!s) return;
    if (s->served.load() != 0) {
        // still read by a server's streams: keep it alive (documented misuse)
        g_last_error = "dc_scene_destroy: scene is registered with a server; not destroyed";
        return;
    }
    delete s;
}

int dc_scene_get_info(dc_scene s, dc_scene_info* info) {
    return guarded([&] {
        DC_REQUIRE(s && info, "null argument");
        info->n_curves = s->geo.n_curves;
        info->N = s->geo.N;
        info->S = s->geo.S;
        info->n_pieces = (int)s->tree.pseg.size();
        info->n_cells = s->tree.n_cells;
        info->n_leaves = s->tree.n_leaves;
        info->depth = s->tree.depth;
        info->root[0] = s->tree.X0;
        info->root[1] = s->tree.Y0;
        info->root[2] = s->tree.side;
        info->solved = s->solved ? 1 : 0;
        info->table_pairs = s->fmm ? s->fmm->tab_ok ? s->fmm->tab_pairs : 0 : 0;
        info->table_bytes = s->fmm ? s->fmm->tab_ok ? (long long)s->fmm->tab_bytes : 0 : 0;
    });
}

int dc_set_solve_tables(dc_scene s, int enable) {
    return guarded([&] {
        DC_REQUIRE(s && enable >= 0 && enable <= 2, "bad argument");
        check_not_served(s);
        DC_REQUIRE(s->fmm != nullptr, "scene has no FMM state");
        FmmState& f = *s->fmm;
        DC_HIP(hipDeviceSynchronize());  // no launch may still read the tables
        f.tab_mode = enable;
        f.tab_tried = false;
        f.tab_ok = false;
        f.tab_bytes = 0;
        f.tab_pairs = 0;
        f.tab_pair_off.release();
        f.tab_piece_off.release();
        f.tab_w_off.release();
        f.tab_piece.release();
        f.tab_w.release();
        f.tab_val.release();
        f.p2m_tab.release();
        f.p2m_tab_p = -1;
    });
}

int dc_get_nodes(dc_scene s, double* xy) {
    return guarded([&] {
        DC_REQUIRE(s && xy, "null argument");
        for (int i = 0; i < s->geo.N; ++i) {
            xy[2 * (size_t)i] = s->geo.node_x[i];
            xy[2 * (size_t)i + 1] = s->geo.node_y[i];
        }
    });
}

int dc_set_boundary(dc_scene s, const double* up, const double* um) {
    return guarded([&] {
        DC_REQUIRE(s && up && um, "null argument");
        check_not_served(s);
        const size_t n3 = 3 * (size_t)s->geo.N;
        for (size_t i = 0; i < n3; ++i)
            DC_REQUIRE(std::isfinite(up[i]) && std::isfinite(um[i]), "non-finite boundary value");
        s->uplus.assign(up, up + n3);
        s->uminus.assign(um, um + n3);
        s->boundary_from_stops = false;
        upload_boundary(s);
    });
}

int dc_solve_densities(dc_scene s, const dc_solve_opts* o, dc_solve_report* rep, void* stream) {
    int rc = DC_OK;
    int g = guarded([&] {
        DC_REQUIRE(s && o && rep, "null argument");
        check_not_served(s);
        check_eval(&o->matvec);
        DC_REQUIRE(o->tol > 0 && o->max_iter >= 1, "bad GMRES options");
        DC_REQUIRE(o->precond == DC_PRECOND_NONE || o->precond == DC_PRECOND_BLOCK,
                   "bad preconditioner");
        std::memset(rep, 0, sizeof(*rep));
        if (s->mu_from_mixed) upload_boundary(s);  // two-sided data again
        const auto t0 = std::chrono::steady_clock::now();
        rc = gmres_solve(s, *o, *rep, as_stream(stream), nullptr, nullptr);
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (rc != DC_OK) g_last_error = "GMRES did not reach the tolerance";
    });
    return g != DC_OK ? g : rc;
}

int dc_solve_mixed(dc_scene s, const int* neumann, const double* values,
                   const dc_solve_opts* o, dc_solve_report* rep, void* stream) {
    int rc = DC_OK;
    int g = guarded([&] {
        DC_REQUIRE(s && neumann && values && o && rep, "null argument");
        check_not_served(s);
        check_eval(&o->matvec);
        DC_REQUIRE(o->tol > 0 && o->max_iter >= 1, "bad GMRES options");
        DC_REQUIRE(o->precond == DC_PRECOND_NONE, "mixed conditions take no preconditioner");
        const int N = s->geo.N;
        std::vector<int> flag(neumann, neumann + N);
        for (int v : flag) DC_REQUIRE(v == 0 || v == 1, "neumann flags must be 0 or 1");
        std::vector<double> vals(values, values + 3 * (size_t)N);
        for (double v : vals) DC_REQUIRE(std::isfinite(v), "non-finite boundary value");
        std::memset(rep, 0, sizeof(*rep));
        DevBuf<int> d_flag;
        DevBuf<double> d_vals;
        d_flag.upload(flag);
        d_vals.upload(vals);
        const MixedBC mixed{d_flag.p, d_vals.p};
        const auto t0 = std::chrono::steady_clock::now();
        rc = gmres_solve(s, *o, *rep, as_stream(stream), &mixed, nullptr);
        s->mu_from_mixed = true;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (rc != DC_OK) g_last_error = "GMRES did not reach the tolerance";
    });
    return g != DC_OK ? g : rc;
}

int dc_get_densities(dc_scene s, double* sigma) {
    return guarded([&] {
        DC_REQUIRE(s && sigma, "null argument");
        DC_REQUIRE(s->solved, "scene has no densities");
        DC_HIP(hipMemcpy(sigma, s->d_sigma.p, 3 * (size_t)s->geo.N * sizeof(double),
                         hipMemcpyDeviceToHost));
    });
}

int dc_set_densities(dc_scene s, const double* sigma) {
    return guarded([&] {
        DC_REQUIRE(s && sigma, "null argument");
        check_not_served(s);
        const size_t n3 = 3 * (size_t)s->geo.N;
        for (size_t i = 0; i < n3; ++i) DC_REQUIRE(std::isfinite(sigma[i]), "non-finite density");
        if (s->mu_from_mixed) upload_boundary(s);  // two-sided data again
        std::vector<double> v(sigma, sigma + n3);
        s->d_sigma.upload(v);
        s->solved = true;
        s->seg_w_valid = false;
        if (s->fmm) fmm_invalidate(*s->fmm);
    });
}

int dc_apply_operator(dc_scene s, const double* x, double* y, int c_mu, const dc_eval_opts* o,
                      void* stream) {
    return guarded([&] {
        DC_REQUIRE(s && x && y, "null argument");
        check_not_served(s);
        check_eval(o);
        apply_operator(s, x, c_mu ? s->d_mu.p : nullptr, y, *o, as_stream(stream));
    });
}

int dc_render(dc_scene s, const dc_viewport* vp, const dc_eval_opts* o, int out_dtype,
              void* out, void* stream) {
    return guarded([&] {
        DC_REQUIRE(s && vp && out, "null argument");
        check_eval(o);
        check_served_opts(s, o);
        DC_REQUIRE(s->solved, "render needs densities (solve or set them first)");
        DC_REQUIRE(vp->W >= 1 && vp->H >= 1 && vp->width > 0 && vp->height > 0 &&
                       std::isfinite(vp->cx) && std::isfinite(vp->cy) &&
                       std::isfinite(vp->width) && std::isfinite(vp->height),
                   "bad viewport");
        DC_REQUIRE(out_dtype == DC_OUT_F32 || out_dtype == DC_OUT_F64, "bad out_dtype");
        hipStream_t st = as_stream(stream);
        if (o->method == DC_METHOD_DIRECT) {
            ensure_seg_weights(s, st);
            TargetGrid g{vp->cx, vp->cy, vp->width, vp->height, vp->W, vp->H};
            launch_direct_targets(&g, nullptr, 0, s->segs(), s->seg_w.p, out_dtype, out, st);
        } else {
            fmm_render(*s, *vp, *o, out_dtype, out, st);
        }
    });
}

int dc_render_noalloc(dc_scene s, const dc_viewport* vp, const dc_eval_opts* o, int out_dtype,
                      void* out, void* stream) {
    return guarded([&] {
        DC_REQUIRE(s && vp && out, "null argument");
        check_eval(o);
        check_served_opts(s, o);
        DC_REQUIRE(o->method == DC_METHOD_FMM, "dc_render_noalloc is an FMM path");
        DC_REQUIRE(s->solved, "render needs densities (solve or set them first)");
        DC_REQUIRE(vp->W >= 1 && vp->H >= 1 && vp->width > 0 && vp->height > 0 &&
                       std::isfinite(vp->cx) && std::isfinite(vp->cy) &&
                       std::isfinite(vp->width) && std::isfinite(vp->height),
                   "bad viewport");
        DC_REQUIRE(out_dtype == DC_OUT_F32 || out_dtype == DC_OUT_F64, "bad out_dtype");
        fmm_render_noalloc(*s, *vp, *o, out_dtype, out, as_stream(stream));
    });
}

int dc_render_batch(dc_scene s, const dc_viewport* vps, int n, const dc_eval_opts* o,
                    int out_dtype, void* const* outs, void* stream) {
    return guarded([&] {
        DC_REQUIRE(s && vps && outs && n >= 1, "bad argument");
        check_eval(o);
        check_served_opts(s, o);
        DC_REQUIRE(o->method == DC_METHOD_FMM, "batched render is an FMM path");
        DC_REQUIRE(s->solved, "render needs densities (solve or set them first)");
        for (int v = 0; v < n; ++v) {
            const dc_viewport* vp = &vps[v];
            DC_REQUIRE(outs[v], "null output");
            DC_REQUIRE(vp->W >= 1 && vp->H >= 1 && vp->width > 0 && vp->height > 0 &&
                           std::isfinite(vp->cx) && std::isfinite(vp->cy) &&
                           std::isfinite(vp->width) && std::isfinite(vp->height),
                       "bad viewport");
        }
        DC_REQUIRE(out_dtype == DC_OUT_F32 || out_dtype == DC_OUT_F64, "bad out_dtype");
        fmm_render_batch(*s, vps, n, *o, out_dtype, outs, as_stream(stream));
    });
}

int dc_render_aa(dc_scene s, const dc_viewport* vp, const dc_eval_opts* o, int aa,
                 int out_dtype, void* out, dc_aa_report* rep, void* stream) {
    return guarded([&] {
        DC_REQUIRE(s && vp && out, "null argument");
        check_eval(o);
        check_served_opts(s, o);
        DC_REQUIRE(o->method == DC_METHOD_FMM, "dc_render_aa is an FMM path");
        DC_REQUIRE(aa >= 2 && aa <= 16, "aa must be in 2..16");
        DC_REQUIRE(s->solved, "render needs densities (solve or set them first)");
        DC_REQUIRE(vp->W >= 1 && vp->H >= 1 && vp->width > 0 && vp->height > 0 &&
                       std::isfinite(vp->cx) && std::isfinite(vp->cy) &&
                       std::isfinite(vp->width) && std::isfinite(vp->height),
                   "bad viewport");
        DC_REQUIRE(out_dtype == DC_OUT_F32 || out_dtype == DC_OUT_F64, "bad out_dtype");
        render_aa(*s, *vp, *o, aa, out_dtype, out, rep, as_stream(stream));
    });
}

void dc_default_tune_opts(dc_tune_opts* t) {
    if (!t) return;
    std::memset(t, 0, sizeof(*t));
    t->target_err = 5e-5;
    t->precision = DC_PREC_F32;
    t->p_min = 8;
    t->p_max = 24;
    t->p_step = 2;
    t->tiles[0] = 8;
    t->tiles[1] = 16;
    t->n_tiles = 2;
    t->samples = 1024;
    t->near_fp64 = 1e-3;
    t->timing_reps = 5;
}

int dc_autotune(dc_scene s, const dc_viewport* vps, int n, const dc_tune_opts* t,
                dc_tune_report* rep, void* stream) {
    return guarded([&] {
        DC_REQUIRE(s && vps && t && rep && n >= 1, "bad argument");
        check_not_served(s);
        DC_REQUIRE(s->solved, "tuning needs densities (solve or set them first)");
        DC_REQUIRE(t->precision == DC_PREC_F32 || t->precision == DC_PREC_F64, "bad precision");
        DC_REQUIRE(t->n_tiles >= 1 && t->n_tiles <= 4, "n_tiles must be in 1..4");
        for (int k = 0; k < t->n_tiles; ++k)
            DC_REQUIRE(t->tiles[k] >= 2 && t->tiles[k] <= 16, "tile sizes must be in 2..16");
        DC_REQUIRE(t->p_min >= 1 && t->p_min <= t->p_max && t->p_max <= DC_P_MAX && t->p_step >= 1,
                   "bad order range");
        DC_REQUIRE(t->samples >= 2 && t->timing_reps >= 1, "bad sample or timing count");
        DC_REQUIRE(t->target_err > 0 && std::isfinite(t->near_fp64) && t->near_fp64 >= 0,
                   "bad target or near_fp64");
        for (int v = 0; v < n; ++v) {
            const dc_viewport* vp = &vps[v];
            DC_REQUIRE(vp->W >= 1 && vp->H >= 1 && vp->width > 0 && vp->height > 0 &&
                           std::isfinite(vp->cx) && std::isfinite(vp->cy) &&
                           std::isfinite(vp->width) && std::isfinite(vp->height),
                       "bad viewport");
        }
        hipStream_t st = as_stream(stream);
        ensure_seg_weights(s, st);
        autotune_scene(*s, vps, n, *t, s->seg_w.p, *rep, st);
    });
}

int dc_eval_points(dc_scene s, const double* xy, int n, const dc_eval_opts* o, int out_dtype,
                   void* out, void* stream) {
    return guarded([&] {
        DC_REQUIRE(s && xy && out && n >= 0, "bad argument");
        check_eval(o);
        DC_REQUIRE(s->solved, "evaluation needs densities");
        DC_REQUIRE(out_dtype == DC_OUT_F32 || out_dtype == DC_OUT_F64, "bad out_dtype");
        hipStream_t st = as_stream(stream);
        ensure_seg_weights(s, st);
        launch_direct_targets(nullptr, xy, n, s->segs(), s->seg_w.p, out_dtype, out, st);
    });
}

struct dc_render_graph_s {
    std::unique_ptr<dc::RenderGraph> g;
};

int dc_render_graph_create(dc_scene s, const dc_viewport* vps, int n, const dc_eval_opts* o,
                           int out_dtype, void* const* outs, dc_render_graph* out) {
    return guarded([&] {
        DC_REQUIRE(s && vps && outs && out && n >= 1, "bad argument");
        *out = nullptr;
        check_eval(o);
        check_not_served(s);
        DC_REQUIRE(o->method == DC_METHOD_FMM, "a render graph is an FMM path");
        DC_REQUIRE(s->solved, "render needs densities (solve or set them first)");
        for (int v = 0; v < n; ++v) {
            const dc_viewport* vp = &vps[v];
            DC_REQUIRE(outs[v], "null output");
            DC_REQUIRE(vp->W >= 1 && vp->H >= 1 && vp->width > 0 && vp->height > 0 &&
                           std::isfinite(vp->cx) && std::isfinite(vp->cy) &&
                           std::isfinite(vp->width) && std::isfinite(vp->height),
                       "bad viewport");
        }
        DC_REQUIRE(out_dtype == DC_OUT_F32 || out_dtype == DC_OUT_F64, "bad out_dtype");
        auto h = std::make_unique<dc_render_graph_s>();
        h->g = fmm_graph_create(*s, vps, n, *o, out_dtype, outs);
        *out = h.release();
    });
}

int dc_render_graph_launch(dc_render_graph g, void* stream) {
    return guarded([&] {
        DC_REQUIRE(g && g->g, "bad argument");
        check_not_served(g->g->s);
        fmm_graph_launch(*g->g, as_stream(stream));
    });
}

void dc_render_graph_destroy(dc_render_graph g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    delete g;
}

int dc_render_counts(dc_scene s, const dc_viewport* vp, const dc_eval_opts* o,
                     dc_work_counts* counts, void* stream) {
    return guarded([&] {
        DC_REQUIRE(s && vp && o && counts, "null argument");
        check_eval(o);
        check_served_opts(s, o);
        DC_REQUIRE(o->method == DC_METHOD_FMM, "work counts are defined for the FMM path");
        DC_REQUIRE(s->solved, "render needs densities (solve or set them first)");
        DC_REQUIRE(vp->W >= 1 && vp->H >= 1 && vp->width > 0 && vp->height > 0, "bad viewport");
        std::memset(counts, 0, sizeof(*counts));
        fmm_render_counts(*s, *vp, *o, counts, as_stream(stream));
    });
}

int dc_set_timing(dc_scene s, int enable) {
    return guarded([&] {
        DC_REQUIRE(s, "null scene");
        FmmState& f = *s->fmm;
        if (enable)
            for (hipEvent_t& e : f.ev)
                if (!e) DC_HIP(hipEventCreate(&e));
        f.timing = enable != 0;
    });
}

int dc_get_timing(dc_scene s, double* ms) {
    return guarded([&] {
        DC_REQUIRE(s && ms, "null argument");
        FmmState& f = *s->fmm;
        for (int i = 0; i < 4; ++i) {
            ms[i] = f.tms[i];
            f.tms[i] = 0;
        }
        ms[4] = f.tcalls;
        f.tcalls = 0;
    });
}

const char* dc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
