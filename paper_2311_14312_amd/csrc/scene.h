// Scene state shared by the entry points and the FMM driver.
#pragma once

#include <atomic>
#include <memory>

#include "fmm.h"
#include "geometry.h"
#include "kernels.h"
#include "tree.h"

struct dc_scene_s {
    dc_scene_opts opts{};
    dc::Geometry geo;
    dc::Tree tree;
    std::vector<double> uplus, uminus;  // [3][N] host
    // The curves and colour stops the scene was made from (adaptive
    // refinement re-discretises them); boundary_from_stops is false once
    // the caller has set boundary values at the nodes.
    std::vector<double> ctrl, left_rgb, right_rgb;
    int n_stops = 0;
    bool boundary_from_stops = false;

    // Segments (device).
    dc::DevBuf<double> seg_x0, seg_y0, seg_tx, seg_ty, seg_len, seg_ell, seg_kappa;
    // Nodes (device).
    dc::DevBuf<double> node_x, node_y, node_tstar;
    dc::DevBuf<int> node_self;
    dc::DevBuf<double> Pi;
    dc::DevBuf<int> panel_curve;  // [N / g]
    // Boundary data and densities (device, [3][N]).
    dc::DevBuf<double> d_uplus, d_uminus, d_mu, d_sigma;
    bool solved = false;
    // d_mu holds the boundary values u of a mixed solve (dc_solve_mixed)
    // instead of u+ - u-
    bool mu_from_mixed = false;
    // Segment weights of the current densities for the direct path [6][S].
    dc::DevBuf<double> seg_w;
    bool seg_w_valid = false;

    // Inverted diagonal blocks (block-Jacobi preconditioner) and their layout.
    dc::DevBuf<double> dinv;
    bool dinv_valid = false;
    dc::DevBuf<int> blk_panel, blk_node0, blk_n;
    dc::DevBuf<long long> blk_doff;
    int blk_count = 0, blk_max_panels = 0;
    dc::BlocksView blocks() const {
        return {blk_count, blk_max_panels, blk_panel.p, blk_node0.p, blk_n.p, blk_doff.p};
    }

    // FMM state (tree on device, expansions, scratch).
    std::unique_ptr<dc::FmmState> fmm;
    // Number of servers the scene is registered with (they read its
    // densities and upward pass from their own streams).
    std::atomic<int> served{0};

    dc::ChordsView segs() const {
        return {geo.S, seg_x0.p, seg_y0.p, seg_tx.p, seg_ty.p, seg_len.p};
    }
    dc::NodesView nodes() const { return {geo.N, node_x.p, node_y.p, node_self.p, node_tstar.p}; }
};
