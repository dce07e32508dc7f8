// Solve-side helpers shared by the entry points (api.cpp) and the adaptive
// refinement (refine.cpp).
#pragma once

#include <memory>

#include "scene.h"

namespace dc {

// Mixed Dirichlet/Neumann data of dc_solve_mixed (device): flag [N] = 1 on
// Neumann nodes; values [3][N] = u* on Dirichlet nodes, psi* on Neumann ones.
struct MixedBC {
    const int* neumann;
    const double* values;
};

// Local re-solve (Sec. 7.1.4) and warm start (Sec. 7.1.1), device arrays:
// cmask [N] = 1 on the constrained nodes, whose values x0 keeps (null: every
// node is solved for); x0 [3][N] the initial guess (null: 1 everywhere).
struct LocalSolve {
    const unsigned char* cmask;
    const double* x0;
};

void check_eval(const dc_eval_opts* o);
void check_not_served(dc_scene s);
// y = G_H x + F_H mu at the nodes (x or mu may be null).
void apply_operator(dc_scene s, const double* x, const double* mu, double* y,
                    const dc_eval_opts& o, hipStream_t st);
// GMRES of Alg. 3 on the scene; writes its densities.  DC_OK or
// DC_ERR_NOT_CONVERGED.
int gmres_solve(dc_scene s, const dc_solve_opts& o, dc_solve_report& rep, hipStream_t st,
                const MixedBC* mixed, const LocalSolve* local);
// A scene from curves and colour stops: P equal panels per curve
// (panel_curve null) or the given panels.
std::unique_ptr<dc_scene_s> make_scene(const double* ctrl, int n_curves, const double* left_rgb,
                                       const double* right_rgb, int n_stops,
                                       const dc_scene_opts* opts, const int* panel_curve,
                                       const double* panel_lo, const double* panel_hi,
                                       int n_panels);

}  // namespace dc
