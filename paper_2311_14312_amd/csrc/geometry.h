// Host-side geometry of a scene (see geometry.cpp).
#pragma once

#include <vector>

#include "dc_common.h"

namespace dc {

struct ArcTable {
    std::vector<double> t, cum;  // breakpoints in t and L(t) there
    double total = 0.0;
};

struct Geometry {
    int n_curves = 0, P = 0, g = 0, s = 0, N = 0, S = 0;
    std::vector<double> gl_x;                       // GL roots on [-1, 1]
    std::vector<double> node_x, node_y, node_lam;   // [N]
    std::vector<int> node_self;                     // [N] self segment
    std::vector<double> node_tstar;                 // [N] arc fraction on it
    std::vector<double> seg_x0, seg_y0, seg_x1, seg_y1;  // [S] chords
    std::vector<double> seg_ell, seg_kappa;         // [S] arc length, scale
    std::vector<double> curve_len;                  // [n_curves]
    std::vector<double> Pi;                         // [s][g]
    // Panels (N / g of them, listed curve by curve, in order along each):
    // curve and normalised arc-length range.  P above is the panel count
    // per curve when every curve has P equal panels, else 0.
    std::vector<int> panel_curve;
    std::vector<double> panel_lo, panel_hi;
    int n_panels() const { return (int)panel_curve.size(); }
};

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
ArcTable build_arc_table(const double* ctrl8);
double param_at_length(const double* ctrl8, const ArcTable& tab, double T);
std::vector<double> interp_matrix(int g, int s);
void discretize(const double* ctrl, int n_curves, int P, int g, int s, Geometry& G);
// Panels of any lengths (adaptive subdivision, Sec. 7): panel k covers
// normalised arc length [lo[k], hi[k]] of curve pc[k].
void discretize_panels(const double* ctrl, int n_curves, const int* pc, const double* lo,
                       const double* hi, int n_panels, int g, int s, Geometry& G);
void boundary_from_stops(const Geometry& G, const double* left, const double* right,
                         int n_stops, std::vector<double>& up, std::vector<double>& um);

}  // namespace dc
