// Adaptive subdivision with local re-solve (Sec. 7): kernels
// (refine_kernels.hip) and the dc_refine driver (refine.cpp).
#pragma once

#include "dc_common.h"

namespace dc {

void launch_panel_tails(int n_panels, int g, int N, const double* wp, const double* sigma,
                        double* tails, hipStream_t st);
void launch_warm_start(int n_new, int g, int N_old, const int* parent, const int* half,
                       const double* lag, const double* sigma_old, double* x0, hipStream_t st);
void launch_curve_indicator(int N, int g, const int* panel_curve, const int curves[3], double* x,
                            hipStream_t st);
void launch_curve_ranges(int n_curves, int N, const int* node0, const double* y, double* range,
                         hipStream_t st);
void launch_constrained_nodes(int N, int g, const int* panel_curve, const unsigned char* resolved,
                              unsigned char* cmask, hipStream_t st);

}  // namespace dc
