// Launch wrappers of the HIP kernels (definitions in the .hip files).
#pragma once

#include "dc_common.h"

namespace dc {

// Structure-of-arrays view of chord elements (segments or clipped pieces).
// x0, y0: start point; tx, ty: unit tangent; len: chord length (FP64).
struct ChordsView {
    int n;
    const double *x0, *y0, *tx, *ty, *len;
};

// Node data for collocation targets.
struct NodesView {
    int N;
    const double *x, *y;
    const int* self_seg;      // [N]
    const double* tstar;      // [N]
};

// w[6][n] = (kappa sigma_bar_c, kappa mu_bar_c) per chord element, where the
// element belongs to segment seg[e] (or e itself when seg == nullptr),
// sigma_bar = Pi sigma per panel (Sec. 5.2).  Either density may be null.
void launch_chord_weights(int n, const int* seg, int s, int g, int N, const double* Pi,
                          const double* kappa, const double* sigma, const double* mu,
                          double* w_f64, float* w_f32, hipStream_t st);

// Direct sum at collocation nodes over every segment, with the singular
// self-segment rule; out[3][N] = sum_j Ghat sigma_bar + Fhat mu_bar.
void launch_direct_nodes(const NodesView& nodes, const ChordsView& segs, const double* ell,
                         const double* kappa, const double* w, double* out,
                         hipStream_t st);

// Direct sum at pixel centres of a viewport (grid != null) or at points.
struct TargetGrid {
    double cx, cy, w, h;
    int W, H;
};
void launch_direct_targets(const TargetGrid* grid, const double* pts, int n_pts,
                           const ChordsView& segs, const double* w, int out_f64,
                           void* out, hipStream_t st);

// ------------------------------------------------------------ GMRES helpers
// dots[c][j] = <V[j][c], w[c]> for j < k (V is [k][3][N]); part holds
// 3 k block_dots_split(N) partial sums.
int block_dots_split(int N);
void launch_block_dots(const double* V, int k, const double* w, int N, double* dots,
                       double* part, hipStream_t st);
// w[c] -= sum_j V[j][c] * h[c][j]; h given on the device [3][kcap] with
// stride kcap.
void launch_block_update(const double* V, int k, const double* h, int kcap, double* w,
                         int N, hipStream_t st);
// y[c] = alpha[c] * x[c] (alpha on the host)
void launch_scale3(const double* x, const double alpha[3], double* y, int N, hipStream_t st);
// y[c] = x[c] / sqrt(n2[c]), 0 where n2[c] <= 0 (n2 [3] on the device)
void launch_scale3_by_norm(const double* x, const double* n2, double* y, int N,
                           hipStream_t st);
// x[c] += sum_j V[j][c] * y[c][j]  (y host-provided on device, stride kcap)
void launch_combine(const double* V, int k, const double* y, int kcap, double* x, int N,
                    hipStream_t st);
// generic: out = a*x + b*y elementwise over n
void launch_axpby(int n, double a, const double* x, double b, const double* y, double* out,
                  hipStream_t st);
void launch_fill(int n, double v, double* out, hipStream_t st);
// [3][N] vectors and a per-node flag [N]: a = v off the flagged nodes, b = v
// on them (zero elsewhere); out0 = flagged ? y : x, out1 = flagged ? x : y.
void launch_mask_split(int N, const int* flag, const double* v, double* a, double* b,
                       hipStream_t st);
void launch_mask_merge(int N, const int* flag, const double* x, const double* y, double* out0,
                       double* out1, hipStream_t st);

// ------------------------------------------------- block-Jacobi preconditioner
// Diagonal blocks: runs of consecutive panels of one curve (every panel of a
// curve when they fit), one after another in D: row-major as assembled,
// transposed in place once inverted (launch_invert_blocks).  Device arrays.
struct BlocksView {
    int n_blocks, max_panels;  // blocks; most panels in one block
    const int* panel_blk;      // [n_panels] block of each panel
    const int* node0;          // [n_blocks] first node of the block
    const int* n;              // [n_blocks] nodes of the block (<= 512)
    const long long* doff;     // [n_blocks] first element of the block in D
};
void launch_curve_blocks(const NodesView& nodes, int g, int s, const ChordsView& segs,
                         const double* ell, const double* kappa, const double* Pi,
                         const BlocksView& bv, double* D, hipStream_t st);
void launch_invert_blocks(const BlocksView& bv, double* D, int* perm, int* singular,
                          hipStream_t st);
// y[ch] = blockdiag(Dinv) x[ch] for the three channels
void launch_block_apply(int N, int g, const BlocksView& bv, const double* Dinv, const double* x,
                        double* y, hipStream_t st);
// [3][N] vectors: out = flag[i] ? a : b (in place allowed)
void launch_select(int N, const unsigned char* flag, const double* a, const double* b,
                   double* out, hipStream_t st);

}  // namespace dc
