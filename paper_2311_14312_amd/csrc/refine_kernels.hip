// Kernels of the adaptive subdivision (Sec. 7): the Legendre tail of every
// panel (Alg. 5), the warm start on the new nodes (Sec. 7.1.1) and the
// potential ranges over the curves that label the re-solving curves
// (Sec. 7.1.4).
#include "refine.h"

namespace dc {

namespace {

constexpr int kNT = 256;

// tails[k] = max_ch |sum_i wp[i] sigma[ch][k g + i]|, wp[i] = (2g-1)/2 w_i
// P_{g-1}(x_i): the highest Legendre coefficient of panel k's density.
__global__ void __launch_bounds__(kNT)
k_panel_tails(int n_panels, int g, int N, const double* __restrict__ wp,
              const double* __restrict__ sigma, double* __restrict__ tails) {
    const int k = blockIdx.x * kNT + threadIdx.x;
    if (k >= n_panels) return;
    double t = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        const double* v = sigma + (size_t)ch * N + (size_t)k * g;
        double a = 0.0;
        for (int i = 0; i < g; ++i) a += wp[i] * v[i];
        t = fmax(t, fabs(a));
    }
    tails[k] = t;
}

// x0[ch][k g + i] of new panel k: its parent's values (half < 0) or their
// Lagrange interpolant at the child's nodes, lag[half][i][m].
__global__ void __launch_bounds__(kNT)
k_warm_start(int n_new, int g, int N_old, const int* __restrict__ parent,
             const int* __restrict__ half, const double* __restrict__ lag,
             const double* __restrict__ sigma_old, double* __restrict__ x0) {
    const long long t = (long long)blockIdx.x * kNT + threadIdx.x;
    const long long N_new = (long long)n_new * g;
    if (t >= 3 * N_new) return;
    const int ch = (int)(t / N_new);
    const int node = (int)(t - (long long)ch * N_new);
    const int k = node / g, i = node - k * g;
    const double* src = sigma_old + (size_t)ch * N_old + (size_t)parent[k] * g;
    const int h = half[k];
    double v;
    if (h < 0) {
        v = src[i];
    } else {
        const double* row = lag + ((size_t)h * g + i) * g;
        v = 0.0;
        for (int m = 0; m < g; ++m) v += row[m] * src[m];
    }
    x0[t] = v;
}

// x[ch][i] = 1 on the nodes of curve curves[ch] (-1: none), else 0.
__global__ void __launch_bounds__(kNT)
k_curve_indicator(int N, int g, const int* __restrict__ panel_curve, int c0, int c1, int c2,
                  double* __restrict__ x) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i >= N) return;
    const int c = panel_curve[i / g];
    x[i] = c == c0 ? 1.0 : 0.0;
    x[(size_t)N + i] = c == c1 ? 1.0 : 0.0;
    x[(size_t)2 * N + i] = c == c2 ? 1.0 : 0.0;
}

// range[ch][c] = max - min of y[ch] over the nodes [node0[c], node0[c+1])
// of curve c (one block per curve and channel; 0 for a curve without nodes).
__global__ void __launch_bounds__(kNT)
k_curve_ranges(int n_curves, int N, const int* __restrict__ node0, const double* __restrict__ y,
               double* __restrict__ range) {
    __shared__ double smin[kNT], smax[kNT];
    const int c = blockIdx.x, ch = blockIdx.y, tid = threadIdx.x;
    const int a = node0[c], b = node0[c + 1];
    double lo = INFINITY, hi = -INFINITY;
    for (int i = a + tid; i < b; i += kNT) {
        const double v = y[(size_t)ch * N + i];
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
    smin[tid] = lo;
    smax[tid] = hi;
    __syncthreads();
    for (int st = kNT / 2; st > 0; st >>= 1) {
        if (tid < st) {
            smin[tid] = fmin(smin[tid], smin[tid + st]);
            smax[tid] = fmax(smax[tid], smax[tid + st]);
        }
        __syncthreads();
    }
    if (tid == 0) range[(size_t)ch * n_curves + c] = b > a ? smax[0] - smin[0] : 0.0;
}

// cmask[i] = 1 on the nodes of curves that are not re-solved.
__global__ void __launch_bounds__(kNT)
k_constrained_nodes(int N, int g, const int* __restrict__ panel_curve,
                    const unsigned char* __restrict__ resolved, unsigned char* __restrict__ cmask) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i >= N) return;
    cmask[i] = resolved[panel_curve[i / g]] ? 0 : 1;
}

inline unsigned blocks(long long n) { return (unsigned)((n + kNT - 1) / kNT); }

}  // namespace

void launch_panel_tails(int n_panels, int g, int N, const double* wp, const double* sigma,
                        double* tails, hipStream_t st) {
    if (n_panels <= 0) return;
    hipLaunchKernelGGL(k_panel_tails, dim3(blocks(n_panels)), dim3(kNT), 0, st, n_panels, g, N,
                       wp, sigma, tails);
    DC_HIP(hipGetLastError());
}

void launch_warm_start(int n_new, int g, int N_old, const int* parent, const int* half,
                       const double* lag, const double* sigma_old, double* x0, hipStream_t st) {
    if (n_new <= 0) return;
    hipLaunchKernelGGL(k_warm_start, dim3(blocks(3LL * n_new * g)), dim3(kNT), 0, st, n_new, g,
                       N_old, parent, half, lag, sigma_old, x0);
    DC_HIP(hipGetLastError());
}

void launch_curve_indicator(int N, int g, const int* panel_curve, const int curves[3], double* x,
                            hipStream_t st) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_curve_indicator, dim3(blocks(N)), dim3(kNT), 0, st, N, g, panel_curve,
                       curves[0], curves[1], curves[2], x);
    DC_HIP(hipGetLastError());
}

void launch_curve_ranges(int n_curves, int N, const int* node0, const double* y, double* range,
                         hipStream_t st) {
    if (n_curves <= 0) return;
    hipLaunchKernelGGL(k_curve_ranges, dim3(n_curves, 3), dim3(kNT), 0, st, n_curves, N, node0,
                       y, range);
    DC_HIP(hipGetLastError());
}

void launch_constrained_nodes(int N, int g, const int* panel_curve, const unsigned char* resolved,
                              unsigned char* cmask, hipStream_t st) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_constrained_nodes, dim3(blocks(N)), dim3(kNT), 0, st, N, g, panel_curve,
                       resolved, cmask);
    DC_HIP(hipGetLastError());
}

}  // namespace dc
