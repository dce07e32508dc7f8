// Direct-sum kernels (brute-force evaluation, Sec. 5.5), density
// interpolation onto chords (Sec. 5.2) and the vector kernels of GMRES.
#include "kernels.h"

namespace dc {

namespace {

constexpr int kNT = 256;

__global__ void __launch_bounds__(kNT)
k_chord_weights(int n, const int* __restrict__ seg, int s, int g, int N,
                const double* __restrict__ Pi, const double* __restrict__ kappa,
                const double* __restrict__ sigma, const double* __restrict__ mu,
                double* __restrict__ w64, float* __restrict__ w32) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int j = seg ? seg[e] : e;
    const int panel = j / s, jj = j - panel * s;
    const double* pr = Pi + (size_t)jj * g;
    const double kap = kappa[j];
    const size_t base = (size_t)panel * g;
    for (int c = 0; c < 3; ++c) {
        double vs = 0.0, vm = 0.0;
        if (sigma)
            for (int i = 0; i < g; ++i) vs += pr[i] * sigma[(size_t)c * N + base + i];
        if (mu)
            for (int i = 0; i < g; ++i) vm += pr[i] * mu[(size_t)c * N + base + i];
        vs *= kap;
        vm *= kap;
        if (w64) {
            w64[(size_t)c * n + e] = vs;
            w64[(size_t)(3 + c) * n + e] = vm;
        }
        if (w32) {
            w32[(size_t)c * n + e] = (float)vs;
            w32[(size_t)(3 + c) * n + e] = (float)vm;
        }
    }
}

// One chord element staged in LDS.
struct SegTile {
    double x0[kNT], y0[kNT], tx[kNT], ty[kNT], len[kNT];
    double w[6][kNT];
};

__device__ inline void stage_segments(SegTile& sh, const ChordsView& segs, const double* w,
                                      int base) {
    const int t = threadIdx.x;
    const int j = base + t;
    if (j < segs.n) {
        sh.x0[t] = segs.x0[j];
        sh.y0[t] = segs.y0[j];
        sh.tx[t] = segs.tx[j];
        sh.ty[t] = segs.ty[j];
        sh.len[t] = segs.len[j];
        for (int c = 0; c < 6; ++c) sh.w[c][t] = w[(size_t)c * segs.n + j];
    }
}

// u(q_i) for every collocation node: sum over all segments of the chord
// closed forms, except the node's own segment, which takes the singular
// single layer of App. D.3 and a zero double layer (App. C.1, D.4).
__global__ void __launch_bounds__(kNT)
k_direct_nodes(NodesView nodes, ChordsView segs, const double* __restrict__ ell,
               const double* __restrict__ kappa, const double* __restrict__ w,
               double* __restrict__ out) {
    __shared__ SegTile sh;
    const int i = blockIdx.x * kNT + threadIdx.x;
    const bool active = i < nodes.N;
    double x = 0, y = 0, ts = 0;
    int self = -1;
    if (active) {
        x = nodes.x[i];
        y = nodes.y[i];
        self = nodes.self_seg[i];
        ts = nodes.tstar[i];
    }
    double acc[3] = {0, 0, 0};
    for (int base = 0; base < segs.n; base += kNT) {
        __syncthreads();
        stage_segments(sh, segs, w, base);
        __syncthreads();
        if (!active) continue;
        const int m = min(kNT, segs.n - base);
        for (int t = 0; t < m; ++t) {
            const int j = base + t;
            if (j == self) {
                // acc holds -2 pi u; Ghat_self = (l - e1 ln e1 - e2 ln e2)/(2 pi)
                const double g2 = self_segment_2pi_G(ell[j], ts);
                const double inv_k = 1.0 / kappa[j];
                for (int c = 0; c < 3; ++c) acc[c] -= g2 * sh.w[c][t] * inv_k;
                continue;
            }
            double il, th;
            chord_log_theta<double>(sh.x0[t] - x, sh.y0[t] - y, sh.tx[t], sh.ty[t], sh.len[t],
                                    il, th);
            for (int c = 0; c < 3; ++c) acc[c] += il * sh.w[c][t] + th * sh.w[3 + c][t];
        }
    }
    if (active)
        for (int c = 0; c < 3; ++c) out[(size_t)c * nodes.N + i] = -acc[c] / kTwoPi;
}

__global__ void __launch_bounds__(kNT)
k_direct_targets(TargetGrid grid, int use_grid, const double* __restrict__ pts, int n_pts,
                 ChordsView segs, const double* __restrict__ w, int out_f64, void* out) {
    __shared__ SegTile sh;
    const int i = blockIdx.x * kNT + threadIdx.x;
    const int n = use_grid ? grid.W * grid.H : n_pts;
    const bool active = i < n;
    double x = 0, y = 0;
    if (active) {
        if (use_grid) {
            const int r = i / grid.W, k = i - r * grid.W;
            x = pixel_x(grid.cx, grid.w, grid.W, k);
            y = pixel_y(grid.cy, grid.h, grid.H, r);
        } else {
            x = pts[2 * (size_t)i];
            y = pts[2 * (size_t)i + 1];
        }
    }
    double acc[3] = {0, 0, 0};
    for (int base = 0; base < segs.n; base += kNT) {
        __syncthreads();
        stage_segments(sh, segs, w, base);
        __syncthreads();
        if (!active) continue;
        const int m = min(kNT, segs.n - base);
        for (int t = 0; t < m; ++t) {
            double il, th;
            chord_log_theta<double>(sh.x0[t] - x, sh.y0[t] - y, sh.tx[t], sh.ty[t], sh.len[t],
                                    il, th);
            for (int c = 0; c < 3; ++c) acc[c] += il * sh.w[c][t] + th * sh.w[3 + c][t];
        }
    }
    if (!active) return;
    for (int c = 0; c < 3; ++c) {
        const double u = -acc[c] / kTwoPi;
        if (out_f64)
            static_cast<double*>(out)[3 * (size_t)i + c] = u;
        else
            static_cast<float*>(out)[3 * (size_t)i + c] = (float)u;
    }
}

// ------------------------------------------------------------------ GMRES
// Fixed-order block reductions (no atomics): results do not depend on
// scheduling.
__device__ inline double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kNT / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    return red[0];
}

// Rows summed by one block of k_block_dots.
constexpr int kDotRows = 8192;

// dots[c k + j] = <V_j^c, w^c> in two steps: block (j, c, s) sums the rows
// [s R, (s + 1) R) into part[(c k + j) S + s] (S = gridDim.z), and
// k_dots_finish adds each dot's S partial sums in order, so the result does
// not depend on the order in which blocks run.
__global__ void __launch_bounds__(kNT)
k_block_dots(const double* __restrict__ V, const double* __restrict__ w, int N,
             double* __restrict__ part, int k) {
    __shared__ double red[kNT];
    const int j = blockIdx.x, c = blockIdx.y, sb = blockIdx.z;
    const double* v = V + ((size_t)j * 3 + c) * N;
    const double* ww = w + (size_t)c * N;
    const int hi = min(N, (sb + 1) * kDotRows);
    double acc = 0.0;
    for (int i = sb * kDotRows + threadIdx.x; i < hi; i += kNT) acc += v[i] * ww[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[((size_t)c * k + j) * gridDim.z + sb] = s;
}

__global__ void __launch_bounds__(kNT)
k_dots_finish(const double* __restrict__ part, int n, int S, double* __restrict__ dots) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int t = 0; t < S; ++t) s += part[(size_t)i * S + t];
    dots[i] = s;
}

// w[c] -= sum_j V_j^c h[c][j]: a workgroup takes kUpdRows rows, its
// kUpdSplit waves a quarter of the vectors each (more loads in flight than
// one thread per row over all vectors), and the quarters are added in order
// through LDS.
constexpr int kUpdRows = 64, kUpdSplit = kNT / kUpdRows;

__global__ void __launch_bounds__(kNT)
k_block_update(const double* __restrict__ V, int k, const double* __restrict__ h, int kcap,
               double* __restrict__ w, int N) {
    __shared__ double part[kUpdSplit][kUpdRows];
    const int r = threadIdx.x % kUpdRows, q = threadIdx.x / kUpdRows;
    const int i = blockIdx.x * kUpdRows + r;
    const int c = blockIdx.y;
    double acc = 0.0;
    if (i < N) {
        const int j1 = ((q + 1) * k) / kUpdSplit;
        for (int j = (q * k) / kUpdSplit; j < j1; ++j)
            acc += V[((size_t)j * 3 + c) * N + i] * h[(size_t)c * kcap + j];
    }
    part[q][r] = acc;
    __syncthreads();
    if (q == 0 && i < N) {
        double sum = part[0][r];
        for (int t = 1; t < kUpdSplit; ++t) sum += part[t][r];
        w[(size_t)c * N + i] -= sum;
    }
}

// Per-channel factors, passed by value (no copy to the device).
struct Scale3 {
    double a[3];
};

__global__ void __launch_bounds__(kNT)
k_scale3(const double* __restrict__ x, Scale3 alpha, double* __restrict__ y, int N) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    const int c = blockIdx.y;
    if (i < N) y[(size_t)c * N + i] = alpha.a[c] * x[(size_t)c * N + i];
}

// y[c] = x[c] / sqrt(n2[c]) (0 where n2[c] <= 0), the squared norms n2 on
// the device.
__global__ void __launch_bounds__(kNT)
k_scale3_norm(const double* __restrict__ x, const double* __restrict__ n2,
              double* __restrict__ y, int N) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= N) return;
    const double v = n2[c];
    const double a = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    y[(size_t)c * N + i] = a * x[(size_t)c * N + i];
}

__global__ void __launch_bounds__(kNT)
k_combine(const double* __restrict__ V, int k, const double* __restrict__ y, int kcap,
          double* __restrict__ x, int N) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= N) return;
    double acc = x[(size_t)c * N + i];
    for (int j = 0; j < k; ++j) acc += V[((size_t)j * 3 + c) * N + i] * y[(size_t)c * kcap + j];
    x[(size_t)c * N + i] = acc;
}

__global__ void __launch_bounds__(kNT)
k_axpby(int n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
        double* __restrict__ out) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i < n) out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ void __launch_bounds__(kNT) k_fill(int n, double v, double* __restrict__ out) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i < n) out[i] = v;
}

// v [3][N] split by a per-node flag: a = v where flag == 0, b = v where
// flag != 0 (zero elsewhere).
__global__ void __launch_bounds__(kNT)
k_mask_split(int N, const int* __restrict__ flag, const double* __restrict__ v,
             double* __restrict__ a, double* __restrict__ b) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i >= 3 * N) return;
    const bool f = flag[i % N] != 0;
    a[i] = f ? 0.0 : v[i];
    b[i] = f ? v[i] : 0.0;
}

// out0 = x where flag == 0 else y;  out1 = y where flag == 0 else x.
__global__ void __launch_bounds__(kNT)
k_mask_merge(int N, const int* __restrict__ flag, const double* __restrict__ x,
             const double* __restrict__ y, double* __restrict__ out0, double* __restrict__ out1) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i >= 3 * N) return;
    const bool f = flag[i % N] != 0;
    out0[i] = f ? y[i] : x[i];
    out1[i] = f ? x[i] : y[i];
}

__global__ void __launch_bounds__(kNT)
k_select(int N, const unsigned char* __restrict__ flag, const double* a, const double* b,
         double* out) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i >= 3 * N) return;
    out[i] = flag[i % N] ? a[i] : b[i];
}

inline unsigned blocks(long long n) { return (unsigned)((n + kNT - 1) / kNT); }

}  // namespace

void launch_chord_weights(int n, const int* seg, int s, int g, int N, const double* Pi,
                          const double* kappa, const double* sigma, const double* mu,
                          double* w_f64, float* w_f32, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_chord_weights, dim3(blocks(n)), dim3(kNT), 0, st, n, seg, s, g, N, Pi,
                       kappa, sigma, mu, w_f64, w_f32);
    DC_HIP(hipGetLastError());
}

void launch_direct_nodes(const NodesView& nodes, const ChordsView& segs, const double* ell,
                         const double* kappa, const double* w, double* out, hipStream_t st) {
    if (nodes.N <= 0) return;
    hipLaunchKernelGGL(k_direct_nodes, dim3(blocks(nodes.N)), dim3(kNT), 0, st, nodes, segs,
                       ell, kappa, w, out);
    DC_HIP(hipGetLastError());
}

void launch_direct_targets(const TargetGrid* grid, const double* pts, int n_pts,
                           const ChordsView& segs, const double* w, int out_f64, void* out,
                           hipStream_t st) {
    TargetGrid gg = grid ? *grid : TargetGrid{0, 0, 0, 0, 0, 0};
    const long long n = grid ? (long long)grid->W * grid->H : n_pts;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_direct_targets, dim3(blocks(n)), dim3(kNT), 0, st, gg, grid ? 1 : 0,
                       pts, n_pts, segs, w, out_f64, out);
    DC_HIP(hipGetLastError());
}

int block_dots_split(int N) { return std::max(1, (N + kDotRows - 1) / kDotRows); }

void launch_block_dots(const double* V, int k, const double* w, int N, double* dots,
                       double* part, hipStream_t st) {
    const int S = block_dots_split(N);
    hipLaunchKernelGGL(k_block_dots, dim3(k, 3, S), dim3(kNT), 0, st, V, w, N, part, k);
    DC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_dots_finish, dim3(blocks(3LL * k)), dim3(kNT), 0, st, part, 3 * k, S,
                       dots);
    DC_HIP(hipGetLastError());
}

void launch_block_update(const double* V, int k, const double* h, int kcap, double* w, int N,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_block_update, dim3((N + kUpdRows - 1) / kUpdRows, 3), dim3(kNT), 0, st,
                       V, k, h, kcap, w, N);
    DC_HIP(hipGetLastError());
}

void launch_scale3(const double* x, const double alpha[3], double* y, int N, hipStream_t st) {
    hipLaunchKernelGGL(k_scale3, dim3(blocks(N), 3), dim3(kNT), 0, st, x,
                       Scale3{{alpha[0], alpha[1], alpha[2]}}, y, N);
    DC_HIP(hipGetLastError());
}

void launch_scale3_by_norm(const double* x, const double* n2, double* y, int N,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_scale3_norm, dim3(blocks(N), 3), dim3(kNT), 0, st, x, n2, y, N);
    DC_HIP(hipGetLastError());
}

void launch_combine(const double* V, int k, const double* y, int kcap, double* x, int N,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_combine, dim3(blocks(N), 3), dim3(kNT), 0, st, V, k, y, kcap, x, N);
    DC_HIP(hipGetLastError());
}

void launch_axpby(int n, double a, const double* x, double b, const double* y, double* out,
                  hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(kNT), 0, st, n, a, x, b, y, out);
    DC_HIP(hipGetLastError());
}

void launch_mask_split(int N, const int* flag, const double* v, double* a, double* b,
                       hipStream_t st) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_mask_split, dim3(blocks(3LL * N)), dim3(kNT), 0, st, N, flag, v, a, b);
    DC_HIP(hipGetLastError());
}

void launch_mask_merge(int N, const int* flag, const double* x, const double* y, double* out0,
                       double* out1, hipStream_t st) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_mask_merge, dim3(blocks(3LL * N)), dim3(kNT), 0, st, N, flag, x, y,
                       out0, out1);
    DC_HIP(hipGetLastError());
}

void launch_select(int N, const unsigned char* flag, const double* a, const double* b,
                   double* out, hipStream_t st) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_select, dim3(blocks(3LL * N)), dim3(kNT), 0, st, N, flag, a, b, out);
    DC_HIP(hipGetLastError());
}

void launch_fill(int n, double v, double* out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(blocks(n)), dim3(kNT), 0, st, n, v, out);
    DC_HIP(hipGetLastError());
}

}  // namespace dc
