// Block-Jacobi preconditioner for the hybrid collocation system: the
// diagonal block of every curve, A_cc[i][i'] = sum_{j in panel(i')} Ghat_ij
// Pi[j][i'] with the singular self-segment rule (the matrix of Eq.
// hybrid_sys restricted to one curve), inverted in place on the device.
// GMRES solves A M^-1 y = b, x = M^-1 y with M = blockdiag(A_cc): the linear
// system and its solution are unchanged; a curve whose own geometry makes
// the first-kind system ill-conditioned (a near-cusp folds two branches onto
// each other) no longer stalls the iteration.
#include "kernels.h"

namespace dc {

namespace {

constexpr int kNT = 256;

// One thread per (node i, panel p' of the node's curve): 16 entries of row i.
__global__ void __launch_bounds__(kNT)
k_curve_blocks(int N, int g, int s, const double* __restrict__ nx,
               const double* __restrict__ ny, const int* __restrict__ self_seg,
               const double* __restrict__ tstar, ChordsView segs,
               const double* __restrict__ ell, const double* __restrict__ kappa,
               const double* __restrict__ Pi, BlocksView bv, double* __restrict__ D) {
    const long long t = (long long)blockIdx.x * kNT + threadIdx.x;
    const int mp = bv.max_panels;
    if (t >= (long long)N * mp) return;
    const int i = (int)(t / mp), pp = (int)(t - (long long)i * mp);
    const int b = bv.panel_blk[i / g];
    const int node0 = bv.node0[b], n = bv.n[b];
    if (pp >= n / g) return;
    const int iloc = i - node0;
    const int panel = node0 / g + pp;
    const double x = nx[i], y = ny[i];
    const int self = self_seg[i];
    double acc[64];
    for (int m = 0; m < g; ++m) acc[m] = 0.0;
    for (int jj = 0; jj < s; ++jj) {
        const int j = panel * s + jj;
        double G;
        if (j == self) {
            G = self_segment_2pi_G(ell[j], tstar[i]) / kTwoPi;
        } else {
            double il, th;
            chord_log_theta<double>(segs.x0[j] - x, segs.y0[j] - y, segs.tx[j], segs.ty[j],
                                    segs.len[j], il, th);
            G = -kappa[j] * il / kTwoPi;
        }
        const double* pr = Pi + (size_t)jj * g;
        for (int m = 0; m < g; ++m) acc[m] += G * pr[m];
    }
    double* row = D + bv.doff[b] + (size_t)iloc * n + (size_t)pp * g;
    for (int m = 0; m < g; ++m) row[m] = acc[m];
}

// Gauss-Jordan with partial pivoting, one block of at most 512 rows per
// workgroup of kGJ threads: kGJRows rows at a time, kGJCols consecutive
// columns per row (a wave reads 512 contiguous bytes of one row).
constexpr int kGJ = 512, kGJCols = 64, kGJRows = kGJ / kGJCols;

__global__ void __launch_bounds__(kGJ)
k_gauss_jordan(BlocksView bv, double* __restrict__ D, int* __restrict__ perm_all,
               int* __restrict__ singular) {
    __shared__ double sval[kGJ];
    __shared__ int sidx[kGJ];
    __shared__ double rowk[512], colk[512];
    const int n = bv.n[blockIdx.x];
    double* a = D + bv.doff[blockIdx.x];
    int* perm = perm_all + bv.node0[blockIdx.x];
    const int tid = threadIdx.x;
    const int ty = tid / kGJCols, tx = tid - ty * kGJCols;
    for (int k = 0; k < n; ++k) {
        // pivot: largest |a[i][k]|, i >= k (first index on ties)
        double best = -1.0;
        int bi = k;
        for (int i = k + tid; i < n; i += kGJ) {
            const double v = fabs(a[(size_t)i * n + k]);
            if (v > best) { best = v; bi = i; }
        }
        sval[tid] = best;
        sidx[tid] = bi;
        __syncthreads();
        for (int st = kGJ / 2; st > 0; st >>= 1) {
            if (tid < st) {
                const double o = sval[tid + st];
                const int oi = sidx[tid + st];
                if (o > sval[tid] || (o == sval[tid] && oi < sidx[tid])) {
                    sval[tid] = o;
                    sidx[tid] = oi;
                }
            }
            __syncthreads();
        }
        const int pr = sidx[0];
        const double pv = a[(size_t)pr * n + k];
        if (tid == 0) {
            perm[k] = pr;
            if (pv == 0.0) singular[0] = 1;
        }
        __syncthreads();
        // swap rows k and pr, then scale row k by 1/pivot (a[k][k] := 1 first)
        const double inv = pv != 0.0 ? 1.0 / pv : 0.0;
        // column k of the other rows, read before anyone changes it (after the
        // swap row pr holds the old row k)
        for (int i = tid; i < n; i += kGJ)
            colk[i] = (i == pr) ? a[(size_t)k * n + k] : a[(size_t)i * n + k];
        __syncthreads();
        for (int j = tid; j < n; j += kGJ) {
            double vk = a[(size_t)k * n + j], vp = a[(size_t)pr * n + j];
            if (pr != k) {
                a[(size_t)pr * n + j] = vk;
                vk = vp;
            }
            vk = (j == k) ? inv : vk * inv;
            a[(size_t)k * n + j] = vk;
            rowk[j] = vk;
        }
        __syncthreads();
        // eliminate column k from every other row (a[i][k] := 0 first)
        for (int i = ty; i < n; i += kGJRows) {
            if (i == k) continue;
            const double f = colk[i];
            if (f == 0.0) continue;
            double* ai = a + (size_t)i * n;
            for (int j = tx; j < n; j += kGJCols) {
                if (j == k)
                    ai[j] = -f * rowk[k];
                else
                    ai[j] -= f * rowk[j];
            }
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges, in reverse order
    for (int k = n - 1; k >= 0; --k) {
        const int pr = perm[k];
        if (pr == k) continue;
        for (int i = tid; i < n; i += kGJ) {
            const double t = a[(size_t)i * n + k];
            a[(size_t)i * n + k] = a[(size_t)i * n + pr];
            a[(size_t)i * n + pr] = t;
        }
        __syncthreads();
    }
}

// y[ch][i] = sum_j Dinv[c][iloc][j] x[ch][c n + j]
// Each inverted block transposed in place (one block per workgroup), so
// that k_block_apply's threads, one per row, read consecutive addresses.
__global__ void __launch_bounds__(kNT)
k_transpose_blocks(BlocksView bv, double* __restrict__ D) {
    const int n = bv.n[blockIdx.x];
    double* a = D + bv.doff[blockIdx.x];
    for (long long q = threadIdx.x; q < (long long)n * n; q += kNT) {
        const int i = (int)(q / n), j = (int)(q - (long long)i * n);
        if (i < j) {
            const double t = a[(size_t)i * n + j];
            a[(size_t)i * n + j] = a[(size_t)j * n + i];
            a[(size_t)j * n + i] = t;
        }
    }
}

// y[ch] = blockdiag(Dinv) x[ch] for the three channels: a workgroup takes
// 64 rows, its four waves a quarter of each row's block each, and the
// quarters are added through LDS.  DinvT holds each block transposed
// (column j of the block's inverse at DinvT + doff + j n), so a wave's
// lanes, one per row, read consecutive addresses.
constexpr int kApplyRows = 64, kApplySplit = kNT / kApplyRows;

__global__ void __launch_bounds__(kNT)
k_block_apply(int N, int g, BlocksView bv, const double* __restrict__ DinvT,
              const double* __restrict__ x, double* __restrict__ y) {
    __shared__ double part[3][kApplySplit][kApplyRows];
    const int r = threadIdx.x % kApplyRows, c = threadIdx.x / kApplyRows;
    const int i = blockIdx.x * kApplyRows + r;
    double acc[3] = {0.0, 0.0, 0.0};
    if (i < N) {
        const int b = bv.panel_blk[i / g];
        const int node0 = bv.node0[b], n = bv.n[b];
        const double* col = DinvT + bv.doff[b] + (i - node0);
        const double* x0 = x + (size_t)node0;
        const int j0 = (c * n) / kApplySplit, j1 = ((c + 1) * n) / kApplySplit;
        for (int j = j0; j < j1; ++j) {
            const double d = col[(size_t)j * n];
            for (int ch = 0; ch < 3; ++ch) acc[ch] += d * x0[(size_t)ch * N + j];
        }
    }
    for (int ch = 0; ch < 3; ++ch) part[ch][c][r] = acc[ch];
    __syncthreads();
    if (c == 0 && i < N)
        for (int ch = 0; ch < 3; ++ch) {
            double v = part[ch][0][r];
            for (int q = 1; q < kApplySplit; ++q) v += part[ch][q][r];
            y[(size_t)ch * N + i] = v;
        }
}

}  // namespace

void launch_curve_blocks(const NodesView& nodes, int g, int s, const ChordsView& segs,
                         const double* ell, const double* kappa, const double* Pi,
                         const BlocksView& bv, double* D, hipStream_t st) {
    DC_REQUIRE(g <= 64, "block preconditioner supports at most 64 GL nodes per panel");
    const long long threads = (long long)nodes.N * bv.max_panels;
    hipLaunchKernelGGL(k_curve_blocks, dim3((unsigned)((threads + kNT - 1) / kNT)), dim3(kNT), 0,
                       st, nodes.N, g, s, nodes.x, nodes.y, nodes.self_seg, nodes.tstar, segs,
                       ell, kappa, Pi, bv, D);
    DC_HIP(hipGetLastError());
}

void launch_invert_blocks(const BlocksView& bv, double* D, int* perm, int* singular,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_gauss_jordan, dim3(bv.n_blocks), dim3(kGJ), 0, st, bv, D, perm,
                       singular);
    DC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_transpose_blocks, dim3(bv.n_blocks), dim3(kNT), 0, st, bv, D);
    DC_HIP(hipGetLastError());
}

void launch_block_apply(int N, int g, const BlocksView& bv, const double* Dinv, const double* x,
                        double* y, hipStream_t st) {
    hipLaunchKernelGGL(k_block_apply, dim3((N + kApplyRows - 1) / kApplyRows), dim3(kNT), 0, st,
                       N, g, bv, Dinv, x, y);
    DC_HIP(hipGetLastError());
}

}  // namespace dc
