// Anti-aliased render (Sec. 8): pixel values as area-weighted averages
// where curves cross pixels.  The paper subdivides the quadtree cells that
// contain curves below the pixel size and sums the children's values
// weighted by area; here every pixel whose square meets a chord segment
// takes the mean of the representation at the centres of its aa x aa equal
// sub-cells (the same area-weighted sum over one level of aa x aa children),
// and every other pixel keeps its centre sample.  The sub-cell samples are
// rendered by the FMM as small viewports in one batched render.
#include <algorithm>
#include <cmath>
#include <vector>

#include "aa.h"

namespace dc {

namespace {

constexpr int kBlock = 16;  // pixels per side of the blocks edge pixels are grouped in

// Where a rendered sub-cell image of a block of edge pixels lives.
struct SubVp {
    long long off;  // first value of its image in the sample buffer
    int W;          // its width in samples
    int r0, k0;     // its first pixel row and column
};

struct AaItem {
    int r, k, sv, pad;
};

__global__ void __launch_bounds__(256)
k_aa_combine(int n, const AaItem* __restrict__ items, const SubVp* __restrict__ svs, int aa,
             const void* __restrict__ samples, int out_f64, void* __restrict__ out, int W) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const AaItem it = items[e];
    const SubVp sv = svs[it.sv];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < aa; ++j) {
        const long long row = (long long)(it.r - sv.r0) * aa + j;
        for (int i = 0; i < aa; ++i) {
            const long long col = (long long)(it.k - sv.k0) * aa + i;
            const long long at = (sv.off + row * sv.W + col) * 3;
            for (int ch = 0; ch < 3; ++ch)
                acc[ch] += out_f64 ? static_cast<const double*>(samples)[at + ch]
                                   : (double)static_cast<const float*>(samples)[at + ch];
        }
    }
    const double inv = 1.0 / ((double)aa * aa);
    const size_t o = ((size_t)it.r * W + it.k) * 3;
    for (int ch = 0; ch < 3; ++ch) {
        if (out_f64) static_cast<double*>(out)[o + ch] = acc[ch] * inv;
        else static_cast<float*>(out)[o + ch] = (float)(acc[ch] * inv);
    }
}

}  // namespace

// Does the closed segment a + t (b - a), t in [0, 1], meet the closed box
// [xa, xb] x [ya, yb]?  (Liang-Barsky clipping.)
bool segment_meets_box(double ax, double ay, double bx, double by, double xa, double xb,
                       double ya, double yb) {
#pragma clang fp contract(off)
    const double dx = bx - ax, dy = by - ay;
    const double p[4] = {-dx, dx, -dy, dy};
    const double q[4] = {ax - xa, xb - ax, ay - ya, yb - ay};
    double t0 = 0.0, t1 = 1.0;
    for (int m = 0; m < 4; ++m) {
        if (p[m] == 0.0) {
            if (q[m] < 0.0) return false;
            continue;
        }
        const double r = q[m] / p[m];
        if (p[m] < 0.0) t0 = std::max(t0, r);
        else t1 = std::min(t1, r);
        if (t0 > t1) return false;
    }
    return true;
}

void aa_edge_pixels(const Geometry& G, const dc_viewport& vp, std::vector<unsigned char>& mask) {
#pragma clang fp contract(off)
    const int W = vp.W, H = vp.H;
    mask.assign((size_t)W * H, 0);
    const double x0 = vp.cx - 0.5 * vp.width, top = vp.cy + 0.5 * vp.height;
    const double pw = vp.width / (double)W, ph = vp.height / (double)H;
    auto col_of = [&](double x) { return (long long)std::floor((x - x0) / pw); };
    auto row_of = [&](double y) { return (long long)std::floor((top - y) / ph); };
    for (int j = 0; j < G.S; ++j) {
        const double ax = G.seg_x0[j], ay = G.seg_y0[j], bx = G.seg_x1[j], by = G.seg_y1[j];
        // the viewport, widened by a pixel (a filter only; the pixel test below decides)
        if (!segment_meets_box(ax, ay, bx, by, x0 - pw, x0 + vp.width + pw,
                               top - vp.height - ph, top + ph))
            continue;
        const long long c0 = std::max(0LL, std::min(col_of(ax), col_of(bx)) - 1);
        const long long c1 = std::min((long long)W - 1, std::max(col_of(ax), col_of(bx)) + 1);
        for (long long k = c0; k <= c1; ++k) {
            const double xa = x0 + (double)k * pw, xb = x0 + (double)(k + 1) * pw;
            // rows the segment can reach inside this column's slab
            double ylo = std::min(ay, by), yhi = std::max(ay, by);
            if (bx != ax) {
                // (the slab widened by 1e-9 pixel: it only proposes rows)
                const double ea = xa - 1e-9 * pw, eb = xb + 1e-9 * pw;
                const double ta = (ea - ax) / (bx - ax), tb = (eb - ax) / (bx - ax);
                const double t0 = std::max(0.0, std::min(ta, tb)), t1 = std::min(1.0, std::max(ta, tb));
                if (t0 > t1) continue;
                const double y0v = ay + t0 * (by - ay), y1v = ay + t1 * (by - ay);
                ylo = std::min(y0v, y1v);
                yhi = std::max(y0v, y1v);
            }
            const long long r0 = std::max(0LL, row_of(yhi) - 1);
            const long long r1 = std::min((long long)H - 1, row_of(ylo) + 1);
            for (long long r = r0; r <= r1; ++r) {
                unsigned char& m = mask[(size_t)r * W + k];
                if (m) continue;
                const double yb = top - (double)r * ph, ya = top - (double)(r + 1) * ph;
                if (segment_meets_box(ax, ay, bx, by, xa, xb, ya, yb)) m = 1;
            }
        }
    }
}

void render_aa(dc_scene_s& s, const dc_viewport& vp, const dc_eval_opts& o, int aa,
               int out_dtype, void* out, dc_aa_report* rep, hipStream_t st) {
    // centre samples everywhere
    fmm_render(s, vp, o, out_dtype, out, st);
    std::vector<unsigned char> mask;
    aa_edge_pixels(s.geo, vp, mask);
    // edge pixels grouped by blocks; each block's bounding rectangle of edge
    // pixels is rendered at aa x aa samples per pixel
    const int W = vp.W, H = vp.H;
    const int bw = (W + kBlock - 1) / kBlock, bh = (H + kBlock - 1) / kBlock;
    const double x0 = vp.cx - 0.5 * vp.width, top = vp.cy + 0.5 * vp.height;
    const double pw = vp.width / (double)W, ph = vp.height / (double)H;
    std::vector<dc_viewport> sub;
    std::vector<SubVp> svs;
    std::vector<AaItem> items;
    long long samples = 0;
    for (int by = 0; by < bh; ++by)
        for (int bx = 0; bx < bw; ++bx) {
            int r0 = H, r1 = -1, k0 = W, k1 = -1;
            for (int r = by * kBlock; r < std::min(H, (by + 1) * kBlock); ++r)
                for (int k = bx * kBlock; k < std::min(W, (bx + 1) * kBlock); ++k)
                    if (mask[(size_t)r * W + k]) {
                        r0 = std::min(r0, r);
                        r1 = std::max(r1, r);
                        k0 = std::min(k0, k);
                        k1 = std::max(k1, k);
                    }
            if (r1 < 0) continue;
            const int nc = k1 - k0 + 1, nr = r1 - r0 + 1;
            dc_viewport v;
            v.width = nc * pw;
            v.height = nr * ph;
            v.cx = x0 + (double)k0 * pw + 0.5 * v.width;
            v.cy = top - (double)r0 * ph - 0.5 * v.height;
            v.W = nc * aa;
            v.H = nr * aa;
            const int sv = (int)sub.size();
            sub.push_back(v);
            svs.push_back(SubVp{samples, v.W, r0, k0});
            samples += (long long)v.W * v.H;
            for (int r = r0; r <= r1; ++r)
                for (int k = k0; k <= k1; ++k)
                    if (mask[(size_t)r * W + k]) items.push_back(AaItem{r, k, sv, 0});
        }
    if (rep) {
        rep->aa_pixels = (long long)items.size();
        rep->blocks = (int)sub.size();
        rep->samples = samples;
    }
    if (items.empty()) {
        DC_HIP(hipStreamSynchronize(st));
        return;
    }
    const size_t esz = out_dtype == DC_OUT_F64 ? 8 : 4;
    DevBuf<char> sbuf;
    DevBuf<SubVp> d_svs;
    DevBuf<AaItem> d_items;
    // the device buffers above are released on return, after the stream's
    // work has finished (also when a launch below throws)
    struct SyncOnExit {
        hipStream_t st;
        ~SyncOnExit() { (void)hipStreamSynchronize(st); }
    } sync_on_exit{st};
    sbuf.alloc((size_t)samples * 3 * esz);
    std::vector<void*> outs(sub.size());
    for (size_t v = 0; v < sub.size(); ++v) outs[v] = sbuf.p + (size_t)svs[v].off * 3 * esz;
    fmm_render_batch(s, sub.data(), (int)sub.size(), o, out_dtype, outs.data(), st);
    d_svs.alloc(svs.size());
    d_items.alloc(items.size());
    DC_HIP(hipMemcpyAsync(d_svs.p, svs.data(), svs.size() * sizeof(SubVp), hipMemcpyHostToDevice,
                          st));
    DC_HIP(hipMemcpyAsync(d_items.p, items.data(), items.size() * sizeof(AaItem),
                          hipMemcpyHostToDevice, st));
    const int n = (int)items.size();
    hipLaunchKernelGGL(k_aa_combine, dim3((n + 255) / 256), dim3(256), 0, st, n, d_items.p,
                       d_svs.p, aa, sbuf.p, out_dtype == DC_OUT_F64 ? 1 : 0, out, W);
    DC_HIP(hipGetLastError());
    DC_HIP(hipStreamSynchronize(st));
}

}  // namespace dc
