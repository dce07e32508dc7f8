// Fast multipole evaluation of the hybrid representation (App. E, Alg. 8).
//
// Expansion basis (App. E.1): I_k(z) = z^k / k!, O_k(z) = (k-1)!/z^k,
// O_0 = -log z.  Coefficients are stored box-scaled so that no factorial or
// power of the box size appears in FP32:
//   multipole  Mt_k = M_k k! / r^k,   local  Lt_k = L_k r^k / k!,
// r = half-width of the box.  Single and double layer share one coefficient
// vector per colour channel (the double layer differs only in the source
// terms, Sec. 6.3), so one pass evaluates u = FMM_G(Pi sigma) + FMM_F(Pi mu).
//
// Targets live in their own tree on the same canonical grid as the source
// quadtree.  For every target box a we keep its near set N(a): for each of
// the 3x3 neighbouring positions at a's level, the deepest source box at a
// level <= level(a) covering it.  From N(parent(a)):
//   - children (at level(a)) of internal boxes that do not touch a form the
//     interaction list of a (incoming-from-outgoing, Eq. i-f-o);
//   - source leaves coarser than a that do not touch a form its bigger
//     separated list (incoming-from-source, App. E.10/E.11);
//   - the rest is N(a).
// At a target leaf the near set is descended: source leaves touching it are
// summed directly (target-from-source, App. D), non-touching children of
// touching boxes form the smaller separated list (target-from-outgoing,
// Eq. t-f-o).  When the target tree is the source tree (the solve) this is
// exactly Alg. 8; for a render the target tree is the complete quadtree over
// the viewport down to pixel tiles.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstddef>
#include <cstring>
#include <string>

#include "scene.h"

// Device scratch of dc_render_noalloc (DC_NOALLOC_SCRATCH_BYTES per GPU,
// held until the process ends).  In host code this name is only a stand-in
// for the symbol: host code uses the address hipGetSymbolAddress returns
// for the current device (noalloc_scratch_ptr), never the name itself.
static __device__ __align__(256) char dc_noalloc_scratch[DC_NOALLOC_SCRATCH_BYTES];

namespace dc {

namespace {

constexpr int kWave = 64;
constexpr int kUCap = 128;   // near leaves per round
constexpr int kWCap = 256;   // smaller-separated boxes per round
constexpr int kSCap = 256;   // traversal stack (>= 9 + 4 * max depth)
// work counters (dc_work_counts order)
enum { kStatP2P = 0, kStatP2P64, kStatM2P, kStatL2P, kStatM2L, kStatP2L, kStatP2L64, kStatL2L,
       kStatLeaf, kNStat };

// 1/n for n < 128 (entry 0 unused): the coefficient recurrences of the
// translation operators multiply by these instead of dividing (an FP64
// division is a long instruction sequence on this hardware).
struct RecipTable {
    double v[128];
    constexpr RecipTable() : v() {
        for (int i = 1; i < 128; ++i) v[i] = 1.0 / i;
    }
};
__constant__ RecipTable kRecip = RecipTable();

template <typename T>
__device__ inline T recip(int n) {
    return (T)kRecip.v[n];
}

struct TreeView {
    int n_cells;
    double X0, Y0, side;
    const int *lvl, *child, *parent, *pbeg, *pend, *npc, *nbeg, *nend, *node_perm;
    const long long *ix, *iy;
    const int* cmask;  // bit q: child q holds pieces
};

struct PieceView {
    int n;
    const double *x0, *y0, *x1, *y1, *tx, *ty, *len;
    const int* seg;
    const double* w64;
    const float* w32;
    const int* heavy;   // FP32 path: piece evaluated in FP64 (large |q| * length)
};

__device__ inline double half_width(const TreeView& t, int l) { return ldexp(t.side, -(l + 1)); }

__device__ inline void center_of(const TreeView& t, int l, long long i, long long j, double& cx,
                                 double& cy) {
    const double h = ldexp(t.side, -(l + 1));
    cx = t.X0 + (double)(2 * i + 1) * h;
    cy = t.Y0 + (double)(2 * j + 1) * h;
}

// Does source box c (any level <= l... or finer) touch target box (l, ti, tj)?
// Boxes touch when their closed squares intersect (edges or corners).
__device__ inline bool touches_at(int lc, long long cx, long long cy, int l, long long ti,
                                  long long tj) {
    if (lc <= l) {
        const int s = l - lc;
        const long long lo_x = cx << s, hi_x = ((cx + 1) << s) - 1;
        const long long lo_y = cy << s, hi_y = ((cy + 1) << s) - 1;
        return ti >= lo_x - 1 && ti <= hi_x + 1 && tj >= lo_y - 1 && tj <= hi_y + 1;
    }
    const int s = lc - l;
    const long long lo_x = ti << s, hi_x = ((ti + 1) << s) - 1;
    const long long lo_y = tj << s, hi_y = ((tj + 1) << s) - 1;
    return cx >= lo_x - 1 && cx <= hi_x + 1 && cy >= lo_y - 1 && cy <= hi_y + 1;
}
__device__ inline bool touches(const TreeView& t, int c, int l, long long ti, long long tj) {
    return touches_at(t.lvl[c], t.ix[c], t.iy[c], l, ti, tj);
}

template <typename T>
__device__ inline cpx<T> to_c(double re, double im) {
    return {(T)re, (T)im};
}

template <typename T>
__device__ inline const T* weights(const PieceView& pv);
template <>
__device__ inline const double* weights<double>(const PieceView& pv) { return pv.w64; }
template <>
__device__ inline const float* weights<float>(const PieceView& pv) { return pv.w32; }

// FP32 arctangent: atan(t) ~ t P(t^2) on [0, 1] (coefficients from a minimax
// fit by Lawson's iteration, fit_atan_poly.py; max error 7e-7), with the
// usual octant reduction.
__device__ inline float atan2_poly(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.f ? mn * __builtin_amdgcn_rcpf(mx) : 0.f;
    const float u = t * t;
    float q = 8.00683815e-03f;
    q = q * u - 3.74428146e-02f;
    q = q * u + 8.43539238e-02f;
    q = q * u - 1.35121688e-01f;
    q = q * u + 1.98873192e-01f;
    q = q * u - 3.33270133e-01f;
    q = q * u + 9.99999404e-01f;
    float r = t * q;
    r = ay > ax ? 1.57079632679f - r : r;
    r = x < 0.f ? 3.14159265359f - r : r;
    return copysignf(r, y);
}

// The same without the guards for zero arguments, for the render's hot
// loop: a zero argument occurs only for a target at a chord end point,
// a near-singular pair whose result is discarded there.
__device__ inline float atan2_poly_nz(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float t = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay));
    const float u = t * t;
    float q = 8.00683815e-03f;
    q = q * u - 3.74428146e-02f;
    q = q * u + 8.43539238e-02f;
    q = q * u - 1.35121688e-01f;
    q = q * u + 1.98873192e-01f;
    q = q * u - 3.33270133e-01f;
    q = q * u + 9.99999404e-01f;
    float r = t * q;
    r = ay > ax ? 1.57079632679f - r : r;
    r = x < 0.f ? 3.14159265359f - r : r;
    return copysignf(r, y);
}

// Natural logarithm from the hardware log2 (v_log_f32).
__device__ inline float fast_ln(float x) {
    return __builtin_amdgcn_logf(x) * 0.69314718056f;
}

// log(1 + x) for x in [-1, 0] to a few ulps from one hardware logarithm:
// with u = 1 + x rounded, log(u) * x / (u - 1) cancels the rounding of u
// (the classical correction for log1p from a plain log).
__device__ inline float fast_log1p(float x) {
    const float u = 1.0f + x;
    const float d = u - 1.0f;
    const float v = fast_ln(fmaxf(u, 1e-37f)) * (x * __builtin_amdgcn_rcpf(d));
    return d == 0.0f ? x : v;  // select, no branch
}

// FP32 chord integral for a pair that is neither near-singular nor heavy,
// in the stable form of chord_log_theta (log of the farther endpoint plus a
// log1p of the ratio), so the rounding error scales with the chord length,
// not with the distance to the target.
__device__ inline void chord_fast(float xi1, float h, float xi2, float la, float& il,
                                  float& th) {
    const float r1 = xi1 * xi1 + h * h;
    const float r2 = xi2 * xi2 + h * h;
    th = atan2_poly(h * la, h * h + xi1 * xi2);
    const float sm = la * (xi1 + xi2);  // r2^2 - r1^2
    const bool one = r1 >= r2;
    const float big = fmaxf(one ? r1 : r2, 1e-37f);
    const float xo = one ? xi2 : -xi1;
    const float arg = (one ? sm : -sm) * __builtin_amdgcn_rcpf(big);
    const float l1p = fast_log1p(arg);
    const float tail = xo == 0.f ? 0.f : xo * 0.5f * l1p;
    il = la * 0.5f * fast_ln(big) + tail - la + h * th;
}

// chord_fast without its guards (see atan2_poly_nz): valid for pairs that
// are neither near-singular nor heavy; other pairs may yield inf or NaN and
// must be discarded by the caller.
__device__ inline void chord_fast_nz(float xi1, float h, float xi2, float la, float& il,
                                     float& th) {
    const float hh = h * h;
    const float r1 = xi1 * xi1 + hh;
    const float r2 = xi2 * xi2 + hh;
    th = atan2_poly_nz(h * la, hh + xi1 * xi2);
    const float sm = la * (xi1 + xi2);  // r2^2 - r1^2
    const bool one = r1 >= r2;
    const float big = one ? r1 : r2;
    const float xo = one ? xi2 : -xi1;
    const float arg = (one ? sm : -sm) * __builtin_amdgcn_rcpf(big);
    const float u = 1.0f + arg;
    const float d = u - 1.0f;
    const float l1p = d == 0.0f ? arg : fast_ln(u) * (arg * __builtin_amdgcn_rcpf(d));
    il = la * 0.5f * fast_ln(big) + xo * 0.5f * l1p - la + h * th;
}

// ------------------------------------------------------------------ upward
// Outgoing-from-source on every leaf (App. E.8, E.9), lane k = coefficient:
//   Mt_k += r wbar qs (B^{k+1} - A^{k+1})/(k+1) + i qm (B^k - A^k),
// A, B = piece end points relative to the box centre in units of r,
// wbar = conjugate unit tangent, qs = kappa sigma_bar, qm = kappa mu_bar
// (the left normal nu = i w makes nu wbar = i).
// G = 64 / (p + 1) groups of p + 1 lanes: group g takes the leaf's pieces
// g, g + G, ...; group 0 adds the others' sums in group order.
//
// The factors of qs and qm depend on the geometry alone.  Repeated
// applications of the operator (GMRES) store them once per piece and order
// (the P2M part of the paper's precomputed per-segment operators, Sec. 6.4)
// and read them instead of raising the end points to the k-th power: the
// same values, summed in the same order.  Mode: kP2MEval computes them,
// kP2MFill only writes them to tab [piece][k][ds, dm], kP2MRead reads them.
enum { kP2MEval = 0, kP2MFill = 1, kP2MRead = 2 };

template <typename T>
__device__ inline void p2m_factors(const PieceView& pv, int e, double cx, double cy, double inv_r,
                                   T rk, int k, cpx<T>& ds, cpx<T>& dm) {
    const cpx<T> A = to_c<T>((pv.x0[e] - cx) * inv_r, (pv.y0[e] - cy) * inv_r);
    const cpx<T> B = to_c<T>((pv.x1[e] - cx) * inv_r, (pv.y1[e] - cy) * inv_r);
    const cpx<T> wbar = {(T)pv.tx[e], (T)(-pv.ty[e])};
    const cpx<T> Ak = cpow(A, k), Bk = cpow(B, k);
    ds = cmul(cscale(csub(cmul(Bk, B), cmul(Ak, A)), rk), wbar);
    const cpx<T> dk = csub(Bk, Ak);
    dm = {-dk.im, dk.re};
}

template <typename T, int Mode = kP2MEval>
__global__ void __launch_bounds__(kWave)
k_p2m(TreeView tv, PieceView pv, int p, cpx<T>* __restrict__ M, cpx<T>* __restrict__ tab) {
    __shared__ cpx<T> red[kWave][3];
    const int c = blockIdx.x;
    if (tv.child[c] >= 0) return;
    const int P1 = p + 1, G = kWave / P1;
    const int g = threadIdx.x / P1, k = threadIdx.x - g * P1;
    const int l = tv.lvl[c];
    const double r = half_width(tv, l);
    double cx, cy;
    center_of(tv, l, tv.ix[c], tv.iy[c], cx, cy);
    const double inv_r = 1.0 / r;
    const T* w = weights<T>(pv);
    cpx<T> acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    const T rk = (T)(r / (k + 1));
    const int e1 = g < G ? tv.pend[c] : 0;
    for (int e = tv.pbeg[c] + g; e < e1; e += G) {
        cpx<T> ds, dm;
        if constexpr (Mode == kP2MRead) {
            ds = tab[((size_t)e * P1 + k) * 2];
            dm = tab[((size_t)e * P1 + k) * 2 + 1];
        } else {
            p2m_factors<T>(pv, e, cx, cy, inv_r, rk, k, ds, dm);
        }
        if constexpr (Mode == kP2MFill) {
            tab[((size_t)e * P1 + k) * 2] = ds;
            tab[((size_t)e * P1 + k) * 2 + 1] = dm;
            continue;
        }
        for (int ch = 0; ch < 3; ++ch) {
            const T qs = w[(size_t)ch * pv.n + e], qm = w[(size_t)(3 + ch) * pv.n + e];
            acc[ch] = cadd(acc[ch], cadd(cscale(ds, qs), cscale(dm, qm)));
        }
    }
    if constexpr (Mode == kP2MFill) return;
    if (g < G)
        for (int ch = 0; ch < 3; ++ch) red[threadIdx.x][ch] = acc[ch];
    __syncthreads();
    if (g != 0) return;
    for (int g2 = 1; g2 < G; ++g2)
        for (int ch = 0; ch < 3; ++ch) acc[ch] = cadd(acc[ch], red[g2 * P1 + k][ch]);
    cpx<T>* out = M + ((size_t)c * P1 + k) * 3;
    for (int ch = 0; ch < 3; ++ch) out[ch] = acc[ch];
}

// Outgoing-from-outgoing (Eq. o-f-o) in scaled form, child quadrant q:
//   Mt'_k = sum_{l<=k} C(k,l) z0^{k-l} 2^{-l} Mt_l,  z0 = (c_child - c)/r'.
// One cell per wave: its four children's expansions are staged in LDS by
// one round of independent loads; G = min(4, 64 / (p + 1)) groups of p + 1
// lanes (lane k = coefficient k) translate children g, g + G, ..., so a
// lane's chain of dependent multiply-adds covers one or two children
// instead of four, and group 0 adds the groups' sums in group order.
template <typename T>
__global__ void __launch_bounds__(kWave)
k_m2m(TreeView tv, int first, int n, int p, cpx<T>* __restrict__ M) {
    __shared__ cpx<T> cm[4 * 3 * kWave];
    const int lane = threadIdx.x, P1 = p + 1, span = 3 * P1;
    const int G = min(4, kWave / P1);
    const int g = lane / P1, k = lane - g * P1;
    const int c = first + (int)blockIdx.x;
    // the children and the mask of those holding pieces, in one round
    const int c0 = tv.child[c];
    const int held = tv.cmask[c];
    if (c0 < 0 || (int)blockIdx.x >= n) return;
    for (int i = lane; i < 4 * span; i += kWave) {
        const int q = i / span;
        if ((held >> q) & 1) cm[i] = M[(size_t)(c0 + q) * span + (i - q * span)];
    }
    __syncthreads();
    cpx<T> acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    if (g < G)
        for (int q = g; q < 4; q += G) {
            if (!((held >> q) & 1)) continue;
            const cpx<T> z0 = {(T)((q & 1) ? 0.5 : -0.5), (T)((q >> 1) ? 0.5 : -0.5)};
            const cpx<T>* cs = cm + q * span;
            cpx<T> pw = {1, 0};
            T binom = 1, sc = (T)ldexp(1.0, -k);
            // the loop counter j = k - l is the same in every lane, so the
            // reciprocals are read at one address per wave
            for (int j = 0; j <= k; ++j) {
                const int l = k - j;
                const cpx<T> f = cscale(pw, binom * sc);
                for (int ch = 0; ch < 3; ++ch) acc[ch] = cadd(acc[ch], cmul(f, cs[l * 3 + ch]));
                binom = binom * (T)l * recip<T>(j + 1);
                sc *= (T)2;
                pw = cmul(pw, z0);
            }
        }
    // the groups' sums, through the staging area once every group is done
    // reading it
    __syncthreads();
    if (g > 0 && g < G)
        for (int ch = 0; ch < 3; ++ch) cm[(g - 1) * span + k * 3 + ch] = acc[ch];
    __syncthreads();
    if (g != 0) return;
    for (int g2 = 1; g2 < G; ++g2)
        for (int ch = 0; ch < 3; ++ch) acc[ch] = cadd(acc[ch], cm[(g2 - 1) * span + k * 3 + ch]);
    cpx<T>* out = M + ((size_t)c * P1 + k) * 3;
    for (int ch = 0; ch < 3; ++ch) out[ch] = acc[ch];
}

// ---------------------------------------------------------------- downward
// Largest entry with first_block <= b (entries sorted by first_block).
template <typename E>
__device__ inline const E& find_entry(const E* e, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (e[mid].first_block <= b) lo = mid; else hi = mid - 1;
    }
    return e[lo];
}

struct DownLevel {
    int solve;             // 1: target boxes are the source boxes of level l
    int l;
    int first;             // solve: first box of level l
    const VpLevel* vl;     // render: one entry per viewport that has level l
    int nvl;
    unsigned long long* stats;  // optional work counters (see kStat*)
};

// Incoming-from-outgoing (Eq. i-f-o), scaled:
//   Lt_k += sum_m T[o][k][m] Mt_m,  T[o][k][m] = (-1)^k c(k,m) w^{k+m},
//   c(k,m) = (k+m-1)!/(k! m!),  w = r / (c_target - c_source),
// and for k = m = 0 the term -log(c_target - c_source) Mt_0.  With source
// and target boxes of one level, w and the log's argument depend only on
// the offset (dx, dy) of the source box in box widths, so T is tabulated
// once per order for the 7 x 7 offsets (m2l_table); the kernel adds the
// level part -log(2r) Mt_0 of the k = 0 term.
// Layout: [o][k][m] complex, o = (dy + 3) * 7 + (dx + 3).

// Incoming-from-source (App. E.10, E.11), scaled.  For a piece with ends
// A, B relative to the box centre in units of r, zA = 1/A, zB = 1/B and
// Lam = Log(B/A) (continuous branch: a chord seen from a point off its line
// subtends less than pi), the contribution to Lt_k is
//   k = 0: -qs [|a| (log r + log A) + wbar r B Lam - |a|]  - i qm Lam
//   k = 1:  qs wbar r Lam                               + i qm (zB - zA)
//   k > 1:  qs wbar r (zA^{k-1} - zB^{k-1})/(k(k-1))    + i qm (zB^k - zA^k)/k
template <typename T>
__device__ inline T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Per-piece data of the incoming-from-source pass, one piece per lane.
// FP32 P2L (FP32 path) for boxes whose pieces all have max|q| length below this
constexpr double kP2LFloat = 0.05;

template <typename T>
struct P2LStage {
    T zAr[kWave], zAi[kWave], zBr[kWave], zBi[kWave];  // 1/A, 1/B
    T wr[kWave], wi[kWave];                             // wbar
    T qs[3][kWave], qm[3][kWave];
};

// Downward pass at one level, one wave per target box: near set from the
// parent's, incoming-from-incoming (L2L) from the parent, incoming-from-
// outgoing (M2L) over the interaction list and incoming-from-source (P2L)
// over the pieces of coarser separated leaves.  Lane layout: ngrp groups of
// p+1 lanes; lane k of a group owns coefficient k.  M2L entries and P2L
// pieces are dealt round-robin to the groups, whose sums are reduced into
// group 0 at the end.
// LDS of one box of the downward pass.
template <typename T, int E = 1>
struct DownShared {
    // E: interaction-list entries per group per staging round of M2L
    static constexpr size_t kStageM2L = 2 * 3 * E * kWave * sizeof(cpx<T>);
    static constexpr size_t kScratch =
        sizeof(P2LStage<double>) > kStageM2L ? sizeof(P2LStage<double>) : kStageM2L;
    // the parent's near set and its metadata
    int PN[9], PL[9], PC[9], PN2[9], Pcnt[9], PT[9], Pb[9], PM[9];
    int IL[36];              // interaction list (compacted)
    signed char To[36];      // its offset classes
    int L4b[9], Pre[10], Nl4;  // separated leaves: first piece, piece offsets
    // Shared in turn by the parent's local expansion (read by L2L, which
    // every lane finishes before the barrier that ends the interaction
    // list), the M2L staging, the P2L staging and the group reduction.
    __align__(16) unsigned char scratch[kScratch];
    static_assert(kScratch >= 3 * (DC_P_MAX + 1) * sizeof(cpx<T>), "scratch holds the parent's L");
    __device__ cpx<T>* ploc() { return reinterpret_cast<cpx<T>*>(scratch); }
};

// Downward pass of one target box (own, at level l, cell (ti, tj), parent
// par) by one wave.  Writes nset[own] (unless the parent is quiet) and,
// unless the box is quiet (render only, owner != nullptr), L[own]; returns
// whether it was quiet.  Near sets hold -1 for cells without pieces.
// Split (render only): the near sets of every box are already in nset
// (k_near_all), owner is unused, and only the box's own incoming terms,
// M2L and P2L without the parent's L2L, are written to L[own] (k_down_l2l
// adds the parent's share level by level); returns whether the box is
// quiet, writing nothing then.
template <typename T, bool Count, int E = 1, bool Split = false>
__device__ bool down_body(DownShared<T, E>& sh, const TreeView& tv, const PieceView& pv, int l,
                          long long ti, long long tj, int own, int par, int p,
                          const cpx<double>* __restrict__ M, cpx<double>* __restrict__ L,
                          int* __restrict__ nset, const cpx<double>* __restrict__ Ttab,
                          int2* __restrict__ owner, unsigned long long* stats, int lane) {
    // the split pass stages one interaction-list entry per group and round
    // (several entries per round are used, and tested, by k_down only)
    static_assert(!Split || E == 1, "split pass: E = 1");
    // Render: the children of a quiet box are quiet (below); they record the
    // owner and leave without using the parent's near set.
    const int2 po = (!Split && owner != nullptr) ? owner[par] : make_int2(par, 0);
    int pn = -1;
    if (lane < 9) {
        pn = nset[(size_t)par * 9 + lane];
        sh.PN[lane] = pn;
    }
    if (po.x != par) {
        if (lane == 0) owner[own] = po;
        return true;
    }
    // Render: a parent's near set without pieces (every cell -1) makes the
    // box quiet (see below) before anything else is loaded; its own near
    // set is then empty too.
    if (Split && __ballot(pn >= 0) == 0) return true;
    if (!Split && owner != nullptr && __ballot(pn >= 0) == 0) {
        if (lane < 9) nset[(size_t)own * 9 + lane] = -1;
        if (lane == 0) owner[own] = po;
        return true;
    }
    // the parent's expansion for L2L, loaded while the near set is resolved
    if constexpr (!Split) {
        for (int i = lane; i < 3 * (p + 1); i += kWave) {
            const cpx<double> v = L[(size_t)par * 3 * (p + 1) + i];
            sh.ploc()[i] = to_c<T>(v.re, v.im);
        }
    }
    __syncthreads();
    // Metadata of the parent's near set, loaded once by lanes 0..8; it
    // serves the near set, the interaction list and the separated leaves.
    if (lane < 9) {
        const int c = sh.PN[lane];
        int lv = -1, ch = -1, np = 0, pc = 0, pb = 0, tch = 1, pm = 0;
        if (c >= 0) {
            lv = tv.lvl[c];
            ch = tv.child[c];
            np = tv.npc[c];
            pm = tv.cmask[c];
            pb = tv.pbeg[c];
            pc = tv.pend[c] - pb;
            tch = touches(tv, c, l, ti, tj) ? 1 : 0;
        }
        sh.PL[lane] = lv;
        sh.PC[lane] = ch;
        sh.PN2[lane] = np;
        sh.Pcnt[lane] = pc;
        sh.PT[lane] = tch;
        sh.Pb[lane] = pb;
        sh.PM[lane] = pm;
    }
    __syncthreads();
    // near set N(own): the 3 x 3 positions around own at level l, each the
    // deepest source box at level <= l covering it, or -1 where that box
    // holds no pieces (its subtree adds nothing to any list)
    if (!Split && lane < 9) {
        const long long px = ti + (lane % 3) - 1, py = tj + (lane / 3) - 1;
        int c = -1;
        const long long lim = 1LL << l;
        if (px >= 0 && py >= 0 && px < lim && py < lim) {
            const int slot = (int)((px >> 1) - (ti >> 1) + 1) + 3 * (int)((py >> 1) - (tj >> 1) + 1);
            c = sh.PN[slot];
            if (c >= 0 && sh.PL[slot] == l - 1 && sh.PC[slot] >= 0) {
                const int q = (int)(px & 1) + 2 * (int)(py & 1);
                c = ((sh.PM[slot] >> q) & 1) ? sh.PC[slot] + q : -1;
            } else if (c >= 0 && sh.PN2[slot] == 0) {
                c = -1;
            }
        }
        nset[(size_t)own * 9 + lane] = c;
    }
    // Render: a box whose parent's near set holds no pieces is quiet: it has
    // no interaction list, no separated leaves and no near field, and so do
    // its descendants; its local expansion is the nearest non-quiet
    // ancestor's, which it records instead of translating it (the L2L
    // translation of a truncated expansion is exact, so evaluating the
    // ancestor's expansion at a pixel gives the same value).
    if (Split || owner != nullptr) {
        const bool quiet = __ballot(lane < 9 && sh.PN[lane] >= 0 && sh.PN2[lane] != 0) == 0;
        if (quiet) {
            if (!Split && lane == 0) owner[own] = po;
            return true;
        }
        if (!Split && lane == 0) owner[own] = make_int2(own, l);
    }
    const int P1 = p + 1;
    const int ngrp = kWave / P1;
    const int grp = lane / P1;
    const int k = lane - grp * P1;
    const bool klane = grp == 0;           // owns coefficient k of the result
    const bool glane = grp < ngrp;         // member of a group
    const double r = half_width(tv, l);
    double cx, cy;
    center_of(tv, l, ti, tj, cx, cy);
    cpx<T> acc[3] = {{0, 0}, {0, 0}, {0, 0}};   // group 0: the result
    cpx<T> gacc[3] = {{0, 0}, {0, 0}, {0, 0}};  // every group: its share
    // incoming-from-incoming from the parent (Eq. i-f-i), scaled:
    //   Lt_k = 2^{-k} sum_{m>=k} C(m,k) z0^{m-k} Lt'_m, z0 = (c - c')/r'
    if (!Split && klane) {
        const cpx<T> z0 = {(T)((ti & 1) ? 0.5 : -0.5), (T)((tj & 1) ? 0.5 : -0.5)};
        const cpx<T>* src = sh.ploc();
        cpx<T> pw = {1, 0};
        T binom = 1;
        const T sc = (T)ldexp(1.0, -k);
        for (int j = 0; j <= p - k; ++j) {  // j = m - k: the same in every lane
            const int m = k + j;
            const cpx<T> f = cscale(pw, binom * sc);
            for (int ch = 0; ch < 3; ++ch) acc[ch] = cadd(acc[ch], cmul(f, src[m * 3 + ch]));
            binom = binom * (T)(m + 1) * recip<T>(j + 1);
            pw = cmul(pw, z0);
        }
    }
    // interaction list: 36 candidates (children of the parent's 9 near-set
    // boxes), compacted with a ballot
    const T log2r = (T)log(2.0 * r);
    {
        bool valid = false;
        int d = -1, o = 0;
        if (lane < 36) {
            const int sl = lane >> 2, q = lane & 3;
            if (sh.PN[sl] >= 0 && sh.PL[sl] == l - 1 && sh.PC[sl] >= 0) {
                const long long ppx = (ti >> 1) + (sl % 3) - 1, ppy = (tj >> 1) + (sl / 3) - 1;
                d = sh.PC[sl] + q;
                const int dx = (int)(2 * ppx + (q & 1) - ti), dy = (int)(2 * ppy + (q >> 1) - tj);
                o = (dy + 3) * 7 + (dx + 3);
                valid = !(dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) && ((sh.PM[sl] >> q) & 1);
            }
        }
        const unsigned long long mask = __ballot(valid);
        if (valid) {
            const int at = __popcll(mask & ((1ULL << lane) - 1ULL));
            sh.IL[at] = d;
            sh.To[at] = (signed char)o;
        }
        __syncthreads();
        const int nIL = __popcll(mask);
        // Source coefficients of each round's ngrp E entries are staged in
        // LDS by the whole wave (coalesced), double-buffered: the loads of
        // round b+1 are in flight while round b is computed.  Group g takes
        // the round's entries g, g + ngrp, ..., so every group sums the same
        // entries in the same order whatever E is.
        const int per_round = ngrp * E * P1 * 3;  // complex values, <= 3 E kWave
        cpx<T>* stage = reinterpret_cast<cpx<T>*>(sh.scratch);
        constexpr int kPer = 3 * E;
        cpx<T> pre[kPer];
        auto fetch = [&](int base) {
            for (int t = 0; t < kPer; ++t) {
                const int i = lane + t * kWave;
                if (i < per_round) {
                    const int g = i / (P1 * 3), off = i - g * (P1 * 3);
                    const int e = base + g;
                    if (e < nIL) {
                        const cpx<double> v = M[(size_t)sh.IL[e] * P1 * 3 + off];
                        pre[t] = to_c<T>(v.re, v.im);
                    } else {
                        pre[t] = cpx<T>{0, 0};
                    }
                }
            }
        };
        auto put = [&](int buf) {
            for (int t = 0; t < kPer; ++t) {
                const int i = lane + t * kWave;
                if (i < per_round) stage[buf * per_round + i] = pre[t];
            }
        };
        if (nIL > 0) {
            fetch(0);
            put(0);
        }
        int buf = 0;
        for (int base = 0; base < nIL; base += ngrp * E) {
            __syncthreads();
            const bool next = base + ngrp * E < nIL;
            if (next) fetch(base + ngrp * E);
            for (int j = 0; j < E; ++j) {
                const int slot = j * ngrp + grp;
                const int e = base + slot;
                if (glane && e < nIL) {
                    const cpx<T>* src = stage + buf * per_round + slot * P1 * 3;
                    const cpx<double>* Tk = Ttab + ((size_t)sh.To[e] * P1 + k) * P1;
                    for (int m = 0; m <= p; ++m) {
                        const cpx<T> t = to_c<T>(Tk[m].re, Tk[m].im);
                        for (int ch = 0; ch < 3; ++ch)
                            gacc[ch] = cadd(gacc[ch], cmul(t, src[m * 3 + ch]));
                    }
                    if (k == 0)
                        for (int ch = 0; ch < 3; ++ch)
                            gacc[ch] = csub(gacc[ch], cscale(src[ch], log2r));
                }
            }
            if (next) put(buf ^ 1);
            buf ^= 1;
        }
        if (Count && lane == 0) atomicAdd(stats + kStatM2L, (unsigned long long)nIL);
        __syncthreads();
    }
    // bigger separated list: coarser source leaves that do not touch us
    if (lane == 0) {
        int nl4 = 0;
        sh.Pre[0] = 0;
        for (int s = 0; s < 9; ++s) {
            const int c = sh.PN[s];
            if (c < 0 || (sh.PL[s] == l - 1 && sh.PC[s] >= 0)) continue;
            bool dup = false;
            for (int s2 = 0; s2 < s; ++s2) dup |= (sh.PN[s2] == c);
            if (dup || sh.PN2[s] == 0 || sh.PT[s]) continue;
            sh.L4b[nl4] = sh.Pb[s];
            sh.Pre[nl4 + 1] = sh.Pre[nl4] + sh.Pcnt[s];
            ++nl4;
        }
        sh.Nl4 = nl4;
    }
    __syncthreads();
    const int nl4 = sh.Nl4, total = sh.Pre[nl4];
    // FP32 arithmetic (FP32 path) only when every piece's charge is small:
    // a separated leaf's pieces can carry large charges of both signs whose
    // contributions cancel, and those boxes take the FP64 form.
    bool p2l32 = false;
    if constexpr (sizeof(T) == 4) {
        if (total > 0) {
            const double* w64 = weights<double>(pv);
            double mq = 0.0;
            for (int g = lane; g < total; g += kWave) {
                int u = 0;
                while (u + 1 < nl4 && sh.Pre[u + 1] <= g) ++u;
                const int e = sh.L4b[u] + (g - sh.Pre[u]);
                double q = 0.0;
                for (int c6 = 0; c6 < 6; ++c6) q = fmax(q, fabs(w64[(size_t)c6 * pv.n + e]));
                mq = fmax(mq, q * pv.len[e]);
            }
            for (int o = kWave / 2; o > 0; o >>= 1) mq = fmax(mq, __shfl_xor(mq, o, kWave));
            p2l32 = mq <= kP2LFloat;
        }
    }
    if (total > 0 && p2l32) {
        P2LStage<T>& sp = *reinterpret_cast<P2LStage<T>*>(sh.scratch);
        const double inv_r = 1.0 / r;
        const T rr = (T)r, logr = (T)log(r);
        const T* w = weights<T>(pv);
        cpx<T> c01[2][3];  // this lane's k = 0, 1 terms, summed over its pieces
        for (int ch = 0; ch < 3; ++ch) c01[0][ch] = c01[1][ch] = {0, 0};
        for (int base = 0; base < total; base += kWave) {
            // stage: one piece per lane
            const int g = base + lane;
            if (g < total) {
                int u = 0;
                while (u + 1 < nl4 && sh.Pre[u + 1] <= g) ++u;
                const int e = sh.L4b[u] + (g - sh.Pre[u]);
                const cpx<T> A = to_c<T>((pv.x0[e] - cx) * inv_r, (pv.y0[e] - cy) * inv_r);
                const cpx<T> B = to_c<T>((pv.x1[e] - cx) * inv_r, (pv.y1[e] - cy) * inv_r);
                const cpx<T> wbar = {(T)pv.tx[e], (T)(-pv.ty[e])};
                const T len = (T)pv.len[e];
                const cpx<T> zA = cinv(A), zB = cinv(B);
                const cpx<T> BA = cmul(B, cpx<T>{A.re, -A.im});
                const T nA = A.re * A.re + A.im * A.im, nB = B.re * B.re + B.im * B.im;
                const cpx<T> Lam = {T(0.5) * log(nB / nA), atan2(BA.im, BA.re)};
                const cpx<T> lA = clog(A);
                const cpx<T> t2 = cmul(cmul(wbar, cscale(B, rr)), Lam);
                const cpx<T> sv0 = {-(len * (logr + lA.re) + t2.re - len), -(len * lA.im + t2.im)};
                const cpx<T> mv0 = {Lam.im, -Lam.re};
                const cpx<T> sv1 = cmul(wbar, cscale(Lam, rr));
                const cpx<T> d1 = csub(zB, zA);
                const cpx<T> mv1 = {-d1.im, d1.re};
                sp.zAr[lane] = zA.re;
                sp.zAi[lane] = zA.im;
                sp.zBr[lane] = zB.re;
                sp.zBi[lane] = zB.im;
                sp.wr[lane] = wbar.re;
                sp.wi[lane] = wbar.im;
                for (int ch = 0; ch < 3; ++ch) {
                    const T qs = w[(size_t)ch * pv.n + e], qm = w[(size_t)(3 + ch) * pv.n + e];
                    sp.qs[ch][lane] = qs;
                    sp.qm[ch][lane] = qm;
                    c01[0][ch] = cadd(c01[0][ch], cadd(cscale(sv0, qs), cscale(mv0, qm)));
                    c01[1][ch] = cadd(c01[1][ch], cadd(cscale(sv1, qs), cscale(mv1, qm)));
                }
            }
            __syncthreads();
            // k >= 2: the groups deal the staged pieces round-robin
            const int n = min(kWave, total - base);
            if (glane && k >= 2) {
                const T sck = rr * recip<T>(k) * recip<T>(k - 1), rk = recip<T>(k);
                for (int j = grp; j < n; j += ngrp) {
                    const cpx<T> zA = {sp.zAr[j], sp.zAi[j]}, zB = {sp.zBr[j], sp.zBi[j]};
                    const cpx<T> pa = cpow(zA, k - 1), pb = cpow(zB, k - 1);
                    const cpx<T> sv = cmul(cpx<T>{sp.wr[j], sp.wi[j]}, cscale(csub(pa, pb), sck));
                    const cpx<T> dd = cscale(csub(cmul(pb, zB), cmul(pa, zA)), rk);
                    const cpx<T> mv = {-dd.im, dd.re};
                    for (int ch = 0; ch < 3; ++ch)
                        gacc[ch] = cadd(gacc[ch], cadd(cscale(sv, sp.qs[ch][j]),
                                                       cscale(mv, sp.qm[ch][j])));
                }
            }
            __syncthreads();
        }
        // k = 0, 1 terms: summed over the wave
        for (int kk = 0; kk < 2; ++kk)
            for (int ch = 0; ch < 3; ++ch) {
                const cpx<T> v = {wave_sum(c01[kk][ch].re), wave_sum(c01[kk][ch].im)};
                if (klane && k == kk) acc[ch] = cadd(acc[ch], v);
            }
        } else if (total > 0) {
        // In FP64 whatever T: a separated leaf's pieces can carry large
        // charges of both signs whose contributions cancel.
        P2LStage<double>& sp = *reinterpret_cast<P2LStage<double>*>(sh.scratch);
        const double inv_r = 1.0 / r;
        const double rr = r, logr = log(r);
        const double* w = weights<double>(pv);
        cpx<double> c01[2][3];  // this lane's k = 0, 1 terms, summed over its pieces
        cpx<double> pacc[3] = {{0, 0}, {0, 0}, {0, 0}};  // this lane's k >= 2 share
        for (int ch = 0; ch < 3; ++ch) c01[0][ch] = c01[1][ch] = {0, 0};
        for (int base = 0; base < total; base += kWave) {
            // stage: one piece per lane
            const int g = base + lane;
            if (g < total) {
                int u = 0;
                while (u + 1 < nl4 && sh.Pre[u + 1] <= g) ++u;
                const int e = sh.L4b[u] + (g - sh.Pre[u]);
                const cpx<double> A = {(pv.x0[e] - cx) * inv_r, (pv.y0[e] - cy) * inv_r};
                const cpx<double> B = {(pv.x1[e] - cx) * inv_r, (pv.y1[e] - cy) * inv_r};
                const cpx<double> wbar = {pv.tx[e], -pv.ty[e]};
                const double len = pv.len[e];
                const cpx<double> zA = cinv(A), zB = cinv(B);
                const cpx<double> BA = cmul(B, cpx<double>{A.re, -A.im});
                const double nA = A.re * A.re + A.im * A.im, nB = B.re * B.re + B.im * B.im;
                const cpx<double> Lam = {0.5 * log(nB / nA), atan2(BA.im, BA.re)};
                const cpx<double> lA = clog(A);
                const cpx<double> t2 = cmul(cmul(wbar, cscale(B, rr)), Lam);
                const cpx<double> sv0 = {-(len * (logr + lA.re) + t2.re - len), -(len * lA.im + t2.im)};
                const cpx<double> mv0 = {Lam.im, -Lam.re};
                const cpx<double> sv1 = cmul(wbar, cscale(Lam, rr));
                const cpx<double> d1 = csub(zB, zA);
                const cpx<double> mv1 = {-d1.im, d1.re};
                sp.zAr[lane] = zA.re;
                sp.zAi[lane] = zA.im;
                sp.zBr[lane] = zB.re;
                sp.zBi[lane] = zB.im;
                sp.wr[lane] = wbar.re;
                sp.wi[lane] = wbar.im;
                for (int ch = 0; ch < 3; ++ch) {
                    const double qs = w[(size_t)ch * pv.n + e], qm = w[(size_t)(3 + ch) * pv.n + e];
                    sp.qs[ch][lane] = qs;
                    sp.qm[ch][lane] = qm;
                    c01[0][ch] = cadd(c01[0][ch], cadd(cscale(sv0, qs), cscale(mv0, qm)));
                    c01[1][ch] = cadd(c01[1][ch], cadd(cscale(sv1, qs), cscale(mv1, qm)));
                }
            }
            __syncthreads();
            // k >= 2: the groups deal the staged pieces round-robin
            const int n = min(kWave, total - base);
            if (glane && k >= 2) {
                const double sck = rr * recip<double>(k) * recip<double>(k - 1), rk = recip<double>(k);
                for (int j = grp; j < n; j += ngrp) {
                    const cpx<double> zA = {sp.zAr[j], sp.zAi[j]}, zB = {sp.zBr[j], sp.zBi[j]};
                    const cpx<double> pa = cpow(zA, k - 1), pb = cpow(zB, k - 1);
                    const cpx<double> sv = cmul(cpx<double>{sp.wr[j], sp.wi[j]}, cscale(csub(pa, pb), sck));
                    const cpx<double> dd = cscale(csub(cmul(pb, zB), cmul(pa, zA)), rk);
                    const cpx<double> mv = {-dd.im, dd.re};
                    for (int ch = 0; ch < 3; ++ch)
                        pacc[ch] = cadd(pacc[ch], cadd(cscale(sv, sp.qs[ch][j]),
                                                       cscale(mv, sp.qm[ch][j])));
                }
            }
            __syncthreads();
        }
        for (int ch = 0; ch < 3; ++ch) gacc[ch] = cadd(gacc[ch], to_c<T>(pacc[ch].re, pacc[ch].im));
        // k = 0, 1 terms: summed over the wave
        for (int kk = 0; kk < 2; ++kk)
            for (int ch = 0; ch < 3; ++ch) {
                const double vr = wave_sum(c01[kk][ch].re), vi = wave_sum(c01[kk][ch].im);
                if (klane && k == kk) acc[ch] = cadd(acc[ch], to_c<T>(vr, vi));
            }
        }
    if (Count && lane == 0) {
        atomicAdd(stats + kStatP2L, (unsigned long long)total);
        if (!p2l32) atomicAdd(stats + kStatP2L64, (unsigned long long)total);
        atomicAdd(stats + kStatL2L, 1ULL);
    }
    // reduce the groups' shares into group 0
    cpx<T>(*sRed)[3] = reinterpret_cast<cpx<T>(*)[3]>(sh.scratch);
    if (glane)
        for (int ch = 0; ch < 3; ++ch) sRed[lane][ch] = gacc[ch];
    __syncthreads();
    if (!klane) return false;
    for (int g = 0; g < ngrp; ++g)
        for (int ch = 0; ch < 3; ++ch) acc[ch] = cadd(acc[ch], sRed[g * P1 + k][ch]);
    cpx<double>* out = L + ((size_t)own * P1 + k) * 3;
    for (int ch = 0; ch < 3; ++ch) out[ch] = {(double)acc[ch].re, (double)acc[ch].im};
    return false;
}

// E > 1: deeper M2L staging for levels with few boxes (same values).
template <typename T, bool Count, int E = 1>
__global__ void __launch_bounds__(kWave, 4)
k_down(TreeView tv, PieceView pv, DownLevel dl, int p, const cpx<double>* __restrict__ M,
       cpx<double>* __restrict__ L, int* __restrict__ nset, const cpx<double>* __restrict__ Ttab,
       int2* __restrict__ owner) {
    __shared__ DownShared<T, E> sh;
    const int lane = threadIdx.x;
    const int l = dl.l;
    long long ti, tj;
    int own, par;
    if (dl.solve) {
        own = dl.first + blockIdx.x;
        if (tv.child[own] < 0 && tv.nend[own] == tv.nbeg[own]) return;  // no targets
        ti = tv.ix[own];
        tj = tv.iy[own];
        par = tv.parent[own];
    } else {
        const VpLevel& e = find_entry(dl.vl, dl.nvl, (int)blockIdx.x);
        const int b = (int)blockIdx.x - e.first_block;
        ti = e.i0 + b % e.wl;
        tj = e.j0 + b / e.wl;
        own = e.off + b;
        par = e.poff + (int)((ti >> 1) - e.pi0) + (int)((tj >> 1) - e.pj0) * e.pwl;
    }
    (void)down_body<T, Count, E>(sh, tv, pv, l, ti, tj, own, par, p, M, L, nset, Ttab, owner,
                                 dl.stats, lane);
}

template <typename T>
__global__ void k_init_root(int p, cpx<T>* __restrict__ L, int* __restrict__ nset) {
    const int t = threadIdx.x;
    if (t < 9) nset[t] = (t == 4) ? 0 : -1;
    for (int i = t; i < (p + 1) * 3; i += blockDim.x) L[i] = {0, 0};
}

// -------------------------------------------------------------- leaf pass
struct LeafArgs {
    // render (k_tile)
    const VpLeaf* vleaf;     // one entry per viewport
    int nvleaf;
    const int* edges;        // pixel ranges of tile columns and rows
    int out_f64;             // images in FP64 (else FP32)
    // solve (k_leaf)
    const int* target_leaves;
    const double *node_x, *node_y;
    double* y;
    int N;
    double near2;            // (near_fp64)^2, FP32 only
    unsigned long long* stats;  // optional work counters
    // heavy small render tiles left to k_tile_big; hv_list null: none
    int* hv_ctl;             // [0] / [2] tiles queued at the front / back, [1] next to take
    int* hv_list;            // queued tiles (global leaf block), hv_list_cap entries
    int hv_list_cap;
    unsigned char* hv_flag;  // per global leaf block: 0 k_tile, 1 queued, 2 done,
                             // 3 k_tile and 4 queued, with the lists kept in `lists`
    int* lists;              // kListInts per global leaf block (8-px tiles)
    // cached near-field tables of the solve (SolveTables), by target leaf
    int* tab_count;                // count pass: [leaf][2] near pieces, separated boxes
    const long long* tab_pair_off; // [leaf] first (node, piece) pair
    const int* tab_piece_off;      // [leaf + 1] first near piece
    const int* tab_w_off;          // [leaf + 1] first separated box
    int* tab_piece;                // near pieces, traversal order
    int* tab_w;                    // separated boxes, traversal order
    double* tab_val;               // [pair][2] (int ln, theta) of the chord integrals
};

template <typename T, int NT>
struct LeafShared {
    T px[NT], py[NT], tx[NT], ty[NT], len[NT];
    T w[6][NT];
    int pid[NT];
    int U[kUCap], Upre[kUCap + 1], W[kWCap], stack[kSCap];
    int nU, nW, nS, more;
};

// Solve leaf pass (Alg. 8 at the source leaves): targets are the
// collocation nodes of each leaf holding nodes; y[3][N] receives the
// representation at the nodes (before the self-segment correction).
// Modes: kLeafEval evaluates; kLeafCount (FP64) counts each leaf's near
// pieces and separated boxes; kLeafFill (FP64) writes the leaf's lists and
// the chord integrals of each (node, near piece) pair into the tables that
// k_leaf_tab reads instead (Sec. 6.4's precomputed operators).
enum { kLeafEval = 0, kLeafCount = 1, kLeafFill = 2 };

template <typename T, int NT, int Mode = kLeafEval>
__global__ void __launch_bounds__(NT)
k_leaf(TreeView tv, PieceView pv, LeafArgs a, int p, const cpx<double>* __restrict__ M,
       const cpx<double>* __restrict__ Lc, const int* __restrict__ nset) {
    static_assert(Mode == kLeafEval || sizeof(T) == 8, "tables hold FP64 values");
    __shared__ LeafShared<T, NT> sh;
    const int tid = threadIdx.x;
    const int own = a.target_leaves[blockIdx.x];
    const long long ti = tv.ix[own], tj = tv.iy[own];
    const int base_pos = tv.nbeg[own];
    const int n_targets = tv.nend[own] - base_pos;
    const int l = tv.lvl[own];
    const double r = half_width(tv, l);
    double cx, cy;
    center_of(tv, l, ti, tj, cx, cy);
    const T* wts = weights<T>(pv);
    const cpx<double>* loc = Lc + (size_t)own * (p + 1) * 3;

    for (int tbase = 0; tbase < n_targets; tbase += NT) {
        // lane tid: target t = tid % TP of this pass, group grp = tid / TP;
        // the G groups split the pass's separated boxes and near pieces
        // (a leaf holds a few nodes: one lane per target would leave most
        // of the wave idle) and their sums are added across the groups
        const int n_here = min(NT, n_targets - tbase);
        int TP = 1;
        while (TP < n_here) TP <<= 1;
        const int G = NT / TP;
        const int t = tid & (TP - 1), grp = tid / TP;
        const int tgt = tbase + t;
        const bool active = t < n_here;
        double x = cx, y = cy;
        int out_idx = 0;
        if (active) {
            const int node = tv.node_perm[base_pos + tgt];
            x = a.node_x[node];
            y = a.node_y[node];
            out_idx = node;
        }
        const T xr = (T)(x - cx), yr = (T)(y - cy);
        double accE[3] = {0, 0, 0};
        // near-field sums are kept in FP64 (an FP64 add issues at the FP32 rate)
        double accP[3] = {0, 0, 0};
        double acc64[3] = {0, 0, 0};
        // table positions of this pass's rounds (count and fill modes)
        int runP = 0, runW = 0;
        // target-from-incoming (Eq. t-f-i): Re sum_k ((x-c)/r)^k Lt_k
        if (Mode == kLeafEval && l >= 2 && grp == 0) {
            const cpx<double> z = {(x - cx) / r, (y - cy) / r};
            for (int ch = 0; ch < 3; ++ch) {
                cpx<double> s = loc[p * 3 + ch];
                for (int kk = p - 1; kk >= 0; --kk) s = cadd(cmul(s, z), loc[kk * 3 + ch]);
                accE[ch] += s.re;
            }
        }
        if (a.stats && tid == 0) {
            const unsigned long long na = (unsigned long long)min(NT, n_targets - tbase);
            if (l >= 2) atomicAdd(a.stats + kStatL2P, na);
            if (tbase == 0) atomicAdd(a.stats + kStatLeaf, 1ULL);
        }
        // near-set traversal, in rounds bounded by the list capacities
        if (tid == 0) {
            sh.nS = 0;
            for (int s = 0; s < 9; ++s) {
                const int c = nset[(size_t)own * 9 + s];
                bool dup = c < 0;
                for (int s2 = 0; s2 < s && !dup; ++s2) dup = nset[(size_t)own * 9 + s2] == c;
                if (!dup && tv.npc[c] > 0) sh.stack[sh.nS++] = c;
            }
        }
        __syncthreads();
        for (;;) {
            if (tid == 0) {
                int nU = 0, nW = 0;
                while (sh.nS > 0 && nU < kUCap && nW + 4 <= kWCap) {
                    const int c = sh.stack[--sh.nS];
                    const int c0 = tv.child[c], cm = tv.cmask[c], lc = tv.lvl[c];
                    const long long bx = tv.ix[c], by = tv.iy[c];
                    if (c0 < 0) {
                        sh.Upre[nU] = 0;
                        sh.U[nU++] = c;
                        continue;
                    }
                    for (int q = 0; q < 4; ++q) {
                        const int d = c0 + q;
                        if (!((cm >> q) & 1)) continue;
                        if (touches_at(lc + 1, 2 * bx + (q & 1), 2 * by + (q >> 1), l, ti, tj)) {
                            if (sh.nS < kSCap) sh.stack[sh.nS++] = d;
                        } else {
                            sh.W[nW++] = d;
                        }
                    }
                }
                int acc = 0;
                for (int u = 0; u < nU; ++u) {
                    sh.Upre[u] = acc;
                    acc += tv.pend[sh.U[u]] - tv.pbeg[sh.U[u]];
                }
                sh.Upre[nU] = acc;
                sh.nU = nU;
                sh.nW = nW;
                sh.more = sh.nS > 0;
            }
            __syncthreads();
            // copy the round's shared scalars: thread 0 rewrites them only after
            // the closing barrier of this round
            const int nU = sh.nU, nW = sh.nW, more = sh.more;
            if (a.stats && tid == 0) {
                const unsigned long long na = (unsigned long long)min(NT, n_targets - tbase);
                atomicAdd(a.stats + kStatM2P, na * nW);
                atomicAdd(a.stats + kStatP2P, na * (unsigned long long)sh.Upre[nU]);
            }
            if constexpr (Mode == kLeafFill) {
                if (tbase == 0)
                    for (int u = tid; u < nW; u += NT)
                        a.tab_w[a.tab_w_off[blockIdx.x] + runW + u] = sh.W[u];
            }
            // target-from-outgoing (Eq. t-f-o), scaled:
            //   Re[-log(x - c) Mt_0 + sum_{k>=1} (1/k) (r/(x-c))^k Mt_k]
            if (Mode == kLeafEval && active) {
                for (int u = grp; u < nW; u += G) {
                    const int d = sh.W[u];
                    const int ld = tv.lvl[d];
                    const double rd = half_width(tv, ld);
                    double dcx, dcy;
                    center_of(tv, ld, tv.ix[d], tv.iy[d], dcx, dcy);
                    const cpx<double> rel = {(x - dcx) / rd, (y - dcy) / rd};
                    const cpx<double> z = cinv(rel);
                    const cpx<double> lg = clog(rel);
                    const double lr = log(rd);
                    const cpx<double>* src = M + (size_t)d * (p + 1) * 3;
                    for (int ch = 0; ch < 3; ++ch) {
                        cpx<double> s = cscale(src[p * 3 + ch], recip<double>(p));
                        for (int kk = p - 1; kk >= 1; --kk)
                            s = cadd(cmul(s, z), cscale(src[kk * 3 + ch], recip<double>(kk)));
                        s = cmul(s, z);
                        const cpx<double> m0 = src[ch];
                        // Re(-(lr + lg) * m0)
                        accE[ch] += s.re - ((lr + lg.re) * m0.re - lg.im * m0.im);
                    }
                }
            }
            // target-from-source (App. D) over the pieces of the near leaves
            const int total = sh.Upre[nU];
            for (int pbase = 0; pbase < total && Mode != kLeafCount; pbase += NT) {
                __syncthreads();
                const int g = pbase + tid;
                if (g < total) {
                    int lo = 0, hi = nU - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (sh.Upre[mid] <= g) lo = mid; else hi = mid - 1;
                    }
                    const int e = tv.pbeg[sh.U[lo]] + (g - sh.Upre[lo]);
                    sh.px[tid] = (T)(pv.x0[e] - cx);
                    sh.py[tid] = (T)(pv.y0[e] - cy);
                    sh.tx[tid] = (T)pv.tx[e];
                    sh.ty[tid] = (T)pv.ty[e];
                    sh.len[tid] = (T)pv.len[e];
                    for (int c6 = 0; c6 < 6; ++c6) sh.w[c6][tid] = wts[(size_t)c6 * pv.n + e];
                    sh.pid[tid] = sizeof(T) == 4 && pv.heavy[e] ? -1 - e : e;
                    if (Mode == kLeafFill && tbase == 0)
                        a.tab_piece[a.tab_piece_off[blockIdx.x] + runP + g] = e;
                }
                __syncthreads();
                if constexpr (Mode == kLeafFill) {
                    // the same closed form as the FP64 evaluation below
                    const int m = min(NT, total - pbase);
                    if (active)
                        for (int j = grp; j < m; j += G) {
                            const T dx = sh.px[j] - xr, dy = sh.py[j] - yr;
                            T il, th;
                            chord_log_theta<T>(dx, dy, sh.tx[j], sh.ty[j], sh.len[j], il, th);
                            const size_t at = (size_t)a.tab_pair_off[blockIdx.x] +
                                              (size_t)(runP + pbase + j) * n_targets + tgt;
                            a.tab_val[2 * at] = il;
                            a.tab_val[2 * at + 1] = th;
                        }
                    continue;
                }
                if (active) {
                    const int m = min(NT, total - pbase);
                    const float near2f = (float)a.near2;
                    for (int j = grp; j < m; j += G) {
                        const T dx = sh.px[j] - xr, dy = sh.py[j] - yr;
                        if (sizeof(T) == 4) {
                            const float tx = (float)sh.tx[j], ty = (float)sh.ty[j];
                            const float la = (float)sh.len[j];
                            const float xi1 = (float)dx * tx + (float)dy * ty;
                            const float h = (float)dy * tx - (float)dx * ty;
                            const float xi2 = xi1 + la;
                            // squared distance to the chord, branch-free
                            const float along = fmaxf(xi1, 0.f) + fmaxf(-xi2, 0.f);
                            const float dd = along * along + h * h;
                            const int pid = sh.pid[j];
                            if (dd < near2f * la * la || pid < 0) {
                                // near-singular pair or heavy piece: closed form in FP64
                                const int e = pid < 0 ? -1 - pid : pid;
                                double il, th;
                                chord_log_theta<double>(pv.x0[e] - x, pv.y0[e] - y, pv.tx[e],
                                                        pv.ty[e], pv.len[e], il, th);
                                for (int ch = 0; ch < 3; ++ch)
                                    acc64[ch] += il * pv.w64[(size_t)ch * pv.n + e] +
                                                 th * pv.w64[(size_t)(3 + ch) * pv.n + e];
                                if (a.stats) atomicAdd(a.stats + kStatP2P64, 1ULL);
                                continue;
                            }
                            float il, th;
                            chord_fast(xi1, h, xi2, la, il, th);
                            for (int ch = 0; ch < 3; ++ch)
                                accP[ch] += (double)(il * (float)sh.w[ch][j] +
                                                     th * (float)sh.w[3 + ch][j]);
                            continue;
                        }
                        T il, th;
                        chord_log_theta<T>(dx, dy, sh.tx[j], sh.ty[j], sh.len[j], il, th);
                        for (int ch = 0; ch < 3; ++ch)
                            accP[ch] += il * sh.w[ch][j] + th * sh.w[3 + ch][j];
                    }
                }
            }
            if constexpr (Mode == kLeafCount) {
                if (tbase == 0 && tid == 0) {
                    a.tab_count[2 * blockIdx.x] += total;
                    a.tab_count[2 * blockIdx.x + 1] += nW;
                }
            }
            runP += total;
            runW += nW;
            __syncthreads();
            if (!more) break;
        }
        if constexpr (Mode != kLeafEval) continue;
        // the groups' sums, added over the lanes that hold the same target
        double tot[3];
        for (int ch = 0; ch < 3; ++ch) {
            tot[ch] = accE[ch] - accP[ch] - acc64[ch];
            for (int off = TP; off < NT; off <<= 1) tot[ch] += __shfl_xor(tot[ch], off, NT);
        }
        if (active && grp == 0) {
            for (int ch = 0; ch < 3; ++ch) a.y[(size_t)ch * a.N + out_idx] = tot[ch] / kTwoPi;
        }
        __syncthreads();
    }
}

// Solve leaf pass from the cached tables (SolveTables): the leaf's
// separated boxes and near pieces as stored by k_leaf's fill pass, and the
// chord integrals of each (node, near piece) pair, so no traversal and no
// closed form is evaluated; the lanes are grouped as in k_leaf.
template <int NT>
__global__ void __launch_bounds__(NT)
k_leaf_tab(TreeView tv, PieceView pv, LeafArgs a, int p, const cpx<double>* __restrict__ M,
           const cpx<double>* __restrict__ Lc) {
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int own = a.target_leaves[b];
    const long long ti = tv.ix[own], tj = tv.iy[own];
    const int base_pos = tv.nbeg[own];
    const int n_targets = tv.nend[own] - base_pos;
    const int l = tv.lvl[own];
    const double r = half_width(tv, l);
    double cx, cy;
    center_of(tv, l, ti, tj, cx, cy);
    const cpx<double>* loc = Lc + (size_t)own * (p + 1) * 3;
    const int poff = a.tab_piece_off[b], np = a.tab_piece_off[b + 1] - poff;
    const int woff = a.tab_w_off[b], nw = a.tab_w_off[b + 1] - woff;
    const double* val = a.tab_val + 2 * (size_t)a.tab_pair_off[b];
    for (int tbase = 0; tbase < n_targets; tbase += NT) {
        const int n_here = min(NT, n_targets - tbase);
        int TP = 1;
        while (TP < n_here) TP <<= 1;
        const int G = NT / TP;
        const int t = tid & (TP - 1), grp = tid / TP;
        const int tgt = tbase + t;
        const bool active = t < n_here;
        double x = cx, y = cy;
        int out_idx = 0;
        if (active) {
            const int node = tv.node_perm[base_pos + tgt];
            x = a.node_x[node];
            y = a.node_y[node];
            out_idx = node;
        }
        double acc[3] = {0, 0, 0};
        if (active && l >= 2 && grp == 0) {
            const cpx<double> z = {(x - cx) / r, (y - cy) / r};
            for (int ch = 0; ch < 3; ++ch) {
                cpx<double> s = loc[p * 3 + ch];
                for (int kk = p - 1; kk >= 0; --kk) s = cadd(cmul(s, z), loc[kk * 3 + ch]);
                acc[ch] += s.re;
            }
        }
        if (active) {
            for (int u = grp; u < nw; u += G) {
                const int d = a.tab_w[woff + u];
                const int ld = tv.lvl[d];
                const double rd = half_width(tv, ld);
                double dcx, dcy;
                center_of(tv, ld, tv.ix[d], tv.iy[d], dcx, dcy);
                const cpx<double> rel = {(x - dcx) / rd, (y - dcy) / rd};
                const cpx<double> z = cinv(rel);
                const cpx<double> lg = clog(rel);
                const double lr = log(rd);
                const cpx<double>* src = M + (size_t)d * (p + 1) * 3;
                for (int ch = 0; ch < 3; ++ch) {
                    cpx<double> s = cscale(src[p * 3 + ch], recip<double>(p));
                    for (int kk = p - 1; kk >= 1; --kk)
                        s = cadd(cmul(s, z), cscale(src[kk * 3 + ch], recip<double>(kk)));
                    s = cmul(s, z);
                    const cpx<double> m0 = src[ch];
                    acc[ch] += s.re - ((lr + lg.re) * m0.re - lg.im * m0.im);
                }
            }
            for (int j = grp; j < np; j += G) {
                const int e = a.tab_piece[poff + j];
                const size_t at = 2 * ((size_t)j * n_targets + tgt);
                const double il = val[at], th = val[at + 1];
                for (int ch = 0; ch < 3; ++ch)
                    acc[ch] -= il * pv.w64[(size_t)ch * pv.n + e] +
                               th * pv.w64[(size_t)(3 + ch) * pv.n + e];
            }
        }
        for (int ch = 0; ch < 3; ++ch)
            for (int off = TP; off < NT; off <<= 1) acc[ch] += __shfl_xor(acc[ch], off, NT);
        if (active && grp == 0)
            for (int ch = 0; ch < 3; ++ch) a.y[(size_t)ch * a.N + out_idx] = acc[ch] / kTwoPi;
    }
}

// Exclusive prefix sum over the 64 lanes of a wave, and the wave total.
__device__ inline int wave_excl_scan(int v, int lane, int& total) {
    int x = v;
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    total = __shfl(x, kWave - 1, kWave);
    return x - v;
}

constexpr int kQCap = 512;   // traversal stack of the render leaf pass
constexpr int kMaxLevels = 64;
// Waves that share one small (8 x 8 pixel) render tile's near field.
constexpr int kSplit = 1;

template <typename T, int NT>
struct TileShared {
    // piece staging (also the partial sums of the near-field split at the
    // end of a pass)
    __align__(16) T px[NT];
    T py[NT], tx[NT], ty[NT], len[NT];
    T w[6][NT];
    int pid[NT];
    unsigned char far[NT];  // FP32: the piece is well separated from the whole tile
    int U[kUCap], Upre[kUCap + 1], W[kWCap], Q[kQCap];
    int nU, nW, nQ, heavy;
};

// A piece whose chord lies at least kGaussSep chord lengths from every
// point of a tile's box is integrated at the tile's pixels by the two-point
// Gauss-Legendre rule (FP32 path): for r >= kGaussSep la the rule's error
// is below la (la/r)^4 / 720 for the single layer and 3e-2 (la/r)^5 for the
// double layer, far under FP32 rounding of the closed form's terms.
constexpr float kGaussSep = 10.0f;
constexpr float kGaussA = 0.21132486540518713f;  // (1 - 1/sqrt(3)) / 2
constexpr float kGaussB = 0.78867513459481287f;  // (1 + 1/sqrt(3)) / 2

// Per-wave LDS buffers of 3 (p + 1) expansion coefficients (L2P and M2P),
// in the dynamic shared memory of the tile kernels (tile_coef_bytes).
__device__ inline cpx<double>* tile_coef(int p, int tid) {
    extern __shared__ cpx<double> tile_dyn[];
    return tile_dyn + (size_t)(tid / kWave) * 3 * (p + 1);
}
inline size_t tile_coef_bytes(int nt, int p) {
    return (size_t)(nt / kWave) * 3 * (p + 1) * sizeof(cpx<double>);
}

// Near-set traversal of a target tile by one wave (lane = lane of wave 0),
// one round: pops boxes from the stack top in chunks of up to 64, sends
// leaves to U (target-from-source), non-touching children of internal
// boxes to W (target-from-outgoing) and pushes touching children.  Chunks
// shrink to one box when the stack nears its capacity, so it never
// overflows: from then on every push is a child of the box just popped,
// which bounds the growth by 3 per level.  The round ends when the stack is
// empty or U or W is full; the order is fixed by the tree alone.
template <typename T, int NT>
__device__ void tile_round(TileShared<T, NT>& sh, const TreeView& tv, int l, long long ti,
                           long long tj, int lane) {
    int size = sh.nQ, nU = 0, nW = 0;
    for (;;) {
        int chunk = size + 3 * kWave + 3 * kMaxLevels <= kQCap ? min(kWave, size) : min(1, size);
        chunk = min(chunk, min(kUCap - nU, (kWCap - nW) / 4));
        if (chunk <= 0) break;
        const int b0 = size - chunk;
        int c = -1, ch0 = -1, isU = 0, wm = 0, fm = 0;
        if (lane < chunk) {
            c = sh.Q[b0 + lane];
            // one round of loads: the children's cells follow from c's
            // (child q is at (2 ix + (q & 1), 2 iy + (q >> 1)) one level down)
            ch0 = tv.child[c];
            const int cm = tv.cmask[c], lc = tv.lvl[c];
            const long long cx = tv.ix[c], cy = tv.iy[c];
            if (ch0 < 0) {
                isU = 1;
            } else {
                for (int q = 0; q < 4; ++q) {
                    if (!((cm >> q) & 1)) continue;  // no pieces below
                    if (touches_at(lc + 1, 2 * cx + (q & 1), 2 * cy + (q >> 1), l, ti, tj))
                        fm |= 1 << q;
                    else
                        wm |= 1 << q;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        const unsigned long long um = __ballot(isU);
        if (isU) sh.U[nU + __popcll(um & ((1ULL << lane) - 1ULL))] = c;
        int wtot, ftot;
        int wp = nW + wave_excl_scan(__popc(wm), lane, wtot);
        int fp = b0 + wave_excl_scan(__popc(fm), lane, ftot);
        for (int q = 0; q < 4; ++q) {
            if ((wm >> q) & 1) sh.W[wp++] = ch0 + q;
            if ((fm >> q) & 1) sh.Q[fp++] = ch0 + q;
        }
        nU += __popcll(um);
        nW += wtot;
        size = b0 + ftot;
        __builtin_amdgcn_wave_barrier();
    }
    // piece offsets of the U leaves
    int run = 0;
    for (int b = 0; b < nU; b += kWave) {
        const int u = b + lane;
        const int cnt = u < nU ? tv.pend[sh.U[u]] - tv.pbeg[sh.U[u]] : 0;
        int tot;
        const int ex = wave_excl_scan(cnt, lane, tot);
        if (u < nU) sh.Upre[u] = run + ex;
        run += tot;
    }
    if (lane == 0) {
        sh.Upre[nU] = run;
        sh.nU = nU;
        sh.nW = nW;
        sh.nQ = size;
    }
}

// Hardware dispatch places block b on XCD b % 8; renumber blocks so that
// each XCD receives one contiguous run of tiles (neighbouring tiles share
// their near pieces, which then stay in that XCD's L2).
__device__ inline int xcd_block(int b, int nb) {
    constexpr int kXcd = 8;
    const int x = b % kXcd, q = nb / kXcd, rmd = nb % kXcd;
    return x * q + min(x, rmd) + b / kXcd;
}

// ------------------------------------------- split render downward pass
// The render's downward pass in three steps whose launches do not depend on
// the tree depth: near sets of every target box of every level at once
// (k_near_all), each box's own incoming terms (M2L over its interaction
// list and P2L over its bigger separated list, from its parent's near set)
// at once (k_down_contrib), then one light launch per level adding the
// parent's translated expansion (L2L) and recording the owners of quiet
// boxes (k_down_l2l).  Coarse levels, whose few boxes each run a long chain
// of dependent loads, then overlap with the finer ones in one launch.

// Cell and parent of global box b, which lies in level-table entry at.
__device__ inline const VpLevel& box_at(const VpLevel* __restrict__ lev, int at, int b,
                                        long long& ti, long long& tj, int& par) {
    const VpLevel& e = lev[at];
    const int rel = b - e.off;
    ti = e.i0 + rel % e.wl;
    tj = e.j0 + rel / e.wl;
    par = e.poff + (int)((ti >> 1) - e.pi0) + (int)((tj >> 1) - e.pj0) * e.pwl;
    return e;
}

// Level-table entry, cell and parent of global box b (entries sorted by off).
__device__ inline const VpLevel& box_entry(const VpLevel* __restrict__ lev, int n_ent, int b,
                                           long long& ti, long long& tj, int& par) {
    int lo = 0, hi = n_ent - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lev[mid].off <= b) lo = mid; else hi = mid - 1;
    }
    return box_at(lev, lo, b, ti, tj, par);
}

// Level-table entries whose first-box offsets k_near_all stages in LDS (a
// longer table is searched in memory).
constexpr int kNearOffs = 1024;

// Near set of box b, cell s (one thread each): the deepest source box at a
// level <= l covering the cell, found by descending the source tree from
// its root along the cell's path, or -1 where that box holds no pieces or
// the cell lies outside the root.  (The same sets as the level-by-level
// construction of down_body.)
__global__ void __launch_bounds__(256)
k_near_all(TreeView tv, const VpLevel* __restrict__ lev, int n_ent, int total,
           int* __restrict__ nset) {
    __shared__ int offs[kNearOffs];
    const bool staged = n_ent <= kNearOffs;
    if (staged)
        for (int i = threadIdx.x; i < n_ent; i += blockDim.x) offs[i] = lev[i].off;
    __syncthreads();
    const long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= 9LL * total) return;
    const int b = (int)(gi / 9), s = (int)(gi - 9LL * b);
    long long ti, tj;
    int par;
    int at = 0;
    if (staged) {
        int lo = 0, hi = n_ent - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (offs[mid] <= b) lo = mid; else hi = mid - 1;
        }
        at = lo;
    }
    const VpLevel& e = staged ? box_at(lev, at, b, ti, tj, par)
                              : box_entry(lev, n_ent, b, ti, tj, par);
    const int l = e.level;
    const long long px = ti + (s % 3) - 1, py = tj + (s / 3) - 1;
    const long long lim = 1LL << l;
    int c = -1;
    if (px >= 0 && py >= 0 && px < lim && py < lim) {
        c = 0;
        for (int d = 0; d < l; ++d) {
            const int ch = tv.child[c];
            if (ch < 0) break;  // a coarser leaf covers the cell
            const int sh = l - d - 1;
            const int q = (int)((px >> sh) & 1) + 2 * (int)((py >> sh) & 1);
            if (!((tv.cmask[c] >> q) & 1)) {
                c = -1;  // that child holds no pieces
                break;
            }
            c = ch + q;
        }
        if (c >= 0 && tv.npc[c] == 0) c = -1;
    }
    nset[(size_t)b * 9 + s] = c;
}

// Own incoming terms of every non-root target box (one wave each): C[b] =
// M2L + P2L from its parent's near set; quiet[b] = 1 (and C[b] unwritten)
// when that near set holds no pieces.
// Waves per SIMD the kernel is compiled for (its register budget): in
// FP32, 5 (96 VGPRs, with a few spills) measured 17 us faster than 4 (115
// VGPRs) on the 2048^2 render, and 6 (80 VGPRs) slower; in FP64 4 (127
// VGPRs): with 5 the spills cost more than the extra waves win.
template <typename T>
constexpr int kContribWaves = sizeof(T) == 4 ? 5 : 4;

template <typename T, bool Count>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kContribWaves<T>)))
k_down_contrib(TreeView tv, PieceView pv, int p, const cpx<double>* __restrict__ M,
               cpx<double>* __restrict__ C, int* __restrict__ nset,
               const cpx<double>* __restrict__ Ttab, const VpLevel* __restrict__ lev, int n_ent,
               int first_box, unsigned char* __restrict__ quiet, unsigned long long* stats) {
    __shared__ DownShared<T, 1> sh;
    const int lane = threadIdx.x;
    const int b = first_box + xcd_block((int)blockIdx.x, (int)gridDim.x);
    long long ti, tj;
    int par;
    const VpLevel& e = box_entry(lev, n_ent, b, ti, tj, par);
    const bool q = down_body<T, Count, 1, true>(sh, tv, pv, e.level, ti, tj, b, par, p, M, C,
                                                nset, Ttab, nullptr, stats, lane);
    if (lane == 0) quiet[b] = q ? 1 : 0;
}

// Boxes of a level up to which k_down_l2l loads ahead of its flags.
constexpr int kL2LAhead = 8192;

// One level of the split pass (G = 64 / (p + 1) boxes per wave, lane k of
// a group = coefficient k): L[b] = C[b] + L2L(L[parent]) (Eq. i-f-i,
// scaled; the same recurrence as down_body's) with owner[b] = (b, l); a
// quiet box records its parent's owner instead (the nearest ancestor that
// is not quiet).
template <typename T>
__global__ void __launch_bounds__(kWave)
k_down_l2l(DownLevel dl, int n_boxes, int p, const cpx<double>* __restrict__ C,
           cpx<double>* __restrict__ L, const unsigned char* __restrict__ quiet,
           int2* __restrict__ owner) {
    __shared__ cpx<T> pl[3 * kWave];  // the groups' parent expansions
    const int lane = threadIdx.x, P1 = p + 1;
    const int G = kWave / P1;
    const int g = lane / P1, k = lane - g * P1;
    const int bi = (int)blockIdx.x * G + g;
    long long ti = 0, tj = 0;
    int own = 0, par = 0;
    bool work = false;
    const bool box = g < G && bi < n_boxes;
    if (box) {
        const VpLevel& e = find_entry(dl.vl, dl.nvl, bi);
        const int bb = bi - e.first_block;
        ti = e.i0 + bb % e.wl;
        tj = e.j0 + bb / e.wl;
        own = e.off + bb;
        par = e.poff + (int)((ti >> 1) - e.pi0) + (int)((tj >> 1) - e.pj0) * e.pwl;
    }
    // On levels with few boxes, whose launches are one chain of dependent
    // loads, every load of a box is issued at once: the parent's owner, the
    // quiet flag, the box's own terms and the parent's expansion (the last
    // two lie inside C and L whatever the flags say, and are used only when
    // the box works: its parent's L and its own C are then written).  On
    // the larger levels, where most boxes are quiet, the terms are loaded
    // only for working boxes.
    const bool ahead = n_boxes <= kL2LAhead;
    int2 po = make_int2(0, 0);
    unsigned char qb = 1;
    cpx<double> cv[3], lv[3];
    if (box) {
        po = owner[par];
        qb = quiet[own];
        if (ahead) {
            for (int ch = 0; ch < 3; ++ch) cv[ch] = C[((size_t)own * P1 + k) * 3 + ch];
            for (int t = 0; t < 3; ++t) lv[t] = L[(size_t)par * 3 * P1 + k + t * P1];
        }
        work = po.x == par && !qb;
        if (k == 0) owner[own] = work ? make_int2(own, dl.l) : po;
        if (work && !ahead) {
            for (int ch = 0; ch < 3; ++ch) cv[ch] = C[((size_t)own * P1 + k) * 3 + ch];
            for (int t = 0; t < 3; ++t) lv[t] = L[(size_t)par * 3 * P1 + k + t * P1];
        }
    }
    cpx<T>* src = pl + g * 3 * P1;
    if (work)
        for (int t = 0; t < 3; ++t) src[k + t * P1] = to_c<T>(lv[t].re, lv[t].im);
    __syncthreads();
    if (!work) return;
    cpx<T> acc[3];
    for (int ch = 0; ch < 3; ++ch) acc[ch] = to_c<T>(cv[ch].re, cv[ch].im);
    const cpx<T> z0 = {(T)((ti & 1) ? 0.5 : -0.5), (T)((tj & 1) ? 0.5 : -0.5)};
    cpx<T> pw = {1, 0};
    T binom = 1;
    const T sc = (T)ldexp(1.0, -k);
    for (int j = 0; j <= p - k; ++j) {  // j = m - k: the same in every lane
        const int m = k + j;
        const cpx<T> f = cscale(pw, binom * sc);
        for (int ch = 0; ch < 3; ++ch) acc[ch] = cadd(acc[ch], cmul(f, src[m * 3 + ch]));
        binom = binom * (T)(m + 1) * recip<T>(j + 1);
        pw = cmul(pw, z0);
    }
    cpx<double>* out = L + ((size_t)own * P1 + k) * 3;
    for (int ch = 0; ch < 3; ++ch) out[ch] = {(double)acc[ch].re, (double)acc[ch].im};
}

// The solve's downward pass split the same way, over the source cells
// (the targets are the cells themselves): near sets of every cell at once,
// every cell's own incoming terms at once, then one light L2L launch per
// level.  The solve's cells are never quiet in practice (a cell's parent's
// near set holds the cell itself); a quiet one would get its parent's
// translated expansion alone.

// Near set of cell c (levels >= 1), position s: as k_near_all.
__global__ void __launch_bounds__(256)
k_near_cells(TreeView tv, int first_cell, int n, int* __restrict__ nset) {
    const long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= 9LL * n) return;
    const int c = first_cell + (int)(gi / 9), s = (int)(gi % 9);
    const int l = tv.lvl[c];
    const long long px = tv.ix[c] + (s % 3) - 1, py = tv.iy[c] + (s / 3) - 1;
    const long long lim = 1LL << l;
    int b = -1;
    if (px >= 0 && py >= 0 && px < lim && py < lim) {
        b = 0;
        for (int d = 0; d < l; ++d) {
            const int ch = tv.child[b];
            if (ch < 0) break;  // a coarser leaf covers the cell
            const int sh = l - d - 1;
            const int q = (int)((px >> sh) & 1) + 2 * (int)((py >> sh) & 1);
            if (!((tv.cmask[b] >> q) & 1)) {
                b = -1;  // that child holds no pieces
                break;
            }
            b = ch + q;
        }
        if (b >= 0 && tv.npc[b] == 0) b = -1;
    }
    nset[(size_t)c * 9 + s] = b;
}

// Own incoming terms C[c] (M2L + P2L from the parent's near set) of every
// cell at levels >= 1, one wave each; quiet[c] = 1 (C[c] unwritten) when
// that near set holds no pieces.
template <typename T>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kContribWaves<T>)))
k_down_contrib_cells(TreeView tv, PieceView pv, int p, const cpx<double>* __restrict__ M,
                     cpx<double>* __restrict__ C, int* __restrict__ nset,
                     const cpx<double>* __restrict__ Ttab, int first_cell,
                     unsigned char* __restrict__ quiet) {
    __shared__ DownShared<T, 1> sh;
    const int lane = threadIdx.x;
    const int c = first_cell + xcd_block((int)blockIdx.x, (int)gridDim.x);
    const bool q = down_body<T, false, 1, true>(sh, tv, pv, tv.lvl[c], tv.ix[c], tv.iy[c], c,
                                                tv.parent[c], p, M, C, nset, Ttab, nullptr,
                                                nullptr, lane);
    if (lane == 0) quiet[c] = q ? 1 : 0;
}

// One level of the solve's L2L (G = 64 / (p + 1) cells per wave, lane k
// of a group = coefficient k): L[c] = C[c] + L2L(L[parent]) in FP64
// (Eq. i-f-i, scaled).
__global__ void __launch_bounds__(kWave)
k_l2l_cells(TreeView tv, int first_cell, int n_cells, int p, const cpx<double>* __restrict__ C,
            cpx<double>* __restrict__ L, const unsigned char* __restrict__ quiet) {
    __shared__ cpx<double> pl[3 * kWave];  // the groups' parent expansions
    const int lane = threadIdx.x, P1 = p + 1;
    const int G = kWave / P1;
    const int g = lane / P1, k = lane - g * P1;
    const int ci = (int)blockIdx.x * G + g;
    const bool work = g < G && ci < n_cells;
    const int c = first_cell + (work ? ci : 0);
    // everything but the parent's expansion in one round of loads (the own
    // terms lie inside C whether or not the cell is quiet, and are used only
    // when it is not: then they are written)
    const int par = tv.parent[c];
    const bool qc = quiet[c] != 0;
    const long long cix = tv.ix[c], ciy = tv.iy[c];
    cpx<double> own[3];
    for (int ch = 0; ch < 3; ++ch) own[ch] = C[((size_t)c * P1 + k) * 3 + ch];
    cpx<double>* src = pl + g * 3 * P1;
    if (work)
        for (int i = k; i < 3 * P1; i += P1) src[i] = L[(size_t)par * 3 * P1 + i];
    __syncthreads();
    if (!work) return;
    cpx<double> acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    if (!qc)
        for (int ch = 0; ch < 3; ++ch) acc[ch] = own[ch];
    const cpx<double> z0 = {(cix & 1) ? 0.5 : -0.5, (ciy & 1) ? 0.5 : -0.5};
    cpx<double> pw = {1, 0};
    double binom = 1;
    const double sc = ldexp(1.0, -k);
    for (int j = 0; j <= p - k; ++j) {  // j = m - k: the same in every lane
        const int m = k + j;
        const cpx<double> f = cscale(pw, binom * sc);
        for (int ch = 0; ch < 3; ++ch) acc[ch] = cadd(acc[ch], cmul(f, src[m * 3 + ch]));
        binom = binom * (double)(m + 1) * recip<double>(j + 1);
        pw = cmul(pw, z0);
    }
    cpx<double>* out = L + ((size_t)c * P1 + k) * 3;
    for (int ch = 0; ch < 3; ++ch) out[ch] = acc[ch];
}

struct Rgb {
    double v[3];
};

// One (pixel, piece) pair of the near field in FP64 (App. D), weighted for
// the three channels.  Out of line: the FP32 render path calls it only for
// the rare near-singular and heavy pairs, and inlined it would set the
// register budget of the whole tile kernel.
__device__ __noinline__ Rgb pair_fp64(const double* __restrict__ x0, const double* __restrict__ y0,
                                      const double* __restrict__ tx, const double* __restrict__ ty,
                                      const double* __restrict__ len,
                                      const double* __restrict__ w64, int n, int e, double x,
                                      double y) {
    double il, th;
    chord_log_theta<double>(x0[e] - x, y0[e] - y, tx[e], ty[e], len[e], il, th);
    Rgb r;
    for (int ch = 0; ch < 3; ++ch)
        r.v[ch] = il * w64[(size_t)ch * n + e] + th * w64[(size_t)(3 + ch) * n + e];
    return r;
}

// Render leaf pass (Alg. 4 at pixel tiles), PX pixels per thread: each
// piece staged in LDS is read once and evaluated against PX pixels, which
// gives every lane PX independent chains of the closed forms.  Same
// arithmetic per (pixel, source) pair as k_leaf; targets are pixels only.
// A tile (target box own, level l, cell (ti, tj) of viewport v, pixels
// [k_lo, k_lo + nx) x [r_lo, r_lo + ny)) is evaluated by one block of NT
// threads: S groups of G = NT / S threads, each group on the same G * PX
// pixels per pass.  The separated boxes are numbered in traversal order and
// group g takes those with number % S == g, and every S-th piece of each
// staged chunk; the value of a pixel is L2P plus the group partial sums,
// added in group order.  A small tile whose first traversal round finds
// more than kHeavyPieces<T> near pieces, or leaves more rounds to come, is
// queued by k_tile_scan and evaluated by k_tile_big (on a second stream,
// concurrently with k_tile), whose blocks split one tile's near field over
// kBigSplit<T> waves.
// Waves per SIMD the one-wave tile kernel is compiled for (its register
// budget, measured best): 4 (FP32 116 VGPRs; FP64 128).  5 in FP32 (96
// VGPRs, 18 spilled) measured a slower leaf pass (0.352 against 0.344 ms).
template <typename T>
constexpr int kTileWaves = 4;
template <typename T>
constexpr int kHeavyPieces = sizeof(T) == 4 ? 128 : 32;
template <typename T>
constexpr int kBigSplit = sizeof(T) == 4 ? 8 : 4;
constexpr int kBigBlocks = 512;  // grid of k_tile_big
// A small tile's traversal lists, kept by k_tile_scan when its first round
// is its only one and finds at most kListW separated boxes (a round never
// holds more than kUCap near leaves), so that k_tile or k_tile_big need not
// repeat the traversal.  Record of kListInts ints per tile: nU, nW,
// U[kListU], Upre[kListU + 1], W[kListW], one int of padding.
constexpr int kListU = kUCap, kListW = 64;
constexpr int kListInts = 2 + kListU + (kListU + 1) + kListW + 1;

// A kept record, loaded into registers (this thread's slots) when a tile's
// evaluation starts, so that the loads overlap the expansion's.
template <int NT>
struct KeptLists {
    static constexpr int kRec = kListInts - 2, kPer = (kRec + NT - 1) / NT;
    int val[kPer];
    int nU = 0, nW = 0;
    bool on = false;
    __device__ void load(const int* rec, int tid) {
        on = rec != nullptr;
        if (!on) return;
        for (int j = 0; j < kPer; ++j) {
            const int i = tid + j * NT;
            val[j] = i < kRec ? rec[2 + i] : 0;
        }
        nU = rec[0];
        nW = rec[1];
    }
};
constexpr int kOverlapTiles = 65536;  // renders with this many tiles overlap k_tile_big
constexpr int kDeepBoxes = 2048;  // render levels below this many boxes use k_down<.., 3>
// Render downward pass: one persistent launch over every level (else one
// k_down launch per level).
constexpr bool kPersistentDown = false;
// Render downward pass split into near sets, own incoming terms and a
// per-level L2L (else one k_down launch per level).
constexpr bool kSplitDown = true;

template <typename T, int PX>
struct TileTargets {
    double x[PX], y[PX];
    T xr[PX], yr[PX];
    bool act[PX];
    int out_idx[PX];
};

// Pixels of one pass (targets tbase + q G + gt of the tile, row-major).
template <typename T, int PX, int G>
__device__ inline void tile_targets(TileTargets<T, PX>& tt, const VpLeaf& v, double cx,
                                    double cy, int k_lo, int nx, int r_lo, int n_targets,
                                    int tbase, int gt) {
    for (int q = 0; q < PX; ++q) {
        const int tgt = tbase + q * G + gt;
        tt.act[q] = tgt < n_targets;
        tt.x[q] = cx;
        tt.y[q] = cy;
        tt.out_idx[q] = 0;
        if (tt.act[q]) {
            const int col = k_lo + tgt % nx, row = r_lo + tgt / nx;
            tt.x[q] = pixel_x(v.vcx, v.vw, v.W, col);
            tt.y[q] = pixel_y(v.vcy, v.vh, v.H, row);
            tt.out_idx[q] = row * v.W + col;
        }
        tt.xr[q] = (T)(tt.x[q] - cx);
        tt.yr[q] = (T)(tt.y[q] - cy);
    }
}

// Copy of n expansion coefficients into this wave's LDS buffer (one
// coalesced load per lane; LDS accesses of one wave complete in order, so
// the wave reads them back without a block barrier).
__device__ inline void stage_coef(cpx<double>* __restrict__ buf, const cpx<double>* __restrict__ src,
                                  int n, int lane) {
    for (int i = lane; i < n; i += kWave) buf[i] = src[i];
    __builtin_amdgcn_wave_barrier();
}

// target-from-incoming (Eq. t-f-i) at the pass's pixels: Re sum_k ((x-c)/r)^k Lt_k
// of the owner's expansion (loc at level lo, centre (ocx, ocy)); adds into acc.
// cbuf: this wave's coefficient buffer.
template <typename T, int PX>
__device__ inline void tile_l2p(const TileTargets<T, PX>& tt, const cpx<double>* loc, int p,
                                int lo, double ro, double ocx, double ocy, cpx<double>* cbuf,
                                int lane, double (&acc)[PX][3]) {
    if (lo < 2) return;
    const double ir = 1.0 / ro;
    if constexpr (sizeof(T) == 4) {
        // FP32 path: the stored FP64 expansion evaluated in FP32 (|z| < 1.5)
        cpx<float>* fbuf = reinterpret_cast<cpx<float>*>(cbuf);
        for (int i = lane; i < (p + 1) * 3; i += kWave)
            fbuf[i] = {(float)loc[i].re, (float)loc[i].im};
        __builtin_amdgcn_wave_barrier();
        for (int q = 0; q < PX; ++q) {
            const cpx<float> z = {(float)((tt.x[q] - ocx) * ir), (float)((tt.y[q] - ocy) * ir)};
            for (int ch = 0; ch < 3; ++ch) {
                cpx<float> s = fbuf[p * 3 + ch];
                for (int kk = p - 1; kk >= 0; --kk) s = cadd(cmul(s, z), fbuf[kk * 3 + ch]);
                acc[q][ch] += (double)s.re;
            }
        }
    } else {
        stage_coef(cbuf, loc, (p + 1) * 3, lane);
        for (int q = 0; q < PX; ++q) {
            const cpx<double> z = {(tt.x[q] - ocx) * ir, (tt.y[q] - ocy) * ir};
            for (int ch = 0; ch < 3; ++ch) {
                cpx<double> s = cbuf[p * 3 + ch];
                for (int kk = p - 1; kk >= 0; --kk) s = cadd(cmul(s, z), cbuf[kk * 3 + ch]);
                acc[q][ch] += s.re;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Traversal stack of a tile: the distinct nonempty cells of its near set.
template <typename T, int NT>
__device__ inline void tile_near_init(TileShared<T, NT>& sh, const TreeView& tv,
                                      const int* __restrict__ nset, int own, int tid) {
    if (tid < kWave) {
        int c = -1;
        bool ok = false;
        if (tid < 9) {
            c = nset[(size_t)own * 9 + tid];
            ok = c >= 0;
            for (int s2 = 0; s2 < tid && ok; ++s2) ok = nset[(size_t)own * 9 + s2] != c;
        }
        const unsigned long long m = __ballot(ok);
        if (ok) sh.Q[__popcll(m & ((1ULL << tid) - 1ULL))] = c;
        if (tid == 0) sh.nQ = __popcll(m);
    }
}

// The expansion a tile evaluates (its own, or its owner's when quiet).
struct TileOwner {
    const cpx<double>* loc;
    int lo;
    double ro, ocx, ocy;
    bool quiet;
};

// Near field of a tile pass (see above): near-set traversal by wave 0 in
// rounds bounded by the list capacities (the stack starts with the
// distinct nonempty cells of the near set), then the round's separated boxes
// (target-from-outgoing) and near pieces (target-from-source) of this
// thread's group.  Adds the group's terms into acc.
template <typename T, int NT, int PX, int S, bool Count>
__device__ void tile_near(TileShared<T, NT>& sh, const TreeView& tv, const PieceView& pv,
                          const LeafArgs& a, int p, const cpx<double>* __restrict__ Ms,
                          const int* __restrict__ nset, int l, long long ti, long long tj,
                          int own, double cx, double cy, const TileTargets<T, PX>& tt,
                          const TileOwner* l2p, const KeptLists<NT>& kl, int n_here, int tid,
                          double (&acc)[PX][3]) {
    constexpr int G = NT / S;
    const int gid = tid / G, gt = tid - gid * G;
    const T* wts = weights<T>(pv);
    // half width of the tile's box (pixel centres lie inside it)
    const float rtile = (float)half_width(tv, l);
    if (kl.on) {
        // the lists of the only round, as k_tile_scan's tile_round left them
        const int nU = kl.nU, nW = kl.nW;
        for (int j = 0; j < KeptLists<NT>::kPer; ++j) {
            const int i = tid + j * NT;
            if (i < kListU) {
                if (i < nU) sh.U[i] = kl.val[j];
            } else if (i < 2 * kListU + 1) {
                if (i - kListU <= nU) sh.Upre[i - kListU] = kl.val[j];
            } else if (i < 2 * kListU + 1 + kListW) {
                if (i - 2 * kListU - 1 < nW) sh.W[i - 2 * kListU - 1] = kl.val[j];
            }
        }
        if (tid == 0) {
            sh.nU = nU;
            sh.nW = nW;
            sh.nQ = 0;
        }
    } else {
        tile_near_init(sh, tv, nset, own, tid);
    }
    __syncthreads();
    int u_run = 0;
    bool first = true;
    for (;;) {
        if (tid < kWave) {
            if (!(first && kl.on)) tile_round(sh, tv, l, ti, tj, tid);
        }
        if (tid >= kWave && first && l2p != nullptr && gid == 1)  // beside wave 0's first round
            tile_l2p<T, PX>(tt, l2p->loc, p, l2p->lo, l2p->ro, l2p->ocx, l2p->ocy,
                            tile_coef(p, tid), tid % kWave, acc);
        first = false;
        __syncthreads();
        const int nU = sh.nU, nW = sh.nW, more = sh.nQ > 0;
        // target-from-outgoing (Eq. t-f-o), scaled:
        //   Re[-log(x - c) Mt_0 + sum_{k>=1} (1/k) (r/(x-c))^k Mt_k]
        // with Ms_k = Mt_k / k precomputed; Mt_0 (the total charge times
        // length) is real, so only log|x - c| is needed
        cpx<double>* const src = tile_coef(p, tid);
        for (int u = ((gid - u_run) % S + S) % S; u < nW; u += S) {
            const int d = sh.W[u];
            stage_coef(src, Ms + (size_t)d * (p + 1) * 3, (p + 1) * 3, tid % kWave);
            const int ld = tv.lvl[d];
            const double rd = half_width(tv, ld), ird = 1.0 / rd;
            double dcx, dcy;
            center_of(tv, ld, tv.ix[d], tv.iy[d], dcx, dcy);
            const double lr = log(rd);
            for (int q = 0; q < PX; ++q) {
                if (!tt.act[q]) continue;
                const cpx<double> rel = {(tt.x[q] - dcx) * ird, (tt.y[q] - dcy) * ird};
                const double n2 = rel.re * rel.re + rel.im * rel.im;
                const double in2 = 1.0 / n2;
                const cpx<double> z = {rel.re * in2, -rel.im * in2};
                const double lgr = lr + 0.5 * log(n2);
                for (int ch = 0; ch < 3; ++ch) {
                    cpx<double> s = src[p * 3 + ch];
                    for (int kk = p - 1; kk >= 1; --kk) s = cadd(cmul(s, z), src[kk * 3 + ch]);
                    s = cmul(s, z);
                    acc[q][ch] += s.re - lgr * src[ch].re;
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (Count && gt == 0) atomicAdd(a.stats + kStatM2P, (unsigned long long)n_here);
        }
        u_run += nW;
        // target-from-source (App. D) over the pieces of the near leaves
        const int total = sh.Upre[nU];
        for (int pbase = 0; pbase < total; pbase += NT) {
            __syncthreads();
            const int g = pbase + tid;
            if (g < total) {
                int lo = 0, hi = nU - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sh.Upre[mid] <= g) lo = mid; else hi = mid - 1;
                }
                const int e = tv.pbeg[sh.U[lo]] + (g - sh.Upre[lo]);
                sh.px[tid] = (T)(pv.x0[e] - cx);
                sh.py[tid] = (T)(pv.y0[e] - cy);
                sh.tx[tid] = (T)pv.tx[e];
                sh.ty[tid] = (T)pv.ty[e];
                sh.len[tid] = (T)pv.len[e];
                for (int c6 = 0; c6 < 6; ++c6) sh.w[c6][tid] = wts[(size_t)c6 * pv.n + e];
                const bool hv = sizeof(T) == 4 && pv.heavy[e];
                sh.pid[tid] = hv ? -1 - e : e;
                if constexpr (sizeof(T) == 4) {
                    // distance from the chord's midpoint to the tile's box,
                    // less half the chord, against kGaussSep chord lengths
                    const float la = (float)sh.len[tid];
                    const float mx = (float)sh.px[tid] + 0.5f * la * (float)sh.tx[tid];
                    const float my = (float)sh.py[tid] + 0.5f * la * (float)sh.ty[tid];
                    const float ex = fmaxf(fabsf(mx) - rtile, 0.f);
                    const float ey = fmaxf(fabsf(my) - rtile, 0.f);
                    const float sep = (kGaussSep + 0.5f) * la;
                    sh.far[tid] = !hv && ex * ex + ey * ey >= sep * sep ? 1 : 0;
                }
            }
            __syncthreads();
            const int m = min(NT, total - pbase);
            if (Count && tid == 0) atomicAdd(a.stats + kStatP2P, (unsigned long long)n_here * m);
            const float near2f = (float)a.near2;
            for (int j = gid; j < m; j += S) {
                const T px0 = sh.px[j], py0 = sh.py[j];
                const T tx = sh.tx[j], ty = sh.ty[j], la = sh.len[j];
                const int pid = sh.pid[j];
                if (sizeof(T) == 4 && sh.far[j]) {
                    // two-point Gauss-Legendre on the chord (a well-separated
                    // piece: uniform over the wave, no near-singular pairs)
                    const float fla = (float)la;
                    float w6[6];
                    for (int c6 = 0; c6 < 6; ++c6) w6[c6] = (float)sh.w[c6][j];
                    for (int q = 0; q < PX; ++q) {
                        const float dx = (float)(px0 - tt.xr[q]), dy = (float)(py0 - tt.yr[q]);
                        const float xi1 = dx * (float)tx + dy * (float)ty;
                        const float h = dy * (float)tx - dx * (float)ty;
                        const float xa = xi1 + kGaussA * fla, xb = xi1 + kGaussB * fla;
                        const float ra = xa * xa + h * h, rb = xb * xb + h * h;
                        const float il = 0.25f * fla * fast_ln(ra * rb);
                        const float th = 0.5f * fla * h *
                                         (__builtin_amdgcn_rcpf(ra) + __builtin_amdgcn_rcpf(rb));
                        for (int ch = 0; ch < 3; ++ch)
                            acc[q][ch] -= (double)(il * w6[ch] + th * w6[3 + ch]);
                    }
                    continue;
                }
                if (sizeof(T) == 8) {
                    for (int q = 0; q < PX; ++q) {
                        T il, th;
                        chord_log_theta<T>(px0 - tt.xr[q], py0 - tt.yr[q], tx, ty, la, il, th);
                        for (int ch = 0; ch < 3; ++ch)
                            acc[q][ch] -= il * sh.w[ch][j] + th * sh.w[3 + ch][j];
                    }
                    continue;
                }
                // FP32: the fast closed form for every pixel, straight-line
                // so the PX chains interleave; near-singular pairs and heavy
                // pieces are then redone in FP64 (rare, divergent)
                float il[PX], th[PX];
                bool slow[PX];
                bool any_slow = false;
                const float fla = (float)la, lim = near2f * fla * fla;
                for (int q = 0; q < PX; ++q) {
                    const float dx = (float)(px0 - tt.xr[q]), dy = (float)(py0 - tt.yr[q]);
                    const float xi1 = dx * (float)tx + dy * (float)ty;
                    const float h = dy * (float)tx - dx * (float)ty;
                    const float xi2 = xi1 + fla;
                    // squared distance to the chord, branch-free
                    const float along = fmaxf(xi1, 0.f) + fmaxf(-xi2, 0.f);
                    slow[q] = along * along + h * h < lim || pid < 0;
                    any_slow |= slow[q] && tt.act[q];
                    chord_fast_nz(xi1, h, xi2, fla, il[q], th[q]);
                }
                float w6[6];
                for (int c6 = 0; c6 < 6; ++c6) w6[c6] = (float)sh.w[c6][j];
                for (int q = 0; q < PX; ++q)
                    for (int ch = 0; ch < 3; ++ch) {
                        const float t = il[q] * w6[ch] + th[q] * w6[3 + ch];
                        acc[q][ch] -= (double)(slow[q] ? 0.f : t);
                    }
                if (any_slow) {
                    const int e = pid < 0 ? -1 - pid : pid;
                    for (int q = 0; q < PX; ++q) {
                        if (!(slow[q] && tt.act[q])) continue;
                        const Rgb d = pair_fp64(pv.x0, pv.y0, pv.tx, pv.ty, pv.len, pv.w64,
                                                pv.n, e, tt.x[q], tt.y[q]);
                        for (int ch = 0; ch < 3; ++ch) acc[q][ch] -= d.v[ch];
                        if (Count) atomicAdd(a.stats + kStatP2P64, 1ULL);
                    }
                }
            }
        }
        __syncthreads();
        if (!more) break;
    }
}

// Adds the partial sums of groups 1..S-1 to group 0's, in group order
// (through the staging arrays; every thread of the block calls it).
template <typename T, int NT, int PX, int S>
__device__ inline void tile_group_sum(TileShared<T, NT>& sh, int tid, double (&acc)[PX][3]) {
    if (S == 1) return;
    constexpr int G = NT / S;
    using Sh = TileShared<T, NT>;
    static_assert((S - 1) * 3 * G * sizeof(double) <= offsetof(Sh, U) - offsetof(Sh, px),
                  "partial sums of one pixel slot fit the staging");
    const int gid = tid / G, gt = tid - gid * G;
    double* red = reinterpret_cast<double*>(sh.px);
    for (int q = 0; q < PX; ++q) {
        __syncthreads();
        if (gid > 0)
            for (int ch = 0; ch < 3; ++ch) red[((size_t)(gid - 1) * 3 + ch) * G + gt] = acc[q][ch];
        __syncthreads();
        if (gid == 0)
            for (int g2 = 1; g2 < S; ++g2)
                for (int ch = 0; ch < 3; ++ch) acc[q][ch] += red[((size_t)(g2 - 1) * 3 + ch) * G + gt];
    }
    __syncthreads();
}

// u / 2pi at the pass's pixels (group 0 holds the sums).
template <typename T, int PX>
__device__ inline void tile_store(const LeafArgs& a, const VpLeaf& v, const TileTargets<T, PX>& tt,
                                  bool group0, const double (&acc)[PX][3]) {
    for (int q = 0; q < PX; ++q) {
        if (!tt.act[q] || !group0) continue;
        for (int ch = 0; ch < 3; ++ch) {
            const double u = acc[q][ch] / kTwoPi;
            if (a.out_f64)
                static_cast<double*>(v.out)[(size_t)tt.out_idx[q] * 3 + ch] = u;
            else
                static_cast<float*>(v.out)[(size_t)tt.out_idx[q] * 3 + ch] = (float)u;
        }
    }
}

// Geometry of a tile's owner expansion (quiet tiles evaluate an ancestor's).
__device__ inline TileOwner tile_owner(const TreeView& tv, const cpx<double>* Lc,
                                       const int2* owner, int p, int l, long long ti,
                                       long long tj, int own) {
    TileOwner o;
    const int2 ow = owner[own];
    o.quiet = ow.x != own;
    o.loc = Lc + (size_t)ow.x * (p + 1) * 3;
    o.lo = ow.y;
    o.ro = half_width(tv, o.lo);
    center_of(tv, o.lo, ti >> (l - o.lo), tj >> (l - o.lo), o.ocx, o.ocy);
    return o;
}

// Leaf evaluation of one tile by one block.
template <typename T, int NT, int PX, int S, bool Count>
__device__ void tile_body(TileShared<T, NT>& sh, const TreeView& tv, const PieceView& pv,
                          const LeafArgs& a, int p, const cpx<double>* __restrict__ Ms,
                          const cpx<double>* __restrict__ Lc, const int* __restrict__ nset,
                          const int2* __restrict__ owner, const VpLeaf& v, int l, long long ti,
                          long long tj, int own, int k_lo, int nx, int r_lo, int ny, int tid,
                          const int* lists) {
    static_assert(NT % S == 0 && (S == 1 || (NT / S) % kWave == 0), "split groups are waves");
    constexpr int G = NT / S;
    const int gid = tid / G, gt = tid - gid * G;
    const int n_targets = nx > 0 ? nx * ny : 0;
    double cx, cy;
    center_of(tv, l, ti, tj, cx, cy);
    KeptLists<NT> kl;
    kl.load(lists, tid);
    const TileOwner o = tile_owner(tv, Lc, owner, p, l, ti, tj, own);
    for (int tbase = 0; tbase < n_targets; tbase += G * PX) {
        TileTargets<T, PX> tt;
        tile_targets<T, PX, G>(tt, v, cx, cy, k_lo, nx, r_lo, n_targets, tbase, gt);
        // u = (E - P) / 2pi: E from expansions, P the near field (FP64 sums)
        double acc[PX][3];
        for (int q = 0; q < PX; ++q)
            for (int ch = 0; ch < 3; ++ch) acc[q][ch] = 0.0;
        // FP64 with several groups: group 1 evaluates the expansion in
        // tile_near while wave 0 runs the first traversal round (measured
        // faster in FP64, slower in FP32).
        const bool l2p_near = sizeof(T) == 8 && S > 1 && G == kWave && !o.quiet;
        if (gid == 0 && !l2p_near)
            tile_l2p<T, PX>(tt, o.loc, p, o.lo, o.ro, o.ocx, o.ocy, tile_coef(p, tid),
                            tid % kWave, acc);
        const int n_here = min(G * PX, n_targets - tbase);
        if (Count && tid == 0) {
            if (o.lo >= 2) atomicAdd(a.stats + kStatL2P, (unsigned long long)n_here);
            if (tbase == 0) atomicAdd(a.stats + kStatLeaf, 1ULL);
        }
        if (!o.quiet)
            tile_near<T, NT, PX, S, Count>(sh, tv, pv, a, p, Ms, nset, l, ti, tj, own, cx, cy, tt,
                                           l2p_near ? &o : nullptr, kl,
                                           n_here, tid, acc);
        tile_group_sum<T, NT, PX, S>(sh, tid, acc);
        tile_store<T, PX>(a, v, tt, gid == 0, acc);
        __syncthreads();
    }
}

// Hardware dispatch places block b on XCD b % 8 (see xcd_block).
template <typename T, int NT, int PX, int S, bool Count>
__global__ void __launch_bounds__(NT)
    __attribute__((amdgpu_waves_per_eu(NT == kWave ? kTileWaves<T> : 4)))
k_tile(TreeView tv, PieceView pv, LeafArgs a, int p, const cpx<double>* __restrict__ Ms,
       const cpx<double>* __restrict__ Lc, const int* __restrict__ nset,
       const int2* __restrict__ owner) {
    const int gb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int fl = a.hv_flag != nullptr ? a.hv_flag[gb] : 0;
    if (fl == 1 || fl == 2 || fl == 4) return;  // queued, or done by k_tile_scan
    const VpLeaf& v = find_entry(a.vleaf, a.nvleaf, gb);
    const int blk = gb - v.first_block;
    __shared__ TileShared<T, NT> sh;
    const int tid = threadIdx.x;
    const int l = v.L;
    const long long ti = v.i0 + blk % v.wl, tj = v.j0 + blk / v.wl;
    const int own = v.off + blk;
    const int ci = (int)(ti - v.i0), cj = (int)(tj - v.j0);
    const int k_lo = a.edges[v.col_at + ci];
    const int nx = a.edges[v.col_at + ci + 1] - k_lo;
    const int r_lo = a.edges[v.row_at + cj + 1];
    const int ny = max(a.edges[v.row_at + cj] - r_lo, 0);
    tile_body<T, NT, PX, S, Count>(sh, tv, pv, a, p, Ms, Lc, nset, owner, v, l, ti, tj, own,
                                   k_lo, nx, r_lo, ny, tid,
                                   fl == 3 ? a.lists + (size_t)gb * kListInts : nullptr);
}

// First pass over every small tile.  A quiet tile (see k_down) is
// evaluated here (its owner's expansion at its pixels, the same arithmetic
// as in tile_body) and flagged done; a heavy one (see above) is queued for
// k_tile_big and flagged; k_tile leaves flagged tiles.  Queuing depends
// only on the tile's own traversal (every tile always takes the same
// path); the two ends of the list never meet, since it can hold every tile.
template <typename T, int MaxPx, int Heavy, bool Count>
__global__ void __launch_bounds__(kWave)
k_tile_scan(TreeView tv, LeafArgs a, int p, const cpx<double>* __restrict__ Lc,
            const int* __restrict__ nset, const int2* __restrict__ owner) {
    __shared__ TileShared<float, 1> sh;  // the traversal lists only
    const int gb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const VpLeaf& v = find_entry(a.vleaf, a.nvleaf, gb);
    const int blk = gb - v.first_block;
    const int tid = threadIdx.x;
    const int l = v.L;
    const long long ti = v.i0 + blk % v.wl, tj = v.j0 + blk / v.wl;
    const int own = v.off + blk;
    const int ci = (int)(ti - v.i0), cj = (int)(tj - v.j0);
    const int k_lo = a.edges[v.col_at + ci];
    const int nx = a.edges[v.col_at + ci + 1] - k_lo;
    const int r_lo = a.edges[v.row_at + cj + 1];
    const int ny = max(a.edges[v.row_at + cj] - r_lo, 0);
    const int n_targets = nx > 0 ? nx * ny : 0;
    int flag = 0;
    if (owner[own].x != own) {
        // quiet: no near field
        double cx, cy;
        center_of(tv, l, ti, tj, cx, cy);
        const TileOwner o = tile_owner(tv, Lc, owner, p, l, ti, tj, own);
        for (int tbase = 0; tbase < n_targets; tbase += kWave) {
            TileTargets<T, 1> tt;
            tile_targets<T, 1, kWave>(tt, v, cx, cy, k_lo, nx, r_lo, n_targets, tbase, tid);
            double acc[1][3] = {{0.0, 0.0, 0.0}};
            tile_l2p<T, 1>(tt, o.loc, p, o.lo, o.ro, o.ocx, o.ocy, tile_coef(p, tid), tid, acc);
            if (Count && tid == 0) {
                const int n_here = min(kWave, n_targets - tbase);
                if (o.lo >= 2) atomicAdd(a.stats + kStatL2P, (unsigned long long)n_here);
                if (tbase == 0) atomicAdd(a.stats + kStatLeaf, 1ULL);
            }
            tile_store<T, 1>(a, v, tt, true, acc);
        }
        flag = 2;
    } else if (n_targets > 0 && n_targets <= MaxPx) {
        tile_near_init(sh, tv, nset, own, tid);
        __syncthreads();
        tile_round(sh, tv, l, ti, tj, tid);
        __syncthreads();
        const int nU = sh.nU, nW = sh.nW, np = sh.Upre[nU];
        // lists of a tile whose first round is its only one, kept
        const bool keep = a.lists != nullptr && sh.nQ == 0 && nU <= kListU && nW <= kListW;
        if (keep) {
            int* rec = a.lists + (size_t)gb * kListInts;
            for (int i = tid; i < nU; i += kWave) rec[2 + i] = sh.U[i];
            for (int i = tid; i <= nU; i += kWave) rec[2 + kListU + i] = sh.Upre[i];
            for (int i = tid; i < nW; i += kWave) rec[3 + 2 * kListU + i] = sh.W[i];
            if (tid == 0) {
                rec[0] = nU;
                rec[1] = nW;
            }
        }
        flag = keep ? 3 : 0;
        if (np > Heavy || sh.nQ > 0) {
            if (tid == 0) {
                // the heaviest (more rounds, or 4x the pieces) from the front
                const bool front = sh.nQ > 0 || np > 4 * Heavy;
                const int h = atomicAdd(&a.hv_ctl[front ? 0 : 2], 1);
                const bool queued = h < a.hv_list_cap;
                if (queued) {
                    a.hv_list[front ? h : a.hv_list_cap - 1 - h] = gb;
                    flag = keep ? 4 : 1;
                }
            }
        }
    }
    if (tid == 0) a.hv_flag[gb] = (unsigned char)flag;
}

// Queued (heavy) tiles, one per block at a time, PX pixels per thread:
// blocks take tiles from a counter until none is left; nothing waits.
template <typename T, bool Count, int PX>
__global__ void __launch_bounds__(kWave * kBigSplit<T>)
k_tile_big(TreeView tv, PieceView pv, LeafArgs a, int p, const cpx<double>* __restrict__ Ms,
           const cpx<double>* __restrict__ Lc, const int* __restrict__ nset,
           const int2* __restrict__ owner) {
    constexpr int S = kBigSplit<T>, NT = kWave * S;
    __shared__ TileShared<T, NT> sh;
    __shared__ int s_it;
    const int tid = threadIdx.x;
    // final counts, set by k_tile: the heaviest first
    const int nf = min(a.hv_ctl[0], a.hv_list_cap);
    const int nb = min(a.hv_ctl[2], a.hv_list_cap - nf);
    for (;;) {
        if (tid == 0) s_it = atomicAdd(&a.hv_ctl[1], 1);
        __syncthreads();
        const int it = s_it;
        __syncthreads();
        if (it >= nf + nb) return;
        const int gb = a.hv_list[it < nf ? it : a.hv_list_cap - 1 - (it - nf)];
        const VpLeaf& v = find_entry(a.vleaf, a.nvleaf, gb);
        const int blk = gb - v.first_block;
        const int l = v.L;
        const long long ti = v.i0 + blk % v.wl, tj = v.j0 + blk / v.wl;
        const int own = v.off + blk;
        const int ci = (int)(ti - v.i0), cj = (int)(tj - v.j0);
        const int k_lo = a.edges[v.col_at + ci];
        const int nx = a.edges[v.col_at + ci + 1] - k_lo;
        const int r_lo = a.edges[v.row_at + cj + 1];
        const int ny = max(a.edges[v.row_at + cj] - r_lo, 0);
        const int* rec = a.hv_flag[gb] == 4 ? a.lists + (size_t)gb * kListInts : nullptr;
        tile_body<T, NT, PX, S, Count>(sh, tv, pv, a, p, Ms, Lc, nset, owner, v, l, ti, tj, own,
                                       k_lo, nx, r_lo, ny, tid, rec);
        __syncthreads();
    }
}

// ------------------------------------------------ persistent downward pass
// One launch runs the downward step of every target box of a batch, over
// all levels and viewports: waves claim boxes from a counter in the plan's
// level-major order, wait until the box's parent has been done, run the
// step (down_body) and mark the box done.  Coarse levels, whose few boxes
// each run a long chain of dependent loads, then overlap with the finer
// levels instead of running one launch after another.  A box's parent has
// a smaller index and was claimed before it by a wave that was already
// running, so every wait ends; each wait is also bounded by the device's
// wall clock (a wave that waits longer sets the stall flag and leaves).
struct DownCtl {
    int next;   // boxes claimed so far (after the roots)
    int error;  // set when a wait ran out
};

// Flags are polled with relaxed loads (coherent across XCDs, no cache
// maintenance) and the acquire is one fence after the flag is seen: an
// acquire load on this hardware invalidates the caches on every poll, and
// thousands of polling waves would keep the working waves' data out of them.
__device__ inline int ld_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_release(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// Polls of one wait at most (with the back-off below, about a second).
constexpr int kMaxPolls = 1 << 20;

template <typename T, bool Count>
__global__ void __launch_bounds__(kWave, 4)
k_down_persist(TreeView tv, PieceView pv, int p, const cpx<double>* __restrict__ M,
               cpx<double>* __restrict__ L, int* __restrict__ nset,
               const cpx<double>* __restrict__ Ttab, int2* __restrict__ owner,
               const VpLevel* __restrict__ lev, int n_ent, int first_box, int total,
               int* __restrict__ done, DownCtl* __restrict__ ctl, long long wait_ticks,
               int* __restrict__ stall, unsigned long long* stats) {
    __shared__ DownShared<T, 1> sh;
    __shared__ int s_b, s_ok;
    const int lane = threadIdx.x;
    for (;;) {
        if (lane == 0) s_b = first_box + atomicAdd(&ctl->next, 1);
        __syncthreads();
        const int b = s_b;
        if (b >= total) return;
        // the level-table entry holding box b (entries are sorted by off)
        int lo = 0, hi = n_ent - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (lev[mid].off <= b) lo = mid; else hi = mid - 1;
        }
        const VpLevel& e = lev[lo];
        const int rel = b - e.off;
        const long long ti = e.i0 + rel % e.wl, tj = e.j0 + rel / e.wl;
        const int par = e.poff + (int)((ti >> 1) - e.pi0) + (int)((tj >> 1) - e.pj0) * e.pwl;
        if (lane == 0) {
            int ok = 1;
            if (ld_relaxed(&done[par]) == 0) {
                // bounded wait: by the wall clock and by the number of polls
                const long long t0 = wall_clock64();
                int nap = 1;
                for (int polls = 1; ld_relaxed(&done[par]) == 0; ++polls) {
                    if (polls >= kMaxPolls ||
                        ((polls & 15) == 0 && wall_clock64() - t0 > wait_ticks)) {
                        atomicOr(&ctl->error, 1);
                        __hip_atomic_store(stall, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        ok = 0;
                        break;
                    }
                    // back-off: 1, 2, 4, 8 and then 8 x 64 clocks between polls
                    if (nap == 1) __builtin_amdgcn_s_sleep(1);
                    else if (nap == 2) __builtin_amdgcn_s_sleep(2);
                    else if (nap == 3) __builtin_amdgcn_s_sleep(4);
                    else __builtin_amdgcn_s_sleep(8);
                    nap = nap < 4 ? nap + 1 : 4;
                }
            }
            // acquire: the parent's outputs are read after the flag
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_ok = ok;
        }
        __syncthreads();
        if (!s_ok) return;
        (void)down_body<T, Count, 1>(sh, tv, pv, e.level, ti, tj, b, par, p, M, L, nset, Ttab,
                                     owner, stats, lane);
        // publish the box's near set, expansion and owner (written by every
        // lane of this one-wave block) with a release store of its flag
        __syncthreads();
        if (lane == 0) st_release(&done[b], 1);
    }
}

// Self-segment correction at the nodes: the FMM summed every piece of the
// node's own segment with the regular closed form; replace that by the
// singular rule (App. C.1, D.3, D.4):
//   y += [ (l - e1 ln e1 - e2 ln e2) sigma_bar + sum_pieces(il qs + th qm) ] / 2pi
__global__ void __launch_bounds__(256)
k_self_correct(int N, const double* __restrict__ nx, const double* __restrict__ ny,
               const int* __restrict__ self_seg, const double* __restrict__ tstar, int s, int g,
               const double* __restrict__ Pi, const double* __restrict__ kappa,
               const double* __restrict__ ell, const double* __restrict__ sigma,
               const double* __restrict__ mu, const int* __restrict__ spb,
               const int* __restrict__ spi, PieceView pv, double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int j = self_seg[i];
    const int panel = j / s, jj = j - panel * s;
    const double* pr = Pi + (size_t)jj * g;
    double sb[3] = {0, 0, 0}, mb[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
        for (int q = 0; q < g; ++q) {
            if (sigma) sb[c] += pr[q] * sigma[(size_t)c * N + (size_t)panel * g + q];
            if (mu) mb[c] += pr[q] * mu[(size_t)c * N + (size_t)panel * g + q];
        }
    }
    const double x = nx[i], yy = ny[i];
    double sil = 0, sth = 0;
    for (int t = spb[j]; t < spb[j + 1]; ++t) {
        const int e = spi[t];
        double il, th;
        chord_log_theta<double>(pv.x0[e] - x, pv.y0[e] - yy, pv.tx[e], pv.ty[e], pv.len[e], il, th);
        sil += il;
        sth += th;
    }
    const double g2 = self_segment_2pi_G(ell[j], tstar[i]);
    const double kap = kappa[j];
    for (int c = 0; c < 3; ++c)
        y[(size_t)c * N + i] += (g2 * sb[c] + sil * kap * sb[c] + sth * kap * mb[c]) / kTwoPi;
}

TreeView tree_view(const FmmState& f) {
    return {f.n_cells, f.X0, f.Y0, f.side, f.lvl.p, f.child.p, f.parent.p, f.pbeg.p,
            f.pend.p, f.npc.p, f.nbeg.p, f.nend.p, f.node_perm.p, f.ix.p, f.iy.p, f.cmask.p};
}
PieceView piece_view(const FmmState& f) {
    return {f.n_pieces, f.px0.p, f.py0.p, f.px1.p, f.py1.p, f.ptx.p, f.pty.p, f.plen.p, f.pseg.p,
            f.w64.p, f.w32.p, f.heavy.p};
}

template <typename T>
cpx<T>* as_cpx(DevBuf<T>& b) {
    return reinterpret_cast<cpx<T>*>(b.p);
}

// Ms_k = Mt_k / k (k >= 1), Ms_0 = Mt_0: the multipoles as the render's
// target-from-outgoing evaluation uses them.
__global__ void __launch_bounds__(256)
k_m2p_scale(int n, int P1, const cpx<double>* __restrict__ M, cpx<double>* __restrict__ Ms) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = (i / 3) % P1;
    const cpx<double> m = M[i];
    Ms[i] = k == 0 ? m : cscale(m, recip<double>(k));
}

__global__ void __launch_bounds__(256)
k_heavy_flags(int n, const double* __restrict__ len, const double* __restrict__ w, double tau,
              int* __restrict__ heavy) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double m = 0;
    for (int c = 0; c < 6; ++c) m = fmax(m, fabs(w[(size_t)c * n + e]));
    heavy[e] = m * len[e] > tau ? 1 : 0;
}

// Pieces whose charge times length exceeds this are evaluated in FP64 by the
// FP32 path (their FP32 rounding alone would approach the error budget).
constexpr double kHeavyTau = 1.0;

// Incoming-from-outgoing operators of the 7 x 7 box offsets (see k_down):
// [o][k][m] complex, o = (dy + 3) * 7 + (dx + 3), (dx, dy) the source box's
// offset in box widths, w = -1 / (2 (dx + i dy)).  Offsets inside the 3 x 3
// neighbourhood are never used and stay zero.
std::vector<double> m2l_table(int p) {
    const int P1 = p + 1;
    std::vector<double> t((size_t)49 * P1 * P1 * 2, 0.0);
    for (int dy = -3; dy <= 3; ++dy)
        for (int dx = -3; dx <= 3; ++dx) {
            if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
            const std::complex<double> z(dx, dy);
            const std::complex<double> w = -1.0 / (2.0 * z);
            std::vector<std::complex<double>> pw(2 * P1);
            pw[0] = 1.0;
            for (int n = 1; n < 2 * P1; ++n) pw[n] = pw[n - 1] * w;
            double* o = t.data() + (size_t)((dy + 3) * 7 + (dx + 3)) * P1 * P1 * 2;
            for (int k = 0; k <= p; ++k) {
                double coef = k == 0 ? 1.0 : 1.0 / k;  // c(k, m) for m = 0 (k > 0) or 1 (k = 0)
                for (int m = 0; m <= p; ++m) {
                    std::complex<double> v;
                    if (k == 0 && m == 0) {
                        v = -std::log(-z);
                    } else {
                        v = ((k & 1) ? -coef : coef) * pw[k + m];
                        coef = coef * (double)(k + m) / (double)(m + 1);
                    }
                    o[((size_t)k * P1 + m) * 2] = v.real();
                    o[((size_t)k * P1 + m) * 2 + 1] = v.imag();
                }
            }
        }
    return t;
}

const cpx<double>* m2l_table_dev(FmmState& f, int p) {
    auto it = f.m2l_tab.find(p);
    if (it == f.m2l_tab.end()) {
        auto buf = std::make_unique<DevBuf<double>>();
        buf->upload(m2l_table(p));
        it = f.m2l_tab.emplace(p, std::move(buf)).first;
    }
    return reinterpret_cast<const cpx<double>*>(it->second->p);
}

// Piece weights and the upward pass for the given densities.  Expansions are
// FP64 in both precision modes: on this hardware an FP64 FMA issues at the
// rate of an unpacked FP32 one, and a leaf's coefficients are sums of charges
// that can cancel by orders of magnitude near cusps.  The FP32 mode keeps
// FP32 for the near-field closed forms, whose logarithms and arctangent are
// where FP64 costs many more instructions.
// Bytes of the cached P2M factors that upward builds for repeated
// operator applications (at most).
constexpr size_t kP2MTableBytes = 8ull << 30;

// The cached P2M factors of order p (built on first use under table mode
// 2; false when they are off or do not fit).  Not built by default: on the
// 200-curve solve (p = 20) reading them took P2M from 70 to 62 us per
// application, for 188 MB; the kernel waits on its leaves' loads either way.
bool p2m_table(FmmState& f, int p, hipStream_t st) {
    if (f.tab_mode != 2 || f.n_pieces == 0) return false;
    if (f.p2m_tab_p == p) return true;
    const size_t n = (size_t)f.n_pieces * (p + 1) * 2;
    if (n * sizeof(cpx<double>) > kP2MTableBytes) return false;
    f.p2m_tab.alloc(2 * n);
    hipLaunchKernelGGL((k_p2m<double, kP2MFill>), dim3(f.n_cells), dim3(kWave), 0, st,
                       tree_view(f), piece_view(f), p, (cpx<double>*)nullptr,
                       as_cpx(f.p2m_tab));
    DC_HIP(hipGetLastError());
    f.p2m_tab_p = p;
    return true;
}

void upward(dc_scene_s& s, FmmState& f, const double* sigma, const double* mu, int p,
            bool want32, hipStream_t st, bool repeated) {
    const Geometry& G = s.geo;
    f.w64.alloc((size_t)6 * f.n_pieces);
    if (want32) {
        f.w32.alloc((size_t)6 * f.n_pieces);
        f.heavy.alloc(f.n_pieces);
    }
    launch_chord_weights(f.n_pieces, f.pseg.p, G.s, G.g, G.N, s.Pi.p, s.seg_kappa.p, sigma, mu,
                         f.w64.p, want32 ? f.w32.p : nullptr, st);
    const size_t nm = (size_t)f.n_cells * (p + 1) * 3 * 2;
    f.M64.alloc(nm);
    const TreeView tv = tree_view(f);
    const PieceView pv = piece_view(f);
    if (repeated && p2m_table(f, p, st))
        hipLaunchKernelGGL((k_p2m<double, kP2MRead>), dim3(f.n_cells), dim3(kWave), 0, st, tv, pv,
                           p, as_cpx(f.M64), as_cpx(f.p2m_tab));
    else
        hipLaunchKernelGGL((k_p2m<double, kP2MEval>), dim3(f.n_cells), dim3(kWave), 0, st, tv, pv,
                           p, as_cpx(f.M64), (cpx<double>*)nullptr);
    DC_HIP(hipGetLastError());
    for (int l = f.depth - 1; l >= 0; --l) {
        const int first = f.level_start[l], cnt = f.level_start[l + 1] - first;
        if (cnt <= 0) continue;
        hipLaunchKernelGGL(k_m2m<double>, dim3(cnt), dim3(kWave), 0, st, tv, first, cnt, p,
                           as_cpx(f.M64));
        DC_HIP(hipGetLastError());
    }
    f.Ms64.alloc(nm);
    hipLaunchKernelGGL(k_m2p_scale, dim3((unsigned)((nm / 2 + 255) / 256)), dim3(256), 0, st,
                       (int)(nm / 2), p + 1, as_cpx(f.M64), as_cpx(f.Ms64));
    DC_HIP(hipGetLastError());
    if (want32) {
        hipLaunchKernelGGL(k_heavy_flags, dim3((f.n_pieces + 255) / 256), dim3(256), 0, st,
                           f.n_pieces, f.plen.p, f.w64.p, kHeavyTau, f.heavy.p);
        DC_HIP(hipGetLastError());
    }
}

// SolveTables: the near field of the solve depends on the geometry alone,
// so the FP64 operator stores, once per scene, each target leaf's near
// pieces and separated boxes and the chord integrals (ln, theta) of each
// (node, near piece) pair (Sec. 6.4: the precomputed operators of every
// GMRES matvec); k_leaf_tab then reads them instead of walking the tree and
// evaluating the closed forms.  Built when the tables fit kSolveTableBytes
// and, unless forced, when the near field averages at least
// kTablePairsPerNode pairs per node: a sparse near field evaluates about as
// fast as the tables read (measured on the 200-curve workload: 58 pairs per
// node at leaf 4, solve 0.53 s without and 0.58 s with the build; 890 at
// leaf 64, 1.56 s without and 1.37 s with).
constexpr size_t kSolveTableBytes = 16ull << 30;
constexpr long long kTablePairsPerNode = 256;

void build_solve_tables(dc_scene_s& s, FmmState& f, LeafArgs a, int p,
                        const cpx<double>* M, const cpx<double>* L, hipStream_t st) {
    f.tab_tried = true;
    const int nl = f.n_target_leaves;
    if (nl <= 0) return;
    const TreeView tv = tree_view(f);
    const PieceView pv = piece_view(f);
    DevBuf<int> count;
    count.upload(std::vector<int>(2 * (size_t)nl, 0));
    a.tab_count = count.p;
    hipLaunchKernelGGL((k_leaf<double, kWave, kLeafCount>), dim3(nl), dim3(kWave), 0, st, tv, pv,
                       a, p, M, L, f.nsetS.p);
    DC_HIP(hipGetLastError());
    std::vector<int> cnt(2 * (size_t)nl), nb(nl);
    DC_HIP(hipMemcpyAsync(cnt.data(), count.p, cnt.size() * sizeof(int), hipMemcpyDeviceToHost,
                          st));
    std::vector<int> tl(nl);
    DC_HIP(hipMemcpyAsync(tl.data(), f.target_leaves.p, nl * sizeof(int), hipMemcpyDeviceToHost,
                          st));
    std::vector<int> nbeg(f.n_cells), nend(f.n_cells);
    DC_HIP(hipMemcpyAsync(nbeg.data(), f.nbeg.p, nbeg.size() * sizeof(int), hipMemcpyDeviceToHost,
                          st));
    DC_HIP(hipMemcpyAsync(nend.data(), f.nend.p, nend.size() * sizeof(int), hipMemcpyDeviceToHost,
                          st));
    DC_HIP(hipStreamSynchronize(st));
    std::vector<long long> pair_off(nl);
    std::vector<int> piece_off(nl + 1), w_off(nl + 1);
    long long pairs = 0, pieces = 0, ws = 0;
    for (int b = 0; b < nl; ++b) {
        pair_off[b] = pairs;
        piece_off[b] = (int)pieces;
        w_off[b] = (int)ws;
        pairs += (long long)cnt[2 * b] * (nend[tl[b]] - nbeg[tl[b]]);
        pieces += cnt[2 * b];
        ws += cnt[2 * b + 1];
        if (pieces >= (1LL << 31) || ws >= (1LL << 31)) return;  // indices would overflow
    }
    piece_off[nl] = (int)pieces;
    w_off[nl] = (int)ws;
    const size_t bytes = (size_t)pairs * 16 + (size_t)(pieces + ws) * 4 + (size_t)nl * 16;
    if (bytes > kSolveTableBytes) return;
    if (f.tab_mode == 1 && pairs < kTablePairsPerNode * (long long)s.geo.N) return;
    f.tab_pair_off.upload(pair_off);
    f.tab_piece_off.upload(piece_off);
    f.tab_w_off.upload(w_off);
    f.tab_piece.alloc(std::max<long long>(1, pieces));
    f.tab_w.alloc(std::max<long long>(1, ws));
    f.tab_val.alloc(2 * (size_t)std::max<long long>(1, pairs));
    a.tab_count = nullptr;
    a.tab_pair_off = f.tab_pair_off.p;
    a.tab_piece_off = f.tab_piece_off.p;
    a.tab_w_off = f.tab_w_off.p;
    a.tab_piece = f.tab_piece.p;
    a.tab_w = f.tab_w.p;
    a.tab_val = f.tab_val.p;
    hipLaunchKernelGGL((k_leaf<double, kWave, kLeafFill>), dim3(nl), dim3(kWave), 0, st, tv, pv,
                       a, p, M, L, f.nsetS.p);
    DC_HIP(hipGetLastError());
    DC_HIP(hipStreamSynchronize(st));
    f.tab_ok = true;
    f.tab_bytes = bytes;
    f.tab_pairs = pairs;
}

template <typename T>
void apply_nodes_t(dc_scene_s& s, FmmState& f, const double* sigma, const double* mu, double* y,
                   const dc_eval_opts& o, hipStream_t st) {
    const int p = o.p;
    upward(s, f, sigma, mu, p, sizeof(T) == 4, st, true);
    f.up_valid = false;  // the cache now holds these densities, not the scene's
    DevBuf<double>& L = f.L64;
    L.alloc((size_t)f.n_cells * (p + 1) * 3 * 2);
    f.nsetS.alloc((size_t)f.n_cells * 9);
    const TreeView tv = tree_view(f);
    const PieceView pv = piece_view(f);
    DevBuf<double>& M = f.M64;
    const cpx<double>* Ttab = m2l_table_dev(f, p);
    hipLaunchKernelGGL(k_init_root<double>, dim3(1), dim3(kWave), 0, st, p, as_cpx(L), f.nsetS.p);
    DC_HIP(hipGetLastError());
    // split downward pass over the cells of levels >= 1 (see k_near_cells)
    const int c1 = f.depth >= 1 ? f.level_start[1] : f.n_cells;
    const int nc = f.n_cells - c1;
    if (nc > 0) {
        f.C64.alloc((size_t)f.n_cells * (p + 1) * 3 * 2);
        f.quietS.alloc(f.n_cells);
        hipLaunchKernelGGL(k_near_cells, dim3((unsigned)((9LL * nc + 255) / 256)), dim3(256), 0, st,
                           tv, c1, nc, f.nsetS.p);
        DC_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_down_contrib_cells<double>), dim3(nc), dim3(kWave), 0, st, tv, pv, p,
                           as_cpx(M), as_cpx(f.C64), f.nsetS.p, Ttab, c1, f.quietS.p);
        DC_HIP(hipGetLastError());
        for (int l = 1; l <= f.depth; ++l) {
            const int first = f.level_start[l];
            const int cnt = f.level_start[l + 1] - first;
            if (cnt <= 0) continue;
            const int G = kWave / (p + 1);
            hipLaunchKernelGGL(k_l2l_cells, dim3((cnt + G - 1) / G), dim3(kWave), 0, st, tv, first,
                               cnt, p, as_cpx(f.C64), as_cpx(L), f.quietS.p);
            DC_HIP(hipGetLastError());
        }
    }
    LeafArgs a{};
    a.target_leaves = f.target_leaves.p;
    a.node_x = s.node_x.p;
    a.node_y = s.node_y.p;
    a.y = y;
    a.N = s.geo.N;
    a.near2 = o.near_fp64 * o.near_fp64;
    if (sizeof(T) == 8 && f.tab_mode != 0 && !f.tab_tried)
        build_solve_tables(s, f, a, p, as_cpx(M), as_cpx(L), st);
    if (f.n_target_leaves > 0 && sizeof(T) == 8 && f.tab_mode != 0 && f.tab_ok) {
        a.tab_pair_off = f.tab_pair_off.p;
        a.tab_piece_off = f.tab_piece_off.p;
        a.tab_w_off = f.tab_w_off.p;
        a.tab_piece = f.tab_piece.p;
        a.tab_w = f.tab_w.p;
        a.tab_val = f.tab_val.p;
        hipLaunchKernelGGL((k_leaf_tab<kWave>), dim3(f.n_target_leaves), dim3(kWave), 0, st, tv,
                           pv, a, p, as_cpx(M), as_cpx(L));
        DC_HIP(hipGetLastError());
    } else if (f.n_target_leaves > 0) {
        hipLaunchKernelGGL((k_leaf<T, kWave>), dim3(f.n_target_leaves), dim3(kWave), 0, st, tv, pv,
                           a, p, as_cpx(M), as_cpx(L), f.nsetS.p);
        DC_HIP(hipGetLastError());
    }
    const Geometry& G = s.geo;
    hipLaunchKernelGGL(k_self_correct, dim3((G.N + 255) / 256), dim3(256), 0, st, G.N,
                       s.node_x.p, s.node_y.p, s.node_self.p, s.node_tstar.p, G.s, G.g, s.Pi.p,
                       s.seg_kappa.p, s.seg_ell.p, sigma, mu, f.seg_piece_beg.p,
                       f.seg_piece_idx.p, pv, y);
    DC_HIP(hipGetLastError());
}

// Target tile level of a viewport: boxes no wider than tile_px pixel pitches
// hold at most tile_px x tile_px pixel centres (rounding of the centres can
// add a row or column now and then; the leaf kernel loops over extra
// targets).
int tile_level(double side, const dc_viewport& vp, int tile_px) {
    const double pitch = std::min(vp.width / vp.W, vp.height / vp.H);
    int Lt = 2;
    while (std::ldexp(side, -Lt) > tile_px * pitch * (1.0 + 1e-12)) {
        ++Lt;
        DC_REQUIRE(Lt <= 60, "viewport pixels are too small for the quadtree root");
    }
    return Lt;
}

// Start of a render: the roots' near sets, expansions and owners (blocks
// 0..n-1), the done flags of the persistent downward pass (the n roots done,
// every other box not; all blocks, a flag per thread) and the counters.
__global__ void k_init_roots(int n, const VpLevel* __restrict__ roots, int p,
                             cpx<double>* __restrict__ L, int* __restrict__ nset,
                             int2* __restrict__ owner, int* __restrict__ hv_ctl,
                             int* __restrict__ done, int total, DownCtl* __restrict__ dctl) {
    const int v = blockIdx.x;
    // the counters of the heavy-tile queue (if any), cleared for this render
    if (v == 0 && hv_ctl != nullptr && threadIdx.x < 3) hv_ctl[threadIdx.x] = 0;
    if (v == 0 && dctl != nullptr && threadIdx.x == 0) {
        dctl->next = 0;
        dctl->error = 0;
    }
    if (done != nullptr) {
        const int i = v * blockDim.x + threadIdx.x;
        if (i < total) done[i] = i < n ? 1 : 0;
    }
    if (v >= n) return;
    const int own = roots[v].off;
    const int t = threadIdx.x;
    if (t == 0) owner[own] = make_int2(own, 0);
    if (t < 9) nset[(size_t)own * 9 + t] = (t == 4) ? 0 : -1;
    for (int i = t; i < (p + 1) * 3; i += blockDim.x) L[(size_t)own * (p + 1) * 3 + i] = {0, 0};
}

// Ticks of the device's constant-rate wall clock in about one second.
long long wall_ticks_per_second() {
    static long long t = 0;
    if (t == 0) {
        int dev = 0, khz = 0;
        DC_HIP(hipGetDevice(&dev));
        DC_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        t = std::max(1, khz) * 1000LL;
    }
    return t;
}

// Blocks of the persistent downward kernel that fit on the device at once
// (its grid: more would only wait to start until the claims run out).
template <typename T, bool Count>
int down_persist_capacity() {
    static int c = 0;
    if (c == 0) {
        int dev = 0, per_cu = 0;
        DC_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        DC_HIP(hipGetDeviceProperties(&prop, dev));
        DC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(k_down_persist<T, Count>), kWave, 0));
        c = std::max(1, per_cu) * prop.multiProcessorCount;
    }
    return c;
}

// Launch of a planned render (plan_render) with its scratch at `scratch`
// (RenderPlan::scratch_bytes, 256-byte aligned) and its descriptor tables
// already written to the pinned host buffer `stage` (RenderPlan::write_tables).
// One downward launch per level covers every viewport that reaches it, and
// one leaf launch covers every viewport's pixel tiles.
// stage: pinned host memory holding the plan's descriptor tables, copied to
// the head of scratch first; null when the caller has already put them
// there.  allow_aux = false keeps every launch on st (no second stream).
template <typename T>
void launch_render_t(dc_scene_s& s, FmmState& f, const RenderPlan& pl, const dc_eval_opts& o,
                     int out_dtype, char* scratch, const void* stage, bool timed,
                     unsigned long long* stats, hipStream_t st, bool allow_aux = true) {
    const int p = o.p;
    DC_REQUIRE(pl.p == p && pl.tile_px == o.tile_px, "render plan does not match the options");
    if (stage != nullptr)
        DC_HIP(hipMemcpyAsync(scratch, stage, pl.desc_bytes, hipMemcpyHostToDevice, st));
    const VpLevel* d_lev = reinterpret_cast<const VpLevel*>(scratch);
    const VpLeaf* d_leaf = reinterpret_cast<const VpLeaf*>(scratch + pl.leaf_at);
    cpx<double>* TL = reinterpret_cast<cpx<double>*>(scratch + pl.tl_at);
    int* nset = reinterpret_cast<int*>(scratch + pl.nset_at);
    int2* owner = reinterpret_cast<int2*>(scratch + pl.owner_at);
    if (timed) DC_HIP(hipEventRecord(f.ev[0], st));
    if (!f.up_valid || f.up_p != p || f.up_prec != (int)sizeof(T)) {
        upward(s, f, s.d_sigma.p, s.d_mu.p, p, sizeof(T) == 4, st, false);
        ++f.up_epoch;
        f.up_valid = true;
        f.up_p = p;
        f.up_prec = (int)sizeof(T);
    }
    const TreeView tv = tree_view(f);
    const PieceView pv = piece_view(f);
    const cpx<double>* M = as_cpx(f.M64);
    const cpx<double>* Ms = as_cpx(f.Ms64);
    const cpx<double>* Ttab = m2l_table_dev(f, p);
    if (timed) DC_HIP(hipEventRecord(f.ev[1], st));
    {
        const int nroots = pl.lev_begin[1] - pl.lev_begin[0];
        int* hv_ctl = o.tile_px <= 8 && pl.hv_flag_at > 0
                          ? reinterpret_cast<int*>(scratch + pl.hv_ctl_at) : nullptr;
        const int total = (int)pl.total_boxes;
        int* done = reinterpret_cast<int*>(scratch + pl.done_at);
        DownCtl* dctl = reinterpret_cast<DownCtl*>(scratch + pl.dctl_at);
        const int init_blocks = std::max(nroots, (total + kWave - 1) / kWave);
        hipLaunchKernelGGL(k_init_roots, dim3(init_blocks), dim3(kWave), 0, st, nroots, d_lev, p,
                           TL, nset, owner, hv_ctl, kPersistentDown ? done : nullptr, total,
                           kPersistentDown ? dctl : nullptr);
        DC_HIP(hipGetLastError());
        if (kPersistentDown && total > nroots) {
            const int n_ent = pl.lev_begin[pl.maxL + 1];
            const long long wait = 2 * wall_ticks_per_second();
            if (stats) {
                const int grid = std::min(total - nroots, down_persist_capacity<T, true>());
                hipLaunchKernelGGL((k_down_persist<T, true>), dim3(grid), dim3(kWave), 0, st, tv,
                                   pv, p, M, TL, nset, Ttab, owner, d_lev, n_ent, nroots, total,
                                   done, dctl, wait, f.stall_dev, stats);
            } else {
                const int grid = std::min(total - nroots, down_persist_capacity<T, false>());
                hipLaunchKernelGGL((k_down_persist<T, false>), dim3(grid), dim3(kWave), 0, st, tv,
                                   pv, p, M, TL, nset, Ttab, owner, d_lev, n_ent, nroots, total,
                                   done, dctl, wait, f.stall_dev, stats);
            }
            DC_HIP(hipGetLastError());
        }
        if (kSplitDown && !kPersistentDown && total > nroots) {
            const int n_ent = pl.lev_begin[pl.maxL + 1];
            cpx<double>* C = reinterpret_cast<cpx<double>*>(scratch + pl.c_at);
            unsigned char* quiet = reinterpret_cast<unsigned char*>(scratch + pl.quiet_at);
            hipLaunchKernelGGL(k_near_all, dim3((unsigned)((9LL * total + 255) / 256)), dim3(256),
                               0, st, tv, d_lev, n_ent, total, nset);
            DC_HIP(hipGetLastError());
            if (stats)
                hipLaunchKernelGGL((k_down_contrib<T, true>), dim3(total - nroots), dim3(kWave), 0,
                                   st, tv, pv, p, M, C, nset, Ttab, d_lev, n_ent, nroots, quiet,
                                   stats);
            else
                hipLaunchKernelGGL((k_down_contrib<T, false>), dim3(total - nroots), dim3(kWave),
                                   0, st, tv, pv, p, M, C, nset, Ttab, d_lev, n_ent, nroots, quiet,
                                   stats);
            DC_HIP(hipGetLastError());
            for (int l = 1; l <= pl.maxL; ++l) {
                DownLevel dl{};
                dl.l = l;
                dl.vl = d_lev + pl.lev_begin[l];
                dl.nvl = pl.lev_begin[l + 1] - pl.lev_begin[l];
                const int G = kWave / (p + 1);
                hipLaunchKernelGGL((k_down_l2l<T>), dim3((pl.lev_blocks[l] + G - 1) / G),
                                   dim3(kWave), 0, st, dl, pl.lev_blocks[l], p, C, TL, quiet,
                                   owner);
                DC_HIP(hipGetLastError());
            }
        }
        for (int l = 1; !kPersistentDown && !kSplitDown && l <= pl.maxL; ++l) {
            DownLevel dl{};
            dl.stats = stats;
            dl.solve = 0;
            dl.l = l;
            dl.vl = d_lev + pl.lev_begin[l];
            dl.nvl = pl.lev_begin[l + 1] - pl.lev_begin[l];
            // levels with few boxes are bound by one wave's latency: deeper staging
            const bool deep = pl.lev_blocks[l] < kDeepBoxes;
            if (stats && deep)
                hipLaunchKernelGGL((k_down<T, true, 3>), dim3(pl.lev_blocks[l]), dim3(kWave), 0,
                                   st, tv, pv, dl, p, M, TL, nset, Ttab, owner);
            else if (stats)
                hipLaunchKernelGGL((k_down<T, true>), dim3(pl.lev_blocks[l]), dim3(kWave), 0, st,
                                   tv, pv, dl, p, M, TL, nset, Ttab, owner);
            else if (deep)
                hipLaunchKernelGGL((k_down<T, false, 3>), dim3(pl.lev_blocks[l]), dim3(kWave),
                                   0, st, tv, pv, dl, p, M, TL, nset, Ttab, owner);
            else
                hipLaunchKernelGGL((k_down<T, false>), dim3(pl.lev_blocks[l]), dim3(kWave), 0, st,
                                   tv, pv, dl, p, M, TL, nset, Ttab, owner);
            DC_HIP(hipGetLastError());
        }
        LeafArgs a{};
        a.out_f64 = out_dtype == DC_OUT_F64;
        a.near2 = o.near_fp64 * o.near_fp64;
        a.stats = stats;
        a.vleaf = d_leaf;
        a.nvleaf = pl.n;
        a.edges = reinterpret_cast<const int*>(scratch + pl.edges_at);
        if (timed) DC_HIP(hipEventRecord(f.ev[2], st));
        // Tiles of up to 8 x 8 pixels: one wave, a pixel per lane; k_tile_scan
        // queues the heavy tiles, which k_tile skips and k_tile_big
        // evaluates.  Up to 16 x 16: 128 threads, two pixels each (a queue
        // for them measured slower on the batch and serving workloads).
        constexpr int NT = kWave * kSplit, NB = kWave * kBigSplit<T>;
        if (o.tile_px > 8) {
            if (stats)
                hipLaunchKernelGGL((k_tile<T, 128, 2, 1, true>), dim3(pl.leaf_blocks), dim3(128),
                                   tile_coef_bytes(128, p), st, tv, pv, a, p, Ms, TL, nset, owner);
            else
                hipLaunchKernelGGL((k_tile<T, 128, 2, 1, false>), dim3(pl.leaf_blocks), dim3(128),
                                   tile_coef_bytes(128, p), st, tv, pv, a, p, Ms, TL, nset, owner);
            DC_HIP(hipGetLastError());
        } else {
            DC_REQUIRE(pl.hv_flag_at > 0, "render plan without the heavy-tile queue");
            a.hv_ctl = reinterpret_cast<int*>(scratch + pl.hv_ctl_at);
            a.hv_list = reinterpret_cast<int*>(scratch + pl.hv_list_at);
            a.hv_list_cap = pl.leaf_blocks;
            a.hv_flag = reinterpret_cast<unsigned char*>(scratch + pl.hv_flag_at);
            a.lists = reinterpret_cast<int*>(scratch + pl.lists_at);
            // (hv_ctl was cleared by k_init_roots)
            if (stats)
                hipLaunchKernelGGL((k_tile_scan<T, kWave, kHeavyPieces<T>, true>),
                                   dim3(pl.leaf_blocks), dim3(kWave), tile_coef_bytes(kWave, p), st,
                                   tv, a, p, TL, nset, owner);
            else
                hipLaunchKernelGGL((k_tile_scan<T, kWave, kHeavyPieces<T>, false>),
                                   dim3(pl.leaf_blocks), dim3(kWave), tile_coef_bytes(kWave, p), st,
                                   tv, a, p, TL, nset, owner);
            DC_HIP(hipGetLastError());
            // large renders: queued tiles on the second stream, concurrently
            // with k_tile; small ones keep everything on st, so renders on
            // different caller streams do not queue behind one another on it
            const bool overlap = allow_aux && pl.leaf_blocks >= kOverlapTiles;
            std::unique_lock<std::mutex> aux_lock(f.aux_mu, std::defer_lock);
            if (overlap) aux_lock.lock();
            hipStream_t aux = overlap ? f.aux_stream() : st;
            if (overlap) {
                DC_HIP(hipEventRecord(f.ev_scan, st));
                DC_HIP(hipStreamWaitEvent(aux, f.ev_scan, 0));
            }
            const int bgrid = std::min(kBigBlocks, pl.leaf_blocks);
            const size_t lb = tile_coef_bytes(NB, p);
            if (stats)
                hipLaunchKernelGGL((k_tile_big<T, true, 1>), dim3(bgrid), dim3(NB), lb, aux, tv, pv,
                                   a, p, Ms, TL, nset, owner);
            else
                hipLaunchKernelGGL((k_tile_big<T, false, 1>), dim3(bgrid), dim3(NB), lb, aux, tv,
                                   pv, a, p, Ms, TL, nset, owner);
            DC_HIP(hipGetLastError());
            if (stats)
                hipLaunchKernelGGL((k_tile<T, NT, 1, kSplit, true>), dim3(pl.leaf_blocks), dim3(NT),
                                   tile_coef_bytes(NT, p), st, tv, pv, a, p, Ms, TL, nset, owner);
            else
                hipLaunchKernelGGL((k_tile<T, NT, 1, kSplit, false>), dim3(pl.leaf_blocks),
                                   dim3(NT), tile_coef_bytes(NT, p), st, tv, pv, a, p, Ms, TL, nset,
                                   owner);
            DC_HIP(hipGetLastError());
            if (overlap) {
                DC_HIP(hipEventRecord(f.ev_big, aux));
                DC_HIP(hipStreamWaitEvent(st, f.ev_big, 0));
            }
        }
    }
    if (timed) {
        DC_HIP(hipEventRecord(f.ev[3], st));
        DC_HIP(hipEventSynchronize(f.ev[3]));
        fmm_check_stall(f);
        float ms[3];
        for (int i = 0; i < 3; ++i) DC_HIP(hipEventElapsedTime(&ms[i], f.ev[i], f.ev[i + 1]));
        f.tms[0] += ms[0];
        f.tms[1] += ms[1];
        f.tms[2] += ms[2];
        f.tms[3] += (double)ms[0] + ms[1] + ms[2];
        f.tcalls++;
    }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    const int i = threadIdx.x;
    if (i < n) p[i] = 0ULL;
}

}  // namespace

void fmm_check_stall(FmmState& f) {
    if (f.stall_host && __atomic_load_n(f.stall_host, __ATOMIC_ACQUIRE) != 0) {
        __atomic_store_n(f.stall_host, 0, __ATOMIC_RELEASE);
        throw Error(DC_ERR_TIMEOUT,
                    "an earlier render of this scene stalled on the device (a bounded wait "
                    "of the render kernel ran out); its images are incomplete");
    }
}

std::unique_ptr<FmmState> fmm_create(const dc_scene_s& s) {
    auto f = std::make_unique<FmmState>();
    DC_HIP(hipHostMalloc(reinterpret_cast<void**>(&f->stall_host), sizeof(int),
                         hipHostMallocMapped));
    *f->stall_host = 0;
    DC_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&f->stall_dev), f->stall_host, 0));
    const Tree& T = s.tree;
    f->n_cells = T.n_cells;
    f->depth = T.depth;
    f->X0 = T.X0;
    f->Y0 = T.Y0;
    f->side = T.side;
    f->level_start = T.level_start;
    f->lvl.upload(T.lvl);
    f->child.upload(T.child);
    f->parent.upload(T.parent);
    f->pbeg.upload(T.pbeg);
    f->pend.upload(T.pend);
    f->npc.upload(T.npc);
    {
        std::vector<int> cm(T.n_cells, 0);
        for (int c = 0; c < T.n_cells; ++c)
            if (T.child[c] >= 0)
                for (int q = 0; q < 4; ++q) cm[c] |= (T.npc[T.child[c] + q] > 0 ? 1 : 0) << q;
        f->cmask.upload(cm);
    }
    f->nbeg.upload(T.nbeg);
    f->nend.upload(T.nend);
    f->node_perm.upload(T.node_perm);
    f->ix.upload(T.ix);
    f->iy.upload(T.iy);
    const size_t np = T.pseg.size();
    f->n_pieces = (int)np;
    std::vector<double> tx(np), ty(np), len(np);
    for (size_t e = 0; e < np; ++e) {
        const double ax = T.px1[e] - T.px0[e], ay = T.py1[e] - T.py0[e];
        len[e] = std::hypot(ax, ay);
        tx[e] = ax / len[e];
        ty[e] = ay / len[e];
    }
    f->px0.upload(T.px0);
    f->py0.upload(T.py0);
    f->px1.upload(T.px1);
    f->py1.upload(T.py1);
    f->ptx.upload(tx);
    f->pty.upload(ty);
    f->plen.upload(len);
    f->pseg.upload(T.pseg);
    // segment -> pieces
    const int S = s.geo.S;
    std::vector<int> beg(S + 1, 0), idx(np);
    for (size_t e = 0; e < np; ++e) beg[T.pseg[e] + 1]++;
    for (int j = 0; j < S; ++j) beg[j + 1] += beg[j];
    std::vector<int> fill(beg.begin(), beg.end() - 1);
    for (size_t e = 0; e < np; ++e) idx[fill[T.pseg[e]]++] = (int)e;
    f->seg_piece_beg.upload(beg);
    f->seg_piece_idx.upload(idx);
    std::vector<int> tl;
    for (int c = 0; c < T.n_cells; ++c)
        if (T.child[c] < 0 && T.nend[c] > T.nbeg[c]) tl.push_back(c);
    f->n_target_leaves = (int)tl.size();
    f->target_leaves.upload(tl);
    return f;
}

void fmm_invalidate(FmmState& f) {
    f.up_valid = false;
    f.gen++;
}

void fmm_render_counts(dc_scene_s& s, const dc_viewport& vp, const dc_eval_opts& o,
                       dc_work_counts* counts, hipStream_t st) {
    FmmState& f = *s.fmm;
    DevBuf<unsigned long long> stats;
    stats.alloc(kNStat);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, stats.p, (int)kNStat);
    DC_HIP(hipGetLastError());
    DevBuf<float> scratch;
    scratch.alloc((size_t)vp.W * vp.H * 3);
    const bool timing = f.timing;
    f.timing = false;
    f.stats = stats.p;
    try {
        fmm_render(s, vp, o, DC_OUT_F32, scratch.p, st);
    } catch (...) {
        f.stats = nullptr;
        f.timing = timing;
        throw;
    }
    f.stats = nullptr;
    f.timing = timing;
    unsigned long long h[kNStat];
    DC_HIP(hipMemcpyAsync(h, stats.p, sizeof(h), hipMemcpyDeviceToHost, st));
    DC_HIP(hipStreamSynchronize(st));
    fmm_check_stall(f);
    counts->p2p_pairs = h[kStatP2P];
    counts->p2p_fp64_pairs = h[kStatP2P64];
    counts->m2p_pairs = h[kStatM2P];
    counts->l2p_targets = h[kStatL2P];
    counts->m2l_pairs = h[kStatM2L];
    counts->p2l_pairs = h[kStatP2L];
    counts->p2l_fp64_pairs = h[kStatP2L64];
    counts->l2l_boxes = h[kStatL2L];
    counts->leaf_boxes = h[kStatLeaf];
    counts->pieces = (unsigned long long)f.n_pieces;
    counts->source_cells = (unsigned long long)f.n_cells;
    counts->levels = tile_level(f.side, vp, o.tile_px) + 1;
    counts->p = o.p;
}

void fmm_apply_nodes(dc_scene_s& s, const double* sigma, const double* mu, double* y,
                     const dc_eval_opts& o, hipStream_t st) {
    if (o.precision == DC_PREC_F32)
        apply_nodes_t<float>(s, *s.fmm, sigma, mu, y, o, st);
    else
        apply_nodes_t<double>(s, *s.fmm, sigma, mu, y, o, st);
}

void plan_render(const FmmState& f, const dc_viewport* vps, int n, int tile_px, int p,
                 RenderPlan& pl) {
    DC_REQUIRE(n >= 1, "empty batch");
    pl.n = n;
    pl.p = p;
    pl.tile_px = tile_px;
    std::vector<int> Lt(n);
    int maxL = 0;
    for (int v = 0; v < n; ++v) {
        Lt[v] = tile_level(f.side, vps[v], tile_px);
        maxL = std::max(maxL, Lt[v]);
    }
    pl.maxL = maxL;
    // rectangles of boxes per (viewport, level)
    std::vector<std::vector<long long>> ri0(n), ri1(n), rj0(n), rj1(n);
    for (int v = 0; v < n; ++v) {
        const dc_viewport& vp = vps[v];
        const double xa = pixel_x(vp.cx, vp.width, vp.W, 0);
        const double xb = pixel_x(vp.cx, vp.width, vp.W, vp.W - 1);
        const double ya = pixel_y(vp.cy, vp.height, vp.H, vp.H - 1);
        const double yb = pixel_y(vp.cy, vp.height, vp.H, 0);
        for (int l = 0; l <= Lt[v]; ++l) {
            const double sl = std::ldexp(f.side, -l);
            const long long a0 = cell_coord(xa, f.X0, sl), a1 = cell_coord(xb, f.X0, sl);
            const long long b0 = cell_coord(ya, f.Y0, sl), b1 = cell_coord(yb, f.Y0, sl);
            const long long lim = 1LL << l;
            DC_REQUIRE(a0 >= 0 && b0 >= 0 && a1 < lim && b1 < lim,
                       "viewport extends outside the scene's quadtree root (enlarge the "
                       "domain in dc_scene_opts)");
            ri0[v].push_back(a0);
            ri1[v].push_back(a1);
            rj0[v].push_back(b0);
            rj1[v].push_back(b1);
        }
    }
    // global layout: level-major, viewports in batch order inside a level
    std::vector<std::vector<int>> offs(n);
    pl.lev.clear();
    pl.vlev.assign((size_t)n * (maxL + 1), -1);
    pl.lev_begin.assign(maxL + 2, 0);
    pl.lev_blocks.assign(maxL + 1, 0);
    long long total = 0;
    for (int l = 0; l <= maxL; ++l) {
        pl.lev_begin[l] = (int)pl.lev.size();
        long long fb = 0;
        for (int v = 0; v < n; ++v) {
            if (l > Lt[v]) continue;
            VpLevel e{};
            e.i0 = ri0[v][l];
            e.j0 = rj0[v][l];
            e.wl = (int)(ri1[v][l] - ri0[v][l] + 1);
            const long long cnt = (long long)e.wl * (rj1[v][l] - rj0[v][l] + 1);
            DC_REQUIRE(total + cnt < (1LL << 31), "render needs too many target boxes");
            e.off = (int)total;
            offs[v].push_back(e.off);
            if (l > 0) {
                e.pi0 = ri0[v][l - 1];
                e.pj0 = rj0[v][l - 1];
                e.pwl = (int)(ri1[v][l - 1] - ri0[v][l - 1] + 1);
                e.poff = offs[v][l - 1];
            }
            e.first_block = (int)fb;
            e.hl = (int)(rj1[v][l] - rj0[v][l] + 1);
            e.level = l;
            fb += cnt;
            total += cnt;
            pl.vlev[(size_t)v * (maxL + 1) + l] = (int)pl.lev.size();
            pl.lev.push_back(e);
        }
        pl.lev_blocks[l] = (int)fb;
    }
    pl.lev_begin[maxL + 1] = (int)pl.lev.size();
    pl.total_boxes = total;
    pl.leaf.assign(n, VpLeaf{});
    pl.edges.clear();
    long long leaf_blocks = 0;
    for (int v = 0; v < n; ++v) {
        VpLeaf& e = pl.leaf[v];
        const int L = Lt[v];
        // pixel ranges of the tile columns and rows, with the same pixel
        // centres and cell rule as the rectangles above: each boundary is
        // guessed from the geometry and settled by the exact rule (cells
        // are monotone in the pixel index)
        {
            const dc_viewport& vp = vps[v];
            const double sl = std::ldexp(f.side, -L);
            const long long i0 = ri0[v][L], i1 = ri1[v][L], j0 = rj0[v][L], j1 = rj1[v][L];
            auto ccol = [&](int k) { return cell_coord(pixel_x(vp.cx, vp.width, vp.W, k), f.X0, sl); };
            auto crow = [&](int r) { return cell_coord(pixel_y(vp.cy, vp.height, vp.H, r), f.Y0, sl); };
            const double px = vp.width / vp.W, py = vp.height / vp.H;
            e.col_at = (int)pl.edges.size();
            for (long long t = i0; t <= i1 + 1; ++t) {
                // first column whose cell is >= t
                double g = std::ceil((f.X0 + (double)t * sl - (vp.cx - 0.5 * vp.width)) / px - 0.5);
                int k = (int)std::min<double>(std::max<double>(g, 0.0), (double)vp.W);
                while (k > 0 && ccol(k - 1) >= t) --k;
                while (k < vp.W && ccol(k) < t) ++k;
                pl.edges.push_back(k);
            }
            e.row_at = (int)pl.edges.size();
            for (long long t = j0 - 1; t <= j1; ++t) {
                // first row whose cell is <= t (rows are numbered downwards)
                double g = std::ceil(((vp.cy + 0.5 * vp.height) - (f.Y0 + (double)(t + 1) * sl)) / py - 0.5);
                int r = (int)std::min<double>(std::max<double>(g, 0.0), (double)vp.H);
                while (r > 0 && crow(r - 1) <= t) --r;
                while (r < vp.H && crow(r) > t) ++r;
                pl.edges.push_back(r);
            }
        }
        e.L = L;
        e.i0 = ri0[v][L];
        e.j0 = rj0[v][L];
        e.wl = (int)(ri1[v][L] - ri0[v][L] + 1);
        e.off = offs[v][L];
        e.vcx = vps[v].cx;
        e.vcy = vps[v].cy;
        e.vw = vps[v].width;
        e.vh = vps[v].height;
        e.W = vps[v].W;
        e.H = vps[v].H;
        e.out = nullptr;
        e.first_block = (int)leaf_blocks;
        e.hl = (int)(rj1[v][L] - rj0[v][L] + 1);
        leaf_blocks += (long long)e.wl * e.hl;
    }
    pl.leaf_blocks = (int)leaf_blocks;
    // scratch layout: [level table | leaf table | edge table | local
    // coefficients | near sets]
    auto up256 = [](size_t x) { return (x + 255) & ~size_t(255); };
    pl.leaf_at = up256(pl.lev.size() * sizeof(VpLevel));
    pl.edges_at = up256(pl.leaf_at + pl.leaf.size() * sizeof(VpLeaf));
    pl.vlev_at = up256(pl.edges_at + pl.edges.size() * sizeof(int));
    pl.desc_bytes = pl.vlev_at + pl.vlev.size() * sizeof(int);
    pl.tl_at = up256(pl.desc_bytes);
    pl.nset_at = up256(pl.tl_at + (size_t)total * (p + 1) * 3 * sizeof(cpx<double>));
    pl.owner_at = up256(pl.nset_at + (size_t)total * 9 * sizeof(int));
    pl.c_at = up256(pl.owner_at + (size_t)total * sizeof(int2));
    pl.quiet_at = up256(pl.c_at + (kSplitDown ? (size_t)total * (p + 1) * 3 * sizeof(cpx<double>) : 0));
    pl.done_at = up256(pl.quiet_at + (kSplitDown ? (size_t)total : 0));
    pl.dctl_at = up256(pl.done_at + (size_t)total * sizeof(int));
    // queue of heavy tiles (it can hold every tile)
    const size_t nl = tile_px <= 8 ? (size_t)pl.leaf_blocks : 0;
    pl.hv_ctl_at = up256(pl.dctl_at + 64);
    pl.hv_list_at = up256(pl.hv_ctl_at + 3 * sizeof(int));
    pl.hv_flag_at = up256(pl.hv_list_at + nl * sizeof(int));
    pl.lists_at = up256(pl.hv_flag_at + nl);
    pl.scratch_bytes = up256(pl.lists_at + nl * kListInts * sizeof(int));
}

void RenderPlan::write_tables(void* host, void* const* outs) const {
    char* h = static_cast<char*>(host);
    std::memcpy(h, lev.data(), lev.size() * sizeof(VpLevel));
    VpLeaf* lf = reinterpret_cast<VpLeaf*>(h + leaf_at);
    for (int v = 0; v < n; ++v) {
        lf[v] = leaf[v];
        lf[v].out = outs[v];
    }
    std::memcpy(h + edges_at, edges.data(), edges.size() * sizeof(int));
    std::memcpy(h + vlev_at, vlev.data(), vlev.size() * sizeof(int));
}

void fmm_launch_render(dc_scene_s& s, const RenderPlan& pl, const dc_eval_opts& o,
                       int out_dtype, char* scratch, const void* stage, hipStream_t st) {
    if (o.precision == DC_PREC_F32)
        launch_render_t<float>(s, *s.fmm, pl, o, out_dtype, scratch, stage, false, nullptr,
                               st);
    else
        launch_render_t<double>(s, *s.fmm, pl, o, out_dtype, scratch, stage, false, nullptr,
                                st);
}

void fmm_prepare(dc_scene_s& s, const dc_eval_opts& o, hipStream_t st) {
    FmmState& f = *s.fmm;
    (void)m2l_table_dev(f, o.p);
    const int prec = o.precision == DC_PREC_F32 ? 4 : 8;
    if (!f.up_valid || f.up_p != o.p || f.up_prec != prec) {
        upward(s, f, s.d_sigma.p, s.d_mu.p, o.p, prec == 4, st, false);
        ++f.up_epoch;
        f.up_valid = true;
        f.up_p = o.p;
        f.up_prec = prec;
    }
}

void fmm_render(dc_scene_s& s, const dc_viewport& vp, const dc_eval_opts& o, int out_dtype,
                void* out, hipStream_t st) {
    void* outs[1] = {out};
    fmm_render_batch(s, &vp, 1, o, out_dtype, outs, st);
}

std::unique_ptr<RenderGraph> fmm_graph_create(dc_scene_s& s, const dc_viewport* vps, int n,
                                              const dc_eval_opts& o, int out_dtype,
                                              void* const* outs) {
    FmmState& f = *s.fmm;
    fmm_check_stall(f);
    auto g = std::make_unique<RenderGraph>();
    g->s = &s;
    g->o = o;
    g->out_dtype = out_dtype;
    plan_render(f, vps, n, o.tile_px, o.p, g->plan);
    DC_HIP(hipHostMalloc(&g->stage, g->plan.desc_bytes, hipHostMallocDefault));
    g->plan.write_tables(g->stage, outs);
    g->scratch.alloc(g->plan.scratch_bytes);
    // everything the launches need but do not make, made now: the upward
    // pass, the operator table and the second stream
    hipStream_t cap = nullptr;
    DC_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    try {
        fmm_prepare(s, o, cap);
        DC_HIP(hipStreamSynchronize(cap));
        {
            std::lock_guard<std::mutex> lk(f.aux_mu);
            (void)f.aux_stream();
        }
        g->gen = f.gen;
        g->up_epoch = f.up_epoch;
        DC_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        try {
            if (o.precision == DC_PREC_F32)
                launch_render_t<float>(s, f, g->plan, o, out_dtype, g->scratch.p, g->stage, false,
                                       nullptr, cap);
            else
                launch_render_t<double>(s, f, g->plan, o, out_dtype, g->scratch.p, g->stage, false,
                                        nullptr, cap);
        } catch (...) {
            hipGraph_t partial = nullptr;
            (void)hipStreamEndCapture(cap, &partial);
            if (partial) (void)hipGraphDestroy(partial);
            throw;
        }
        DC_HIP(hipStreamEndCapture(cap, &g->graph));
        DC_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    } catch (...) {
        (void)hipStreamDestroy(cap);
        throw;
    }
    DC_HIP(hipStreamDestroy(cap));
    return g;
}

void fmm_graph_launch(RenderGraph& g, hipStream_t st) {
    FmmState& f = *g.s->fmm;
    fmm_check_stall(f);
    const int prec = g.o.precision == DC_PREC_F32 ? 4 : 8;
    DC_REQUIRE(f.gen == g.gen, "the scene's densities changed since the render graph was made");
    DC_REQUIRE(f.up_valid && f.up_p == g.o.p && f.up_prec == prec && f.up_epoch == g.up_epoch,
               "the scene's resident expansions were rebuilt since the render graph was made "
               "(make the graph again)");
    DC_HIP(hipGraphLaunch(g.exec, st));
}

namespace {

// Per-device address of dc_noalloc_scratch, looked up once per device with
// that device current (each GPU holds its own copy of the array).
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kMaxDevices] = {};

char* noalloc_scratch_ptr() {
    int dev = 0;
    DC_HIP(hipGetDevice(&dev));
    DC_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[dev] == nullptr) {
        void* p = nullptr;
        DC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(dc_noalloc_scratch)));
        DC_REQUIRE(p != nullptr, "no device address for the allocation-free scratch");
        g_noalloc_ptr[dev] = static_cast<char*>(p);
    }
    return g_noalloc_ptr[dev];
}

// Descriptor tables reach the device scratch as kernel arguments, in chunks
// (no copy from host memory, so the launches can be captured in a graph).
constexpr int kPutChunk = 2048;
struct PutChunk {
    unsigned int off, n;
    unsigned char b[kPutChunk];
};

__global__ void __launch_bounds__(256) k_put_bytes(PutChunk c, char* __restrict__ dst) {
    for (unsigned int i = threadIdx.x; i < c.n; i += blockDim.x) dst[c.off + i] = (char)c.b[i];
}

}  // namespace

void fmm_render_noalloc(dc_scene_s& s, const dc_viewport& vp, const dc_eval_opts& o,
                        int out_dtype, void* out, hipStream_t st) {
    FmmState& f = *s.fmm;
    fmm_check_stall(f);
    const int prec = o.precision == DC_PREC_F32 ? 4 : 8;
    DC_REQUIRE(f.up_valid && f.up_p == o.p && f.up_prec == prec && f.m2l_tab.count(o.p) == 1,
               "dc_render_noalloc: the scene is not prepared for this order and precision "
               "(render it once with dc_render, or register it with a server, using the "
               "same order and precision first)");
    RenderPlan& pl = f.noalloc_plan;
    plan_render(f, &vp, 1, o.tile_px, o.p, pl);
    if (pl.scratch_bytes > (size_t)DC_NOALLOC_SCRATCH_BYTES)
        throw Error(DC_ERR_INVALID,
                    "dc_render_noalloc: this render needs " + std::to_string(pl.scratch_bytes) +
                        " bytes of scratch, more than DC_NOALLOC_SCRATCH_BYTES (" +
                        std::to_string((size_t)DC_NOALLOC_SCRATCH_BYTES) +
                        "); use dc_render, a smaller viewport or larger tiles");
    char* scr = noalloc_scratch_ptr();
    f.noalloc_tables.resize(pl.desc_bytes);
    void* outs[1] = {out};
    pl.write_tables(f.noalloc_tables.data(), outs);
    for (size_t off = 0; off < pl.desc_bytes; off += kPutChunk) {
        PutChunk c;
        c.off = (unsigned int)off;
        c.n = (unsigned int)std::min<size_t>(kPutChunk, pl.desc_bytes - off);
        std::memcpy(c.b, f.noalloc_tables.data() + off, c.n);
        hipLaunchKernelGGL(k_put_bytes, dim3(1), dim3(256), 0, st, c, scr);
        DC_HIP(hipGetLastError());
    }
    if (o.precision == DC_PREC_F32)
        launch_render_t<float>(s, f, pl, o, out_dtype, scr, nullptr, false, nullptr, st, false);
    else
        launch_render_t<double>(s, f, pl, o, out_dtype, scr, nullptr, false, nullptr, st, false);
}

void fmm_render_batch(dc_scene_s& s, const dc_viewport* vps, int n, const dc_eval_opts& o,
                      int out_dtype, void* const* outs, hipStream_t st) {
    FmmState& f = *s.fmm;
    fmm_check_stall(f);
    RenderPlan& pl = f.plan;
    plan_render(f, vps, n, o.tile_px, o.p, pl);
    PinnedStage& ps = f.stage[f.stage_next];
    f.stage_next = (f.stage_next + 1) % FmmState::kStages;
    void* stage = ps.acquire(pl.desc_bytes);
    pl.write_tables(stage, outs);
    if (f.scratch.n < pl.scratch_bytes) {
        if (f.aux) DC_HIP(hipStreamSynchronize(f.aux));  // its kernels read the old scratch
        f.scratch.alloc(pl.scratch_bytes);
    }
    if (o.precision == DC_PREC_F32)
        launch_render_t<float>(s, f, pl, o, out_dtype, f.scratch.p, stage, f.timing, f.stats,
                               st);
    else
        launch_render_t<double>(s, f, pl, o, out_dtype, f.scratch.p, stage, f.timing, f.stats,
                                st);
    ps.mark_used(st);
}

}  // namespace dc
