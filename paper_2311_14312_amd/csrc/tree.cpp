// Quadtree construction and chord clipping (Sec. 6.1, 6.2; App. E.5).
//
// Boxes split while they hold more than leaf_max GL nodes; every split
// creates all four children, so the tree is a full quadtree whose leaves
// tile the root box.  Every chord segment is then cut at the midlines of the
// boxes it crosses until each part ("piece") lies inside a single leaf; the
// clipped pieces carry the segment's density (Sec. 6.2), which keeps every
// part of a chord on the correct side of the near/far split of the FMM.
#include "tree.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace dc {

namespace {

bool less_msb(unsigned long long a, unsigned long long b) { return a < b && a < (a ^ b); }

// Morton order with the y bit above the x bit on every level, which makes
// quadrant q = qx + 2 qy increase along the order.
bool morton_less(long long ax, long long ay, long long bx, long long by) {
    const unsigned long long dx = (unsigned long long)(ax ^ bx);
    const unsigned long long dy = (unsigned long long)(ay ^ by);
    if (!less_msb(dy, dx)) return ay < by;
    return ax < bx;
}

struct Piece {
    double x0, y0, x1, y1;
    int seg, leaf;
};

void clip(const Tree& T, int cell, double x0, double y0, double x1, double y1, int seg,
          std::vector<Piece>& out) {
    if (T.child[cell] < 0) {
        if (x0 != x1 || y0 != y1) out.push_back({x0, y0, x1, y1, seg, cell});
        return;
    }
    const int l = T.lvl[cell];
    const double half = std::ldexp(T.side, -(l + 1));
    const double mx = T.X0 + (double)(2 * T.ix[cell] + 1) * half;
    const double my = T.Y0 + (double)(2 * T.iy[cell] + 1) * half;
    // Parameters where the chord crosses the two midlines.
    double cuts[4];
    int nc = 0;
    cuts[nc++] = 0.0;
    double tx = -1.0, ty = -1.0;
    if ((x0 < mx && x1 > mx) || (x0 > mx && x1 < mx)) tx = (mx - x0) / (x1 - x0);
    if ((y0 < my && y1 > my) || (y0 > my && y1 < my)) ty = (my - y0) / (y1 - y0);
    if (tx > 0.0 && tx < 1.0) cuts[nc++] = tx;
    if (ty > 0.0 && ty < 1.0 && ty != tx) cuts[nc++] = ty;
    cuts[nc++] = 1.0;
    std::sort(cuts, cuts + nc);
    auto point = [&](double t, double& px, double& py) {
        if (t == 0.0) { px = x0; py = y0; return; }
        if (t == 1.0) { px = x1; py = y1; return; }
        px = x0 + t * (x1 - x0);
        py = y0 + t * (y1 - y0);
        if (t == tx) px = mx;  // a cut point sits exactly on its midline
        if (t == ty) py = my;
    };
    for (int k = 0; k + 1 < nc; ++k) {
        double ax, ay, bx, by;
        point(cuts[k], ax, ay);
        point(cuts[k + 1], bx, by);
        const double cx = 0.5 * (ax + bx), cy = 0.5 * (ay + by);
        const int q = (cx >= mx ? 1 : 0) + (cy >= my ? 2 : 0);
        clip(T, T.child[cell] + q, ax, ay, bx, by, seg, out);
    }
}

}  // namespace

void build_tree(const Geometry& G, int leaf_max, int max_depth, const double* domain, Tree& T) {
    DC_REQUIRE(leaf_max >= 1, "leaf_max must be >= 1");
    DC_REQUIRE(max_depth >= 1 && max_depth <= 40, "max_depth must be in 1..40");
    // Root box.
    double xmin = domain[0], ymin = domain[1], xmax = domain[2], ymax = domain[3];
    DC_REQUIRE(std::isfinite(xmin) && std::isfinite(ymin) && std::isfinite(xmax) &&
                   std::isfinite(ymax) && xmax >= xmin && ymax >= ymin,
               "bad domain rectangle");
    for (int i = 0; i < G.N; ++i) {
        xmin = std::min(xmin, G.node_x[i]); xmax = std::max(xmax, G.node_x[i]);
        ymin = std::min(ymin, G.node_y[i]); ymax = std::max(ymax, G.node_y[i]);
    }
    for (int j = 0; j < G.S; ++j) {
        xmin = std::min({xmin, G.seg_x0[j], G.seg_x1[j]});
        xmax = std::max({xmax, G.seg_x0[j], G.seg_x1[j]});
        ymin = std::min({ymin, G.seg_y0[j], G.seg_y1[j]});
        ymax = std::max({ymax, G.seg_y0[j], G.seg_y1[j]});
    }
    double side = std::max(xmax - xmin, ymax - ymin);
    side = side * (1.0 + 1e-6) + 1e-12;
    T.side = side;
    T.X0 = 0.5 * (xmin + xmax) - 0.5 * side;
    T.Y0 = 0.5 * (ymin + ymax) - 0.5 * side;

    // Node keys at the finest level and Morton sort.
    const int D = max_depth;
    const double sideD = std::ldexp(side, -D);
    const long long kmax = (1LL << D) - 1;
    std::vector<long long> kx(G.N), ky(G.N);
    for (int i = 0; i < G.N; ++i) {
        kx[i] = std::min(std::max(cell_coord(G.node_x[i], T.X0, sideD), 0LL), kmax);
        ky[i] = std::min(std::max(cell_coord(G.node_y[i], T.Y0, sideD), 0LL), kmax);
    }
    T.node_perm.resize(G.N);
    std::iota(T.node_perm.begin(), T.node_perm.end(), 0);
    std::stable_sort(T.node_perm.begin(), T.node_perm.end(), [&](int a, int b) {
        return morton_less(kx[a], ky[a], kx[b], ky[b]);
    });

    // Top-down split, level by level.
    T.lvl.assign(1, 0);
    T.ix.assign(1, 0);
    T.iy.assign(1, 0);
    T.parent.assign(1, -1);
    T.child.assign(1, -1);
    T.nbeg.assign(1, 0);
    T.nend.assign(1, G.N);
    T.level_start.assign(1, 0);
    int lstart = 0, lend = 1, l = 0;
    while (lstart < lend) {
        T.level_start.push_back(lend);
        for (int c = lstart; c < lend; ++c) {
            const int a = T.nbeg[c], b = T.nend[c];
            if (b - a <= leaf_max || l >= D) continue;
            const int shift = D - l - 1;
            auto quad = [&](int pos) {
                const int i = T.node_perm[pos];
                return (int)(((kx[i] >> shift) & 1) + 2 * ((ky[i] >> shift) & 1));
            };
            T.child[c] = (int)T.lvl.size();
            int from = a;
            for (int q = 0; q < 4; ++q) {
                int to = from;
                while (to < b && quad(to) == q) ++to;
                T.lvl.push_back(l + 1);
                T.ix.push_back(2 * T.ix[c] + (q & 1));
                T.iy.push_back(2 * T.iy[c] + (q >> 1));
                T.parent.push_back(c);
                T.child.push_back(-1);
                T.nbeg.push_back(from);
                T.nend.push_back(to);
                from = to;
            }
            DC_REQUIRE(from == b, "internal error: node partition");
        }
        lstart = lend;
        lend = (int)T.lvl.size();
        ++l;
    }
    T.n_cells = (int)T.lvl.size();
    T.depth = T.lvl.back();
    // level_start has one entry per level plus the end
    T.level_start.resize(T.depth + 2);
    T.level_start[T.depth + 1] = T.n_cells;

    // Clip every chord at the leaves.
    std::vector<Piece> pieces;
    pieces.reserve((size_t)G.S * 5 / 4 + 16);
    for (int j = 0; j < G.S; ++j)
        clip(T, 0, G.seg_x0[j], G.seg_y0[j], G.seg_x1[j], G.seg_y1[j], j, pieces);
    // Counting sort by leaf (stable: segment order within a leaf).
    std::vector<int> count(T.n_cells + 1, 0);
    for (const Piece& p : pieces) count[p.leaf + 1]++;
    for (int c = 0; c < T.n_cells; ++c) count[c + 1] += count[c];
    T.pbeg.assign(count.begin(), count.end() - 1);
    T.pend.resize(T.n_cells);
    for (int c = 0; c < T.n_cells; ++c) T.pend[c] = count[c + 1];
    const size_t np = pieces.size();
    T.px0.resize(np); T.py0.resize(np); T.px1.resize(np); T.py1.resize(np);
    T.pseg.resize(np); T.pleaf.resize(np);
    std::vector<int> fill(T.pbeg);
    for (const Piece& p : pieces) {
        const int k = fill[p.leaf]++;
        T.px0[k] = p.x0; T.py0[k] = p.y0; T.px1[k] = p.x1; T.py1[k] = p.y1;
        T.pseg[k] = p.seg; T.pleaf[k] = p.leaf;
    }
    // Pieces per subtree, bottom-up; leaf count; node -> leaf.
    T.npc.assign(T.n_cells, 0);
    T.n_leaves = 0;
    T.leaf_of_node.assign(G.N, -1);
    for (int c = T.n_cells - 1; c >= 0; --c) {
        if (T.child[c] < 0) {
            T.npc[c] = T.pend[c] - T.pbeg[c];
            T.n_leaves++;
            for (int pos = T.nbeg[c]; pos < T.nend[c]; ++pos) T.leaf_of_node[T.node_perm[pos]] = c;
        } else {
            T.pend[c] = T.pbeg[c];  // internal cells own no pieces
            int s = 0;
            for (int q = 0; q < 4; ++q) s += T.npc[T.child[c] + q];
            T.npc[c] = s;
        }
    }
}

}  // namespace dc
