// Non-uniform quadtree over the GL nodes with the chords clipped at its
// leaves (Sec. 6.1, 6.2; App. E.5).  Built on the host once per scene.
#pragma once

#include <cstdint>
#include <vector>

#include "geometry.h"

namespace dc {

struct Tree {
    double X0 = 0, Y0 = 0, side = 1;  // root box [X0, X0+side] x [Y0, Y0+side]
    int depth = 0;                    // deepest level present
    int n_cells = 0, n_leaves = 0;
    // Cells are stored level by level; the 4 children of a cell are
    // consecutive, ordered by quadrant q = qx + 2 qy (qx, qy in {0, 1}).
    std::vector<int> level_start;     // [depth + 2]
    std::vector<int> lvl;             // [n_cells]
    std::vector<long long> ix, iy;    // cell coordinates at its level
    std::vector<int> parent, child;   // child = first child or -1 (leaf)
    std::vector<int> nbeg, nend;      // node range in sorted node order
    std::vector<int> pbeg, pend;      // piece range (leaves; empty otherwise)
    std::vector<int> npc;             // pieces in the subtree
    std::vector<int> node_perm;       // sorted position -> node index
    std::vector<int> leaf_of_node;    // node index -> leaf cell
    // Pieces: chord parts, each inside one leaf, sorted by leaf.
    std::vector<double> px0, py0, px1, py1;
    std::vector<int> pseg, pleaf;
};

// Build the tree: root box covers the nodes, the chords and `domain`
// (xmin, ymin, xmax, ymax); a box is split while it holds more than
// leaf_max nodes and its level is below max_depth.
void build_tree(const Geometry& G, int leaf_max, int max_depth, const double* domain, Tree& T);

}  // namespace dc
