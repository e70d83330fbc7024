// Quadtree with target confinement regions and the GIGAQBX interaction lists (host side).
//
// Stage 1 of the Algorithm (Sec. 4.4) and the lists of Sec. 4.3 (Definitions 1-9, Remark 1).
// Pure C++, no HIP: it runs on any host and is exercised by the CPU test-suite through a
// host-only library context.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace gq {

struct TreeParams {
  int n_max = 64;
  int count_mode = 0;          // 0: sources + eligible centers, 1: sources only
  double t_f = 0.9;
  int w3far_min_sources = 15;  // Remark 1 threshold, 0 disables
  int max_levels = 24;
  int tcr_shape = 0;           // 0: l-inf square (Definition 1); 1: l2 disk of the same radius
  int level_restrict = 0;      // 1: refine until adjacent leaves differ by at most one level
};

// Compressed sparse rows: entries of row b are idx[start[b] .. start[b+1]).
struct Csr {
  std::vector<int64_t> start;
  std::vector<int32_t> idx;
  int64_t row_size(int64_t b) const { return start[b + 1] - start[b]; }
};

struct Tree {
  // Root square: lower-left corner and side (a power of two); box (level l, i, j) has side
  // side/2^l and center lo + (i + 1/2, j + 1/2) * side/2^l, all exact dyadic values.
  double lo[2] = {0, 0};
  double side = 1;
  int n_levels = 0;

  // Boxes in level-major (breadth-first) order; children in quadrant order x + 2 y.
  std::vector<int32_t> level, parent;
  std::vector<int32_t> child;        // 4 per box, -1 if absent
  std::vector<int64_t> bi, bj;       // integer coordinates at the box's level
  std::vector<int64_t> level_start;  // boxes of level l are [level_start[l], level_start[l+1])
  std::vector<double> cx, cy;        // box centers

  // Particles in tree order. Sources are ordered depth-first by leaf, so every box's subtree
  // sources are contiguous; centers are ordered depth-first by owning box (pre-order).
  std::vector<int64_t> src_order, ctr_order;            // tree position -> caller index
  std::vector<int64_t> src_begin, src_end;              // subtree source range per box
  std::vector<int64_t> ctr_begin, ctr_end;              // owned center range per box
  std::vector<int32_t> ctr_box;                         // owning box per tree-order center
  std::vector<uint8_t> has_tgt;                         // box or a descendant owns centers

  // Interaction lists (rows only for boxes where the list is defined).
  Csr list1;    // U: leaf source boxes, for boxes owning centers       (Def. 2)
  Csr list2;    // V: same-level boxes, for target-or-ancestor boxes    (Def. 3)
  Csr list3c;   // W close: leaf boxes evaluated directly                (Def. 5)
  Csr list3f;   // W far: boxes whose multipoles are taken to QBX locals (Def. 6)
  Csr list4c;   // X close: leaf boxes evaluated directly                (Def. 8)
  Csr list4f;   // X far: leaf boxes whose sources form box locals       (Def. 9)
  std::vector<int32_t> list2_offset;  // per V entry: (ox + 5) * 11 + (oy + 5), o = (c_b - c_d)/side_l

  // Direct (near-field) work per box owning centers: merged source ranges [first, second)
  // covering the sources of List 1 U List 3 close U List 4 close.
  std::vector<int64_t> near_row;                // n_boxes + 1
  std::vector<int64_t> near_lo, near_hi;        // ranges

  // Forests (several independent geometries in one context): box levels are then "virtual"
  // levels, an index into level_side_table (one entry per (tree, depth)); level_start and
  // n_levels stay indexed by depth, so the boxes of one depth of every tree are contiguous.
  // Empty for a single tree, whose level l has side side / 2^l.
  std::vector<double> level_side_table;
  std::vector<int32_t> root_of_level;           // forests: root box of each virtual level's tree

  // Statistics.
  int64_t n_leaves = 0, n_target_boxes = 0, n_suspended = 0;
  int64_t near_pairs = 0, list3f_pairs = 0, list4f_sources = 0, near_sources = 0;
  int64_t n_local_boxes = 0;
  int64_t max_list4 = 0;                        // largest List 4 (Definition 7) of any box

  int64_t n_boxes() const { return (int64_t)level.size(); }
  bool is_leaf(int64_t b) const {
    return child[4 * b] < 0 && child[4 * b + 1] < 0 && child[4 * b + 2] < 0 && child[4 * b + 3] < 0;
  }
  double half(int64_t b) const { return 0.5 * side / (double)(int64_t(1) << level[b]); }
  int64_t n_src_subtree(int64_t b) const { return src_end[b] - src_begin[b]; }
};

// Build the tree and lists. src_xy (ns x 2), ctr_xy (nc x 2), ctr_r (nc). Returns "" on success,
// else an error message.
std::string build_tree(Tree &t, int64_t ns, const double *src_xy, int64_t nc, const double *ctr_xy,
                       const double *ctr_r, const TreeParams &p);

// Sum over the centers c with caller index < n_user of the number of sources y with
// |y - c|_inf <= 8 r_c / t_f (every source of c's own tree when t_f = 0): N_C M_C of Sec. 4.6.1.
// sxy, cxy, cr are in caller order; the square is answered by a walk down c's own tree that adds
// whole subtrees inside it and tests sources only in leaves that straddle its edge.
int64_t sources_near_centers(const Tree &t, const double *sxy, const double *cxy, const double *cr,
                             int64_t n_user, double t_f);

// Merge independent trees into one forest. Tree k's sources are the caller's sources
// src_base[k] + (its local indices); its centers map through ctr_global[k] (local -> caller
// index). Boxes are renumbered depth-major across trees (depth, then tree, then the tree's own
// order); sources and centers keep each tree's order, trees one after another.
void merge_forest(const std::vector<Tree> &trees, const std::vector<int64_t> &src_base,
                  const std::vector<std::vector<int64_t>> &ctr_global, Tree &out);

}  // namespace gq
