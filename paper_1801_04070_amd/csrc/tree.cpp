// Quadtree with target confinement regions and the GIGAQBX interaction lists (host side).
//
// Tree (Sec. 4.3 opening paragraphs, Stage 1 of the Algorithm in Sec. 4.4):
//   - the root square covers every source, every center and every whole QBX disk;
//   - a box is subdivided while it owns more than n_max particles eligible for its children;
//     sources are always eligible, a center is eligible only if its disk fits the target
//     confinement region TCR(child) = square of radius |child| (1 + t_f) about the child center,
//     otherwise the center stays with the parent ("suspended" in a non-leaf box);
//   - empty children are pruned.
// Lists (Sec. 4.3.2, Definitions 2-9, adequate separation of Definition 1, Remark 1):
//   List 1 (U), List 2 (V), List 3 (W) split into close/far by d < TCR(b), List 4 (X) split into
//   close/far by TCR(b) < d and inherited down the tree.
// Readings of the paper's prose: "adjacent" means the closed squares intersect (a box is adjacent
// to itself and to its descendants); the 2-colleagues of b include b; only leaves own sources.
#include "tree.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>
#include <unordered_map>

namespace gq {
namespace {

struct BuildBox {
  int level;
  int64_t i, j;
  int32_t parent;
  int32_t child[4];
  std::vector<int32_t> src, ctr;  // owned particles (caller indices)
};

inline uint64_t box_key(int l, int64_t i, int64_t j) {
  return ((uint64_t)l << 58) | ((uint64_t)i << 29) | (uint64_t)j;
}

void flatten(const std::vector<std::vector<int32_t>> &rows, Csr &out) {
  out.start.assign(rows.size() + 1, 0);
  for (size_t b = 0; b < rows.size(); ++b) out.start[b + 1] = out.start[b] + (int64_t)rows[b].size();
  out.idx.resize(out.start.back());
  for (size_t b = 0; b < rows.size(); ++b)
    std::copy(rows[b].begin(), rows[b].end(), out.idx.begin() + out.start[b]);
}

}  // namespace

std::string build_tree(Tree &t, int64_t ns, const double *sxy, int64_t nc, const double *cxy,
                       const double *cr, const TreeParams &p) {
  t = Tree();
  if (p.n_max < 1) return "n_max must be >= 1";
  if (!(p.t_f >= 0.0 && p.t_f < 1.0)) return "t_f must satisfy 0 <= t_f < 1";
  if (p.max_levels < 1 || p.max_levels > 28) return "max_levels must be in 1..28";
  if (ns < 0 || nc < 0 || ns + nc == 0) return "empty geometry";

  // ---- root square ----
  double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
  for (int64_t s = 0; s < ns; ++s) {
    double x = sxy[2 * s], y = sxy[2 * s + 1];
    if (!std::isfinite(x) || !std::isfinite(y)) return "non-finite source coordinate";
    xmin = std::min(xmin, x); xmax = std::max(xmax, x);
    ymin = std::min(ymin, y); ymax = std::max(ymax, y);
  }
  for (int64_t c = 0; c < nc; ++c) {
    double x = cxy[2 * c], y = cxy[2 * c + 1], r = cr[c];
    if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(r) || r <= 0)
      return "non-finite center coordinate or non-positive radius";
    xmin = std::min(xmin, x - r); xmax = std::max(xmax, x + r);
    ymin = std::min(ymin, y - r); ymax = std::max(ymax, y + r);
  }
  double extent = std::max(xmax - xmin, ymax - ymin);
  if (!(extent > 0)) extent = 1.0;
  double side = std::exp2(std::ceil(std::log2(extent)));
  const double grid = side * std::exp2(-20.0);
  const double mx = std::round(0.5 * (xmin + xmax) / grid) * grid;
  const double my = std::round(0.5 * (ymin + ymax) / grid) * grid;
  for (;;) {
    double lx = mx - 0.5 * side, ly = my - 0.5 * side;
    if (lx <= xmin && ly <= ymin && xmax < lx + side && ymax < ly + side) {
      t.lo[0] = lx; t.lo[1] = ly;
      break;
    }
    side *= 2.0;
  }
  t.side = side;

  // ---- subdivision (level-synchronous: boxes are appended in breadth-first order) ----
  std::vector<BuildBox> bx;
  bx.reserve((size_t)(2 * (ns + nc) / std::max(1, p.n_max) + 16));
  {
    BuildBox root{0, 0, 0, -1, {-1, -1, -1, -1}, {}, {}};
    root.src.resize(ns);
    for (int64_t s = 0; s < ns; ++s) root.src[s] = (int32_t)s;
    root.ctr.resize(nc);
    for (int64_t c = 0; c < nc; ++c) root.ctr[c] = (int32_t)c;
    bx.push_back(std::move(root));
  }
  // Split box b into its non-empty quadrants (sources by quadrant, centers whose disk fits the
  // child's TCR; the others stay, suspended). force: split whatever the count of eligible
  // particles. Returns whether children were made.
  auto subdivide = [&](size_t b, bool force) {
    if (bx[b].level >= p.max_levels - 1) return false;
    const int lev = bx[b].level;
    const double h = 0.5 * side / (double)(int64_t(1) << lev);  // |b|
    const double ccx = t.lo[0] + (bx[b].i + 0.5) * 2 * h, ccy = t.lo[1] + (bx[b].j + 0.5) * 2 * h;
    const double hc = 0.5 * h;                                   // |child|
    auto quad = [&](double x, double y) { return (x >= ccx ? 1 : 0) + (y >= ccy ? 2 : 0); };
    std::vector<int8_t> cq(bx[b].ctr.size());
    int64_t n_elig_ctr = 0;
    for (size_t k = 0; k < bx[b].ctr.size(); ++k) {
      int32_t c = bx[b].ctr[k];
      double x = cxy[2 * c], y = cxy[2 * c + 1];
      int q = quad(x, y);
      double chx = ccx + ((q & 1) ? hc : -hc), chy = ccy + ((q & 2) ? hc : -hc);
      const double dist = p.tcr_shape == 1 ? std::hypot(x - chx, y - chy)
                                            : std::max(std::fabs(x - chx), std::fabs(y - chy));
      bool fits = dist + cr[c] <= hc * (1.0 + p.t_f);
      cq[k] = fits ? (int8_t)q : (int8_t)-1;
      n_elig_ctr += fits;
    }
    int64_t count = (int64_t)bx[b].src.size() + (p.count_mode == 0 ? n_elig_ctr : 0);
    if (!force && count <= p.n_max) return false;
    std::vector<int32_t> csrc[4], cctr[4], keep;
    for (int32_t s : bx[b].src) csrc[quad(sxy[2 * s], sxy[2 * s + 1])].push_back(s);
    for (size_t k = 0; k < bx[b].ctr.size(); ++k) {
      if (cq[k] < 0) keep.push_back(bx[b].ctr[k]);
      else cctr[cq[k]].push_back(bx[b].ctr[k]);
    }
    bool any = false;
    for (int q = 0; q < 4; ++q) {
      if (csrc[q].empty() && cctr[q].empty()) continue;
      any = true;
      BuildBox ch{lev + 1, 2 * bx[b].i + (q & 1), 2 * bx[b].j + ((q >> 1) & 1), (int32_t)b,
                  {-1, -1, -1, -1}, std::move(csrc[q]), std::move(cctr[q])};
      bx[b].child[q] = (int32_t)bx.size();
      bx.push_back(std::move(ch));
    }
    if (any) {
      bx[b].src.clear();
      bx[b].src.shrink_to_fit();
      bx[b].ctr = std::move(keep);
    }
    return any;
  };
  for (size_t b = 0; b < bx.size(); ++b) subdivide(b, false);

  // ---- level restriction (Remark 2, optional): split source leaves until no leaf has an
  // adjacent source leaf two or more levels coarser (adjacent: the closed squares touch, corners
  // included). Leaves that hold only centers own no sources for any list and are not split (their
  // centers may not fit a child's TCR). A leaf b at level l looks at the cells of its 8
  // same-level neighbours; the deepest box covering such a cell, if a source leaf two or more
  // levels coarser, is split (empty quadrants stay absent), and the new leaves are checked in
  // turn. Boxes are then renumbered level-major again.
  if (p.level_restrict) {
    std::unordered_map<uint64_t, int32_t> at;
    at.reserve(bx.size() * 2);
    for (size_t b = 0; b < bx.size(); ++b) at[box_key(bx[b].level, bx[b].i, bx[b].j)] = (int32_t)b;
    auto leaf = [&](int32_t b) {
      return bx[b].child[0] < 0 && bx[b].child[1] < 0 && bx[b].child[2] < 0 && bx[b].child[3] < 0;
    };
    auto cover = [&](int l, int64_t i, int64_t j) -> int32_t {
      if (i < 0 || j < 0 || i >= (int64_t(1) << l) || j >= (int64_t(1) << l)) return -1;
      for (; l >= 0; --l, i >>= 1, j >>= 1) {
        auto it = at.find(box_key(l, i, j));
        if (it != at.end()) return it->second;
      }
      return -1;
    };
    std::vector<int32_t> work;
    for (size_t b = 0; b < bx.size(); ++b)
      if (leaf((int32_t)b)) work.push_back((int32_t)b);
    while (!work.empty()) {
      const int32_t b = work.back();
      work.pop_back();
      if (!leaf(b)) continue;
      const int l = bx[b].level;
      bool again = false;
      for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj) {
          if (!di && !dj) continue;
          const int32_t e = cover(l, bx[b].i + di, bx[b].j + dj);
          if (e < 0 || !leaf(e) || bx[e].level >= l - 1 || bx[e].src.empty()) continue;
          const size_t first = bx.size();
          if (!subdivide((size_t)e, true)) continue;
          for (size_t k = first; k < bx.size(); ++k) {
            at[box_key(bx[k].level, bx[k].i, bx[k].j)] = (int32_t)k;
            work.push_back((int32_t)k);
          }
          again = true;
        }
      if (again) work.push_back(b);  // the covering boxes may still be too coarse
    }
    std::vector<int32_t> perm(bx.size());
    for (size_t k = 0; k < perm.size(); ++k) perm[k] = (int32_t)k;
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int32_t a, int32_t b2) { return bx[a].level < bx[b2].level; });
    std::vector<int32_t> inv(bx.size());
    for (size_t k = 0; k < perm.size(); ++k) inv[perm[k]] = (int32_t)k;
    std::vector<BuildBox> nbx;
    nbx.reserve(bx.size());
    for (int32_t o : perm) {
      BuildBox bb = std::move(bx[o]);
      if (bb.parent >= 0) bb.parent = inv[bb.parent];
      for (int q = 0; q < 4; ++q)
        if (bb.child[q] >= 0) bb.child[q] = inv[bb.child[q]];
      nbx.push_back(std::move(bb));
    }
    bx.swap(nbx);
  }

  const int64_t nb = (int64_t)bx.size();
  t.level.resize(nb); t.parent.resize(nb); t.child.resize(4 * nb);
  t.bi.resize(nb); t.bj.resize(nb); t.cx.resize(nb); t.cy.resize(nb);
  int max_level = 0;
  for (int64_t b = 0; b < nb; ++b) {
    t.level[b] = bx[b].level;
    t.parent[b] = bx[b].parent;
    for (int q = 0; q < 4; ++q) t.child[4 * b + q] = bx[b].child[q];
    t.bi[b] = bx[b].i; t.bj[b] = bx[b].j;
    double s = side / (double)(int64_t(1) << bx[b].level);
    t.cx[b] = t.lo[0] + (bx[b].i + 0.5) * s;
    t.cy[b] = t.lo[1] + (bx[b].j + 0.5) * s;
    max_level = std::max(max_level, bx[b].level);
  }
  t.n_levels = max_level + 1;
  t.level_start.assign(t.n_levels + 1, 0);
  for (int64_t b = 0; b < nb; ++b) t.level_start[t.level[b] + 1]++;
  for (int l = 0; l < t.n_levels; ++l) t.level_start[l + 1] += t.level_start[l];

  // ---- depth-first particle order ----
  t.src_order.reserve(ns); t.ctr_order.reserve(nc);
  t.src_begin.assign(nb, 0); t.src_end.assign(nb, 0);
  t.ctr_begin.assign(nb, 0); t.ctr_end.assign(nb, 0);
  t.ctr_box.reserve(nc);
  {
    std::vector<std::pair<int32_t, int>> stack;  // (box, next child quadrant to visit)
    stack.push_back({0, -1});
    while (!stack.empty()) {
      auto &top = stack.back();
      int32_t b = top.first;
      if (top.second < 0) {  // pre-order visit
        t.ctr_begin[b] = (int64_t)t.ctr_order.size();
        for (int32_t c : bx[b].ctr) { t.ctr_order.push_back(c); t.ctr_box.push_back(b); }
        t.ctr_end[b] = (int64_t)t.ctr_order.size();
        t.src_begin[b] = (int64_t)t.src_order.size();
        for (int32_t s : bx[b].src) t.src_order.push_back(s);
        top.second = 0;
      }
      int q = top.second;
      while (q < 4 && bx[b].child[q] < 0) ++q;
      if (q < 4) {
        top.second = q + 1;
        stack.push_back({bx[b].child[q], -1});
      } else {
        t.src_end[b] = (int64_t)t.src_order.size();
        stack.pop_back();
      }
    }
  }
  bx.clear();
  bx.shrink_to_fit();

  // has_tgt: the box or a descendant owns centers (reverse breadth-first accumulation)
  t.has_tgt.assign(nb, 0);
  for (int64_t b = nb - 1; b >= 0; --b) {
    if (t.ctr_end[b] > t.ctr_begin[b]) t.has_tgt[b] = 1;
    if (t.has_tgt[b] && t.parent[b] >= 0) t.has_tgt[t.parent[b]] = 1;
  }
  for (int64_t b = 0; b < nb; ++b) {
    t.n_leaves += t.is_leaf(b);
    t.n_target_boxes += t.ctr_end[b] > t.ctr_begin[b];
    t.n_local_boxes += t.has_tgt[b];
    if (!t.is_leaf(b)) t.n_suspended += t.ctr_end[b] - t.ctr_begin[b];
  }

  // ---- interaction lists ----
  std::unordered_map<uint64_t, int32_t> lookup;
  lookup.reserve((size_t)nb * 2);
  for (int64_t b = 0; b < nb; ++b) lookup[box_key(t.level[b], t.bi[b], t.bj[b])] = (int32_t)b;
  auto find = [&](int l, int64_t i, int64_t j) -> int32_t {
    if (l < 0 || i < 0 || j < 0) return -1;
    int64_t n = int64_t(1) << l;
    if (i >= n || j >= n) return -1;
    auto it = lookup.find(box_key(l, i, j));
    return it == lookup.end() ? -1 : it->second;
  };
  const int L = max_level;
  auto adjacent = [&](int32_t a, int32_t b) {  // closed squares intersect
    int sa = L - t.level[a], sb = L - t.level[b];
    int64_t ax0 = t.bi[a] << sa, ax1 = (t.bi[a] + 1) << sa, ay0 = t.bj[a] << sa, ay1 = (t.bj[a] + 1) << sa;
    int64_t bx0 = t.bi[b] << sb, bx1 = (t.bi[b] + 1) << sb, by0 = t.bj[b] << sb, by1 = (t.bj[b] + 1) << sb;
    return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
  };
  auto has_src = [&](int32_t b) { return t.src_end[b] > t.src_begin[b]; };
  auto linf = [&](int32_t a, int32_t b) {
    return std::max(std::fabs(t.cx[a] - t.cx[b]), std::fabs(t.cy[a] - t.cy[b]));
  };
  const double tf1 = 1.0 + p.t_f;
  // Euclidean distance from the center of box a to the closed square of radius s about the
  // center of box e
  auto dist2_sq = [&](int32_t a, int32_t e, double s) {
    const double dx = std::max(std::fabs(t.cx[a] - t.cx[e]) - s, 0.0);
    const double dy = std::max(std::fabs(t.cy[a] - t.cy[e]) - s, 0.0);
    return std::hypot(dx, dy);
  };
  // d < TCR(b): l-inf distance of d and TCR(b) at least 2|d| (Definition 1): for the square TCR,
  // l-inf distance of the centers at least 3|d| + |b|(1 + t_f); for the disk TCR (radius
  // |b|(1 + t_f) about c_b), the disk does not reach into the square of radius 3|d| about c_d
  auto box_sep_tcr = [&](int32_t d, int32_t b) {
    if (p.tcr_shape == 1) return dist2_sq(b, d, 3 * t.half(d)) >= t.half(b) * tf1;
    return linf(d, b) >= 3 * t.half(d) + t.half(b) * tf1;
  };
  // TCR(b) < d: l-inf distance of TCR(b) and d at least 2|b|(1 + t_f): square TCR, centers at
  // least 3|b|(1 + t_f) + |d| apart in l-inf; disk TCR, the disk outside the square of radius
  // |d| + 2|b|(1 + t_f) about c_d
  auto tcr_sep_box = [&](int32_t b, int32_t d) {
    if (p.tcr_shape == 1) return dist2_sq(b, d, t.half(d) + 2 * t.half(b) * tf1) >= t.half(b) * tf1;
    return linf(d, b) >= 3 * t.half(b) * tf1 + t.half(d);
  };

  // Leaves with sources at levels <= level(b) whose squares touch b's square.
  auto coarse_adjacent_leaves = [&](int32_t b, std::vector<int32_t> &out) {
    out.clear();
    std::vector<int32_t> anc;
    for (int32_t a = b; a >= 0; a = t.parent[a]) anc.push_back(a);
    for (int32_t a : anc) {
      int l = t.level[a];
      for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj) {
          int32_t e = find(l, t.bi[a] + di, t.bj[a] + dj);
          if (e >= 0 && t.is_leaf(e) && has_src(e) && adjacent(e, b)) out.push_back(e);
        }
    }
  };

  std::vector<std::vector<int32_t>> U(nb), V(nb), Wc(nb), Wf(nb), Xc(nb), Xf(nb);
  std::vector<std::vector<int32_t>> Voff(nb);
  std::vector<int32_t> tmp, W, X;

  // collect all source leaves in the subtree of e
  std::vector<int32_t> stk;
  auto subtree_leaves = [&](int32_t e, std::vector<int32_t> &out) {
    stk.clear();
    stk.push_back(e);
    while (!stk.empty()) {
      int32_t x = stk.back();
      stk.pop_back();
      if (!has_src(x)) continue;
      if (t.is_leaf(x)) { out.push_back(x); continue; }
      for (int q = 3; q >= 0; --q)
        if (t.child[4 * x + q] >= 0) stk.push_back(t.child[4 * x + q]);
    }
  };

  for (int64_t b32 = 0; b32 < nb; ++b32) {
    const int32_t b = (int32_t)b32;
    if (!t.has_tgt[b]) continue;
    const int lb = t.level[b];
    const int32_t pb = t.parent[b];

    // List 2 (Definition 3): children of the 2-colleagues of parent(b), 2-well-separated from b.
    if (pb >= 0) {
      for (int di = -2; di <= 2; ++di)
        for (int dj = -2; dj <= 2; ++dj) {
          int32_t e = find(lb - 1, t.bi[pb] + di, t.bj[pb] + dj);
          if (e < 0) continue;
          for (int q = 0; q < 4; ++q) {
            int32_t d = t.child[4 * e + q];
            if (d < 0 || !has_src(d)) continue;
            int64_t ox = t.bi[b] - t.bi[d], oy = t.bj[b] - t.bj[d];
            if (std::max(std::llabs(ox), std::llabs(oy)) <= 2) continue;
            V[b].push_back(d);
            Voff[b].push_back((int32_t)((ox + 5) * 11 + (oy + 5)));
          }
        }
    }

    // List 4 (Definition 7).
    X.clear();
    for (int di = -2; di <= 2; ++di)
      for (int dj = -2; dj <= 2; ++dj) {
        if (std::max(std::abs(di), std::abs(dj)) != 2) continue;  // non-adjacent 2-colleagues
        int32_t e = find(lb, t.bi[b] + di, t.bj[b] + dj);
        if (e >= 0 && t.is_leaf(e) && has_src(e)) X.push_back(e);
      }
    if (pb >= 0) {
      // leaves that are 2-colleagues of an ancestor of b, adjacent to parent(b) but not to b
      coarse_adjacent_leaves(pb, tmp);
      for (int32_t d : tmp)
        if (!adjacent(d, b)) X.push_back(d);
    }
    // List 4 close / far (Definitions 8, 9): candidates are X(b) and X_close(parent(b)).
    auto place4 = [&](int32_t d) {
      if (tcr_sep_box(b, d)) Xf[b].push_back(d);
      else Xc[b].push_back(d);
    };
    t.max_list4 = std::max<int64_t>(t.max_list4, (int64_t)X.size());
    for (int32_t d : X) place4(d);
    if (pb >= 0)
      for (int32_t d : Xc[pb]) place4(d);

    if (t.ctr_end[b] == t.ctr_begin[b]) continue;  // Lists 1 and 3 only for boxes owning centers

    // List 1 (Definition 2) and List 3 (Definition 4).
    if (t.is_leaf(b)) {
      if (has_src(b)) U[b].push_back(b);
    } else {
      subtree_leaves(b, U[b]);
    }
    coarse_adjacent_leaves(b, tmp);
    for (int32_t d : tmp)
      if (d != b) U[b].push_back(d);
    W.clear();
    std::vector<int32_t> dstk;
    for (int di = -2; di <= 2; ++di)
      for (int dj = -2; dj <= 2; ++dj) {
        if (di == 0 && dj == 0) continue;
        int32_t e = find(lb, t.bi[b] + di, t.bj[b] + dj);
        if (e < 0 || t.is_leaf(e)) continue;
        // descend from the 2-colleague e: the first non-adjacent boxes are in List 3, adjacent
        // leaves on the way are in List 1
        dstk.clear();
        dstk.push_back(e);
        while (!dstk.empty()) {
          int32_t x = dstk.back();
          dstk.pop_back();
          for (int q = 0; q < 4; ++q) {
            int32_t ch = t.child[4 * x + q];
            if (ch < 0 || !has_src(ch)) continue;
            if (adjacent(ch, b)) {
              if (t.is_leaf(ch)) U[b].push_back(ch);
              else dstk.push_back(ch);
            } else {
              W.push_back(ch);
            }
          }
        }
      }
    // List 3 close / far (Definitions 5, 6) with the Remark 1 demotion of small far boxes.
    for (int32_t w0 : W) {
      dstk.clear();
      dstk.push_back(w0);
      while (!dstk.empty()) {
        int32_t d = dstk.back();
        dstk.pop_back();
        if (box_sep_tcr(d, b)) {
          if (p.w3far_min_sources > 0 && t.n_src_subtree(d) < p.w3far_min_sources)
            subtree_leaves(d, Wc[b]);
          else
            Wf[b].push_back(d);
        } else if (t.is_leaf(d)) {
          Wc[b].push_back(d);
        } else {
          for (int q = 0; q < 4; ++q) {
            int32_t ch = t.child[4 * d + q];
            if (ch >= 0 && has_src(ch)) dstk.push_back(ch);
          }
        }
      }
    }
  }

  flatten(U, t.list1); flatten(V, t.list2); flatten(Wc, t.list3c); flatten(Wf, t.list3f);
  flatten(Xc, t.list4c); flatten(Xf, t.list4f);
  t.list2_offset.resize(t.list2.idx.size());
  for (int64_t b = 0; b < nb; ++b)
    std::copy(Voff[b].begin(), Voff[b].end(), t.list2_offset.begin() + t.list2.start[b]);

  // ---- merged near-field source ranges for boxes owning centers ----
  t.near_row.assign(nb + 1, 0);
  std::vector<std::pair<int64_t, int64_t>> rng;
  for (int64_t b = 0; b < nb; ++b) {
    int64_t nown = t.ctr_end[b] - t.ctr_begin[b];
    rng.clear();
    if (nown > 0) {
      for (const std::vector<int32_t> *lst : {&U[b], &Wc[b], &Xc[b]})
        for (int32_t d : *lst) rng.push_back({t.src_begin[d], t.src_end[d]});
      std::sort(rng.begin(), rng.end());
      int64_t nsrc = 0;
      size_t k0 = t.near_lo.size();
      for (auto &r : rng) {
        nsrc += r.second - r.first;
        if (t.near_lo.size() > k0 && t.near_hi.back() == r.first) t.near_hi.back() = r.second;
        else { t.near_lo.push_back(r.first); t.near_hi.push_back(r.second); }
      }
      t.near_pairs += nown * nsrc;
      t.near_sources += nsrc;
      t.list3f_pairs += nown * (int64_t)Wf[b].size();
    }
    for (int32_t d : Xf[b]) t.list4f_sources += t.n_src_subtree(d);
    t.near_row[b + 1] = (int64_t)t.near_lo.size();
  }
  return "";
}

int64_t sources_near_centers(const Tree &t, const double *sxy, const double *cxy, const double *cr,
                             int64_t n_user, double t_f) {
  const int64_t nb = t.n_boxes(), nc = (int64_t)t.ctr_order.size();
  auto half_of = [&](int64_t b) {
    const double s = t.level_side_table.empty() ? std::ldexp(t.side, -t.level[b])
                                                : t.level_side_table[t.level[b]];
    return 0.5 * s;
  };
  std::atomic<int64_t> next{0}, total{0};
  auto work = [&]() {
    std::vector<int32_t> stk;
    int64_t sum = 0;
    for (int64_t k0; (k0 = next.fetch_add(1024)) < nc;) {
      for (int64_t k = k0; k < std::min<int64_t>(nc, k0 + 1024); ++k) {
        const int64_t c = t.ctr_order[k];
        if (c >= n_user) continue;
        int32_t root = t.ctr_box[k];
        while (t.parent[root] >= 0) root = t.parent[root];
        if (!(t_f > 0.0)) {
          sum += t.n_src_subtree(root);
          continue;
        }
        const double R = 8.0 * cr[c] / t_f, x = cxy[2 * c], y = cxy[2 * c + 1];
        stk.assign(1, root);
        while (!stk.empty()) {
          const int32_t b = stk.back();
          stk.pop_back();
          if (t.src_end[b] <= t.src_begin[b]) continue;
          const double h = half_of(b);
          const double dx = std::fabs(t.cx[b] - x), dy = std::fabs(t.cy[b] - y);
          if (dx - h > R || dy - h > R) continue;             // square and box disjoint
          if (dx + h <= R && dy + h <= R) {                      // box inside the square
            sum += t.n_src_subtree(b);
            continue;
          }
          if (t.is_leaf(b)) {
            for (int64_t i = t.src_begin[b]; i < t.src_end[b]; ++i) {
              const int64_t s = t.src_order[i];
              sum += std::max(std::fabs(sxy[2 * s] - x), std::fabs(sxy[2 * s + 1] - y)) <= R;
            }
            continue;
          }
          for (int q = 0; q < 4; ++q)
            if (t.child[4 * b + q] >= 0) stk.push_back(t.child[4 * b + q]);
        }
      }
    }
    total += sum;
  };
  (void)nb;
  const int nthr = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int i = 1; i < nthr; ++i) pool.emplace_back(work);
  work();
  for (auto &th : pool) th.join();
  return total.load();
}

void merge_forest(const std::vector<Tree> &trees, const std::vector<int64_t> &src_base,
                  const std::vector<std::vector<int64_t>> &ctr_global, Tree &f) {
  f = Tree();
  const size_t K = trees.size();
  int depth = 0;
  for (const Tree &t : trees) depth = std::max(depth, t.n_levels);
  f.n_levels = depth;
  f.lo[0] = trees.empty() ? 0.0 : trees[0].lo[0];
  f.lo[1] = trees.empty() ? 0.0 : trees[0].lo[1];
  f.side = trees.empty() ? 1.0 : trees[0].side;
  // virtual levels: tree k, depth l -> vbase[k] + l
  std::vector<int32_t> vbase(K + 1, 0);
  for (size_t k = 0; k < K; ++k) vbase[k + 1] = vbase[k] + trees[k].n_levels;
  f.level_side_table.resize(vbase[K]);
  for (size_t k = 0; k < K; ++k)
    for (int l = 0; l < trees[k].n_levels; ++l)
      f.level_side_table[vbase[k] + l] = std::ldexp(trees[k].side, -l);
  // new box numbering, depth-major
  std::vector<std::vector<int32_t>> map(K);
  std::vector<std::pair<int, int64_t>> order;  // (tree, old box) in new order
  f.level_start.assign(depth + 1, 0);
  for (int l = 0; l < depth; ++l) {
    f.level_start[l] = (int64_t)order.size();
    for (size_t k = 0; k < K; ++k) {
      const Tree &t = trees[k];
      if (l >= t.n_levels) continue;
      for (int64_t b = t.level_start[l]; b < t.level_start[l + 1]; ++b) order.push_back({(int)k, b});
    }
  }
  f.level_start[depth] = (int64_t)order.size();
  for (size_t k = 0; k < K; ++k) map[k].assign(trees[k].n_boxes(), -1);
  for (size_t i = 0; i < order.size(); ++i) map[order[i].first][order[i].second] = (int32_t)i;
  const int64_t nb = (int64_t)order.size();
  f.root_of_level.resize(vbase[K]);
  for (size_t k = 0; k < K; ++k)
    for (int l = 0; l < trees[k].n_levels; ++l) f.root_of_level[vbase[k] + l] = map[k][0];
  // particle offsets in the merged tree order
  std::vector<int64_t> sbase(K + 1, 0), cbase(K + 1, 0);
  for (size_t k = 0; k < K; ++k) {
    sbase[k + 1] = sbase[k] + (int64_t)trees[k].src_order.size();
    cbase[k + 1] = cbase[k] + (int64_t)trees[k].ctr_order.size();
  }
  for (size_t k = 0; k < K; ++k) {
    for (int64_t s : trees[k].src_order) f.src_order.push_back(src_base[k] + s);
    for (int64_t c : trees[k].ctr_order) f.ctr_order.push_back(ctr_global[k][c]);
    for (int32_t b : trees[k].ctr_box) f.ctr_box.push_back(map[k][b]);
  }
  f.level.resize(nb); f.parent.resize(nb); f.child.resize(4 * nb); f.bi.resize(nb); f.bj.resize(nb);
  f.cx.resize(nb); f.cy.resize(nb); f.src_begin.resize(nb); f.src_end.resize(nb);
  f.ctr_begin.resize(nb); f.ctr_end.resize(nb); f.has_tgt.resize(nb);
  auto remap_csr = [&](Csr Tree::*field, Csr &out) {
    out.start.assign(nb + 1, 0);
    out.idx.clear();
    for (int64_t i = 0; i < nb; ++i) {
      const Tree &t = trees[order[i].first];
      const Csr &c = t.*field;
      const int64_t b = order[i].second;
      out.start[i] = (int64_t)out.idx.size();
      if (!c.start.empty())
        for (int64_t e = c.start[b]; e < c.start[b + 1]; ++e)
          out.idx.push_back(map[order[i].first][c.idx[e]]);
    }
    out.start[nb] = (int64_t)out.idx.size();
  };
  f.near_row.assign(nb + 1, 0);
  for (int64_t i = 0; i < nb; ++i) {
    const int k = order[i].first;
    const Tree &t = trees[k];
    const int64_t b = order[i].second;
    f.level[i] = vbase[k] + t.level[b];
    f.parent[i] = t.parent[b] < 0 ? -1 : map[k][t.parent[b]];
    for (int q = 0; q < 4; ++q) {
      const int32_t c = t.child[4 * b + q];
      f.child[4 * i + q] = c < 0 ? -1 : map[k][c];
    }
    f.bi[i] = t.bi[b]; f.bj[i] = t.bj[b]; f.cx[i] = t.cx[b]; f.cy[i] = t.cy[b];
    f.src_begin[i] = sbase[k] + t.src_begin[b]; f.src_end[i] = sbase[k] + t.src_end[b];
    f.ctr_begin[i] = cbase[k] + t.ctr_begin[b]; f.ctr_end[i] = cbase[k] + t.ctr_end[b];
    f.has_tgt[i] = t.has_tgt[b];
    f.near_row[i] = (int64_t)f.near_lo.size();
    for (int64_t g = t.near_row[b]; g < t.near_row[b + 1]; ++g) {
      f.near_lo.push_back(sbase[k] + t.near_lo[g]);
      f.near_hi.push_back(sbase[k] + t.near_hi[g]);
    }
  }
  f.near_row[nb] = (int64_t)f.near_lo.size();
  remap_csr(&Tree::list1, f.list1);
  remap_csr(&Tree::list2, f.list2);
  remap_csr(&Tree::list3c, f.list3c);
  remap_csr(&Tree::list3f, f.list3f);
  remap_csr(&Tree::list4c, f.list4c);
  remap_csr(&Tree::list4f, f.list4f);
  // List 2 offsets follow the V entries of each box in the new row order
  for (int64_t i = 0; i < nb; ++i) {
    const Tree &t = trees[order[i].first];
    const int64_t b = order[i].second;
    for (int64_t e = t.list2.start[b]; e < t.list2.start[b + 1]; ++e)
      f.list2_offset.push_back(t.list2_offset[e]);
  }
  for (const Tree &t : trees) {
    f.n_leaves += t.n_leaves; f.n_target_boxes += t.n_target_boxes; f.n_suspended += t.n_suspended;
    f.near_pairs += t.near_pairs; f.list3f_pairs += t.list3f_pairs;
    f.list4f_sources += t.list4f_sources; f.near_sources += t.near_sources;
    f.max_list4 = std::max(f.max_list4, t.max_list4);
    f.n_local_boxes += t.n_local_boxes;
  }
}

}  // namespace gq
