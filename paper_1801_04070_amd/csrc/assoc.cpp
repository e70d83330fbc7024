// Target-to-center association (Sec. 2.2.2, placing centers and identifying QBX targets), host
// side. A target that lies in a QBX expansion disk, or outside every disk by at most the slack
// factor (the paper observes that up to 20 % costs little accuracy), is evaluated through the
// center whose disk it lies deepest in (smallest |x - c| / r_c). A target farther than far_factor
// radii from every center is left to the conventional (point) evaluation. Targets in between are
// near the curve but not covered by any disk: they are counted as gaps (the paper refines the
// geometry for them) and left to the conventional evaluation as well.
//
// The query over centers is an area query on a uniform grid: every center is entered into the
// cells its disk of radius far_factor r_c overlaps, so a target needs to look into its own cell
// only.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/gigaqbx.h"

namespace {
thread_local std::string g_assoc_error;
}

extern "C" const char *gq_associate_last_error(void) { return g_assoc_error.c_str(); }

extern "C" gq_status gq_associate_targets(int64_t n_ctr, const double *ctr_xy, const double *ctr_r,
                                          int64_t n_tgt, const double *tgt_xy, double slack,
                                          double far_factor, int32_t *tgt_ctr, int64_t *n_gap) {
  auto fail = [](const char *m) {
    g_assoc_error = m;
    return GQ_EINVAL;
  };
  if (n_ctr < 0 || n_tgt < 0) return fail("negative size");
  if (n_ctr >= (int64_t(1) << 31)) return fail("too many centers");
  if ((n_ctr > 0 && (!ctr_xy || !ctr_r)) || (n_tgt > 0 && (!tgt_xy || !tgt_ctr)))
    return fail("null array");
  if (!(slack >= 0.0) || !(far_factor >= 1.0 + slack) || !std::isfinite(far_factor))
    return fail("need slack >= 0 and a finite far_factor >= 1 + slack");
  for (int64_t c = 0; c < n_ctr; ++c)
    if (!std::isfinite(ctr_xy[2 * c]) || !std::isfinite(ctr_xy[2 * c + 1]) || !(ctr_r[c] > 0) ||
        !std::isfinite(ctr_r[c]))
      return fail("non-finite center or non-positive radius");
  for (int64_t t = 0; t < n_tgt; ++t)
    if (!std::isfinite(tgt_xy[2 * t]) || !std::isfinite(tgt_xy[2 * t + 1]))
      return fail("non-finite target");
  // grid cell: the median reach far_factor r_c (cells per center stay few for every radius of
  // the same order; a much larger disk simply covers more cells)
  double cell = 1.0;
  if (n_ctr > 0) {
    std::vector<double> r(ctr_r, ctr_r + n_ctr);
    std::nth_element(r.begin(), r.begin() + n_ctr / 2, r.end());
    cell = far_factor * r[n_ctr / 2];
  }
  auto key = [](int64_t i, int64_t j) { return (uint64_t)(i + (1ll << 31)) << 32 | (uint64_t)(j + (1ll << 31)); };
  std::unordered_map<uint64_t, std::vector<int32_t>> grid;
  grid.reserve((size_t)n_ctr * 2 + 1);
  for (int64_t c = 0; c < n_ctr; ++c) {
    const double R = far_factor * ctr_r[c];
    const int64_t i0 = (int64_t)std::floor((ctr_xy[2 * c] - R) / cell);
    const int64_t i1 = (int64_t)std::floor((ctr_xy[2 * c] + R) / cell);
    const int64_t j0 = (int64_t)std::floor((ctr_xy[2 * c + 1] - R) / cell);
    const int64_t j1 = (int64_t)std::floor((ctr_xy[2 * c + 1] + R) / cell);
    if ((i1 - i0 + 1) * (j1 - j0 + 1) > (int64_t)1 << 24) return fail("center disk far larger than the grid cell");
    for (int64_t i = i0; i <= i1; ++i)
      for (int64_t j = j0; j <= j1; ++j) grid[key(i, j)].push_back((int32_t)c);
  }
  std::atomic<int64_t> next{0}, gaps{0};
  auto work = [&]() {
    int64_t ng = 0;
    for (int64_t t0; (t0 = next.fetch_add(4096)) < n_tgt;) {
      for (int64_t t = t0; t < std::min<int64_t>(n_tgt, t0 + 4096); ++t) {
        const double x = tgt_xy[2 * t], y = tgt_xy[2 * t + 1];
        int32_t best = -1;
        double best_rho = INFINITY;
        auto it = grid.find(key((int64_t)std::floor(x / cell), (int64_t)std::floor(y / cell)));
        if (it != grid.end())
          for (int32_t c : it->second) {
            const double rho = std::hypot(x - ctr_xy[2 * c], y - ctr_xy[2 * c + 1]) / ctr_r[c];
            if (rho < best_rho || (rho == best_rho && c < best)) {
              best_rho = rho;
              best = c;
            }
          }
        tgt_ctr[2 * t + 1] = -1;
        if (best >= 0 && best_rho <= 1.0 + slack) {
          tgt_ctr[2 * t] = best;
        } else {
          tgt_ctr[2 * t] = -1;
          if (best >= 0 && best_rho < far_factor) ++ng;
        }
      }
    }
    gaps += ng;
  };
  const int nthr = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int k = 1; k < nthr && (int64_t)k * 4096 < n_tgt; ++k) pool.emplace_back(work);
  work();
  for (auto &th : pool) th.join();
  if (n_gap) *n_gap = gaps.load();
  return GQ_OK;
}
