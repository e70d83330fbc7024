// Library context: host copies of the geometry, the host tree/lists, and every device buffer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gigaqbx.h"
#include "tables.hpp"
#include "tree.hpp"

namespace gq {

// Device buffers. Sources and centers are stored in tree order (see tree.hpp); every box
// array has one entry per box in breadth-first order.
struct DevBuffers {
  // sources (tree order)
  double2 *sxy = nullptr, *snrm = nullptr;
  double *sw = nullptr;
  int32_t *sperm = nullptr;          // caller index of each tree-order source
  // centers (tree order) and their targets
  double2 *cxy = nullptr;
  double *cr = nullptr;
  int32_t *cperm = nullptr;          // caller index of each tree-order center
  int32_t *cbox = nullptr;           // owning box
  int32_t *c2t_start = nullptr;      // CSR center -> target slots (slot = 2 * target + column)
  int32_t *c2t_slot = nullptr;
  // targets (caller order)
  double2 *txy = nullptr;
  int32_t *tctr = nullptr;           // (n_tgt, 2) association as given
  // boxes
  double2 *bc = nullptr;             // centers
  int32_t *blevel = nullptr, *bparent = nullptr, *bchild = nullptr;
  int32_t *bsrc0 = nullptr, *bsrc1 = nullptr;
  // Stage 7 gather: boxes owning centers, and per box its ancestors with a nonzero own local
  int2 *l2g_item = nullptr;          // per wavefront: (first pair, end of pairs), whole boxes
  int2 *l2g_pr = nullptr;            // per pair: (ancestor or -1, box)
  double4 *l2g_tw = nullptr;         // per pair: t = (c_b - c_a)/s_a and 1/u, u = (c_b - c_a)/s_b
  double *l2g_binom_t = nullptr;     // [P1 (k)][P1 (m)]  C(k, m)
  // Stage 2: moment items (box, first source, end, partial slot or -1) and the split boxes
  // (box, first partial, end)
  int4 *p2m_item = nullptr, *p2m_red = nullptr;
  // Stage 4 flat list: per wavefront (first pair, end), per pair (d, offset, box, 0) and
  // log s_b + log|o|
  int2 *m2l_item = nullptr;
  int4 *m2l_pr = nullptr;
  double *m2l_plog = nullptr;
  // Stage 4 for density batches: target boxes grouped by parent; per group record one source box
  // (or -1), the compact offset of each member that lists it (4 bytes, 0xFF: none), the group;
  // per record log s_b + log|o| of each member; per group its member boxes (-1: none); o^-k of
  // the offsets List 2 uses
  int2 *m2g_item = nullptr;          // per work-group: (first record, end), whole groups
  int4 *m2g_rec = nullptr;
  double4 *m2g_plog = nullptr;
  int4 *m2g_grp = nullptr;
  double2 *m2g_opow = nullptr;
  float2 *m2g_opow_f = nullptr;
  // Stage 6b: boxes with List 4 far sources (box, first, end) and the sources, flattened
  int4 *p2l_item = nullptr;
  int32_t *p2l_src = nullptr;
  double *level_side = nullptr, *level_inv_side = nullptr, *level_log_side = nullptr;
  // lists
  int32_t *wf_idx = nullptr;         // List 3 far entries (indexed by the far work items)
  // direct (near-field) work: expanded source lists, balanced work items, partial-row layout
  int32_t *near_src = nullptr;       // per box owning centers: its direct sources (tree order)
  int4 *near_items = nullptr;        // 2 x int4 per item: direct-source chunks (see api.cpp)
  int4 *near_mitems = nullptr;       // 2 x int4 per item: a chunk and up to 4 of its box's centers
  int4 *near_vitems = nullptr;       // the same with up to 16 centers (values at the targets)
  int4 *cval_items = nullptr;        // 2 x int4: (box, first center, n <= 32, List 3 far start), (n far)
                                     // (the matrix-core direct pass of S and D batches)
  int4 *far_items = nullptr;         // 2 x int4 per item: List 3 far chunks
  // Stage 5b packed across boxes (far_pairs_per_lane 1): per wavefront 2 x int4 (first pair,
  // pairs, first staged box, staged boxes), (first unit, units, 0, 0); per pair the LDS slot of
  // its List 3 far box and a double4 (c - c_d, s_d, r); the staged boxes; per unit (one
  // (center, far chunk) row) an int4 (row, first lane, lanes, 0)
  int4 *m2q_wave = nullptr;
  int32_t *m2q_slot = nullptr;
  double4 *m2q_geo = nullptr;
  int32_t *m2q_stage = nullptr;
  int4 *m2q_unit = nullptr;
  double2 *m2q_uz = nullptr;  // per packed unit: (x - c)/r of its center's target
  int32_t *bctr0 = nullptr, *bctr1 = nullptr;   // owned center range per box
  int32_t *part_base = nullptr;      // first near row of each box
  int32_t *n_chunks = nullptr;       // source chunks (rows per center) of each box
  int32_t *n_near_chunks = nullptr;  // of them direct-source chunks (the first ones)
  int32_t *ctr_list = nullptr;       // tree-order centers grouped by order
  double2 *anear = nullptr;          // near rows: [row][p_qbx + 1] scaled coefficients
  double *nval = nullptr;            // direct values at the targets, one per near row (R38 paths)
  // tables
  double2 *opow = nullptr;
  double *m2l_bt = nullptr;
  // the same tables rounded to FP32 for the mixed-precision box expansions
  float *m2l_bt_f = nullptr;
  float2 *opow_f = nullptr;
  double *l2q_binom = nullptr;       // [P1][PQB + 1]  C(k, m)
  double *m2q_binom = nullptr;       // [P1][PQB + 1]  C(k + m - 1, m)
  // workspace
  double *sq = nullptr;              // per-source charge  w * sigma
  double2 *sdip = nullptr;           // per-source dipole  w * tau * n
  double2 *M = nullptr, *L = nullptr;
  double2 *Lf = nullptr;             // complete locals of the boxes owning centers (Stage 7)
  double2 *Mp = nullptr;             // partial moments of split boxes: [slot][partial][2 P1]
  double *tv = nullptr;              // per target slot values
};

// Per-order ranges of the work lists (items of k_near / k_m2qbxl, centers of k_qbx_center).
struct OrderBucket {
  int pq = 0;
  int64_t near0 = 0, near1 = 0, far0 = 0, far1 = 0, ctr0 = 0, ctr1 = 0;
  int64_t m2q0 = 0, m2q1 = 0;        // packed Stage 5b wavefronts
  int64_t nmf0 = 0, nmf1 = 0;        // matrix-core direct items
  int64_t nvf0 = 0, nvf1 = 0;        // matrix-core direct items summed at the targets
  int64_t cv0 = 0, cv1 = 0;          // center-stage items summed at the targets (k_ctr_val)
};

}  // namespace gq

struct gq_ctx {
  int device = -1;
  hipStream_t stream = nullptr;      // caller's stream (borrowed)
  hipStream_t side = nullptr;        // library stream for work that overlaps the tree passes
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_up = nullptr;
  std::string err;

  // geometry (caller order, host copies)
  int64_t ns = 0, nc = 0, nt = 0;
  // Conventional (point) targets: a target that lists no center gets an internal center at its
  // own position with a tiny radius, appended after the caller's nc_user centers. At the target
  // itself only the constant term of that center's expansion survives, which is the plain point
  // value (direct sum + M2P + L2P).
  int64_t nc_user = 0, n_pt = 0;
  // Independent geometries in one context (gq_set_geometry_batch): caller-order offsets of each
  // geometry's sources, centers and targets (n_geom + 1 each), and the geometry of every
  // internal point-target center. n_geom = 1 for gq_set_geometry.
  int64_t n_geom = 1;
  std::vector<int64_t> geom_src_off, geom_ctr_off, geom_tgt_off;
  std::vector<int32_t> pt_geom;
  std::vector<double> src_xy, src_nrm, src_w, ctr_xy, ctr_r, tgt_xy;
  std::vector<int32_t> tgt_ctr;
  bool have_geom = false, built = false;
  // target normals for GQ_SP (caller order, host copy and its device copy) and the flag that
  // makes the stages of an evaluation of GQ_SP differentiate at the targets
  std::vector<double> tgt_nrm;
  double2 *tnrm_dev = nullptr;
  bool eval_sp = false;
  // every center (caller's and internal) serves at most one target slot: the fused S and D
  // direct pass of one density then sums at the targets (set at upload)
  bool one_target_per_center = false;

  gq_params params{};
  gq::Tree tree;
  gq::Tables tables;
  std::vector<int> pq_values;        // compiled QBX orders <= params.p_qbx, ascending
  std::vector<int32_t> box_pq;       // QBX order of each box (largest order of its centers)
  std::vector<int32_t> ctr_pq;       // compiled QBX order of each tree-order center (empty: the
                                     // uniform build order)
  std::vector<gq::OrderBucket> buckets;  // per order: item and center ranges
  std::vector<void *> nw_allocations;    // direct / List 3 far work, re-uploaded on order changes
  int64_t n_tboxes = 0;              // number of target-or-ancestor boxes
  int64_t n_l2g_sinks = 0;           // boxes owning centers (Stage 7 gather)
  int64_t n_l2g_items = 0;           // Stage 7 wavefronts
  int64_t n_p2l_boxes = 0;           // boxes with List 4 far sources (Stage 6b)
  int64_t n_m2l_items = 0;           // Stage 4 wavefronts
  int64_t n_m2g_items = 0;           // Stage 4 work-groups of grouped records (density batches)
  int32_t m2g_n_off = 0;             // distinct List 2 offsets
  int64_t n_p2m_items = 0, n_p2m_red = 0, n_p2m_parts = 0;  // Stage 2 work
  int64_t n_near_items = 0, n_far_items = 0, n_near_rows = 0;
  int64_t n_m2q_waves = 0;           // packed Stage 5b wavefronts (0: per-box items)
  int64_t n_m2q_pairs = 0, n_m2q_units = 0;
  int far_chunk = 16;                // List 3 far boxes per work item (sizes k_m2qbxl's LDS)
  int m2q_stage_rows = 16;           // staged multipoles per packed Stage 5b wavefront
  // Shallowest depth whose multipoles are read (List 2 / List 3 far) and shallowest depth with a
  // non-zero M2L/P2L local: M2M above the first and L2L out of depths above the second have no
  // effect on any result and are not launched.
  gq::DevBuffers d;
  std::vector<void *> allocations;   // tree, list and table allocations, freed together
  std::vector<void *> ws_allocations;  // per-density workspace, sized for ws_batch densities
  int ws_batch = 0;
  double build_ms = 0;
  int64_t m_c_sum = -1;              // N_C M_C (Sec. 4.6.1), computed on demand after a build

  // bumped whenever device buffers a captured graph refers to are freed or replaced
  uint64_t generation = 0;
  hipStream_t capture = nullptr;     // library stream used only to capture evaluation graphs
  hipEvent_t gev_fork = nullptr, gev_up = nullptr, gev_join = nullptr;  // fork/join in captures
  // GQ_S_AND_D: one library stream per kind (both forked from and joined back to the caller's
  // stream), with hand-over events
  hipStream_t main1 = nullptr, main2 = nullptr;
  hipEvent_t ev_pair_in = nullptr, ev_pair_out1 = nullptr, ev_pair_out2 = nullptr;

  // stage profiling (HIP events on the context stream)
  bool profiling = false;
  int cur_kind = 1;
  struct ProfRecord { int slot; hipEvent_t a, b; };
  std::vector<ProfRecord> prof;
  std::vector<hipEvent_t> event_pool;
};
