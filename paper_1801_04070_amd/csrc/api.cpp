// C-ABI implementation (host side): argument checking, geometry and tree upload, evaluation
// orchestration. Every step of an evaluation runs in the HIP kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>

#include "context.hpp"
#include "kernels.hpp"

namespace {

thread_local std::string g_create_error;

gq_status fail(gq_ctx *ctx, gq_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  else g_create_error = msg;
  return st;
}

#define GQ_HIP(ctx, call)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(ctx, GQ_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

void free_workspace(gq_ctx *ctx) {
  ctx->generation++;
  if (ctx->device >= 0) {
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    if (ctx->main1) (void)hipStreamSynchronize(ctx->main1);
    if (ctx->main2) (void)hipStreamSynchronize(ctx->main2);
    for (void *p : ctx->ws_allocations) (void)hipFree(p);
  }
  ctx->ws_allocations.clear();
  ctx->ws_batch = 0;
  ctx->d.sq = nullptr; ctx->d.sdip = nullptr; ctx->d.M = nullptr; ctx->d.L = nullptr;
  ctx->d.Lf = nullptr; ctx->d.Mp = nullptr;
  ctx->d.anear = nullptr; ctx->d.nval = nullptr; ctx->d.tv = nullptr;
}

void drop_target_normals(gq_ctx *ctx) {
  if (ctx->tnrm_dev && ctx->device >= 0) {
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->tnrm_dev);
  }
  ctx->tnrm_dev = nullptr;
  ctx->tgt_nrm.clear();
}

void free_device(gq_ctx *ctx) {
  free_workspace(ctx);
  ctx->generation++;
  if (ctx->device >= 0) {
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (void *p : ctx->allocations) (void)hipFree(p);
    for (void *p : ctx->nw_allocations) (void)hipFree(p);
  }
  ctx->allocations.clear();
  ctx->nw_allocations.clear();
  ctx->d = gq::DevBuffers();
  ctx->built = false;
}

template <typename T>
gq_status upload(gq_ctx *ctx, T *&dst, const void *src, size_t count) {
  dst = nullptr;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(ctx, GQ_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  ctx->allocations.push_back(p);
  if (src && count) {
    e = hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(ctx, GQ_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  dst = static_cast<T *>(p);
  return GQ_OK;
}

template <typename T>
gq_status alloc_ws(gq_ctx *ctx, T *&dst, size_t count) {
  dst = nullptr;
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return fail(ctx, GQ_ENOMEM, std::string("hipMalloc (workspace): ") + hipGetErrorString(e));
  ctx->ws_allocations.push_back(p);
  dst = static_cast<T *>(p);
  return GQ_OK;
}

#define GQ_TRY(expr)                 \
  do {                               \
    gq_status s_ = (expr);           \
    if (s_ != GQ_OK) return s_;      \
  } while (0)

// Direct-interaction work (Stages 3, 5a, 6a) and the per-box form of the multipole-to-QBX-local
// work (Stage 5b) are split into items of one wavefront each: a box, one chunk of its direct
// sources (at most kNearChunk) or of its List 3 far boxes (at most kFarChunk), and a block of
// n_cl of its centers. The wave runs n_cl centers x n_sl slices over the chunk (n_cl n_sl <= 64),
// the shape minimising a simple cost model (per-element work + slice reduction + fixed cost per
// wave): any n_sl for the direct items, powers of two for the List 3 far items. Each (center,
// chunk) result goes to its own row; the rows of a box are laid out [chunk][center], direct
// chunks first.
constexpr int kMomentChunk = 512;  // sources per Stage 2 work item
constexpr int kM2LRun = 64;        // List 2 pairs per Stage 4 wavefront (whole boxes, at least)
constexpr int kNearChunk = 1024;   // defaults of gq_params.near_chunk / far_chunk
constexpr int kFarChunk = 16;
constexpr int kM2qStageRows = 16;  // multipoles staged per packed Stage 5b wavefront (at least)

int pick_lg(int64_t nc, int64_t len, double elem_cost) {
  int best_lg = 0;
  double best = 1e300;
  for (int lg = 0; lg <= 6; ++lg) {
    const int64_t ncl = int64_t(1) << lg, nsl = 64 >> lg;
    const double waves = (double)((nc + ncl - 1) / ncl);
    const double cost = waves * ((double)((len + nsl - 1) / nsl) * elem_cost + (6 - lg) * 60.0 + 150.0);
    if (cost <= best) { best = cost; best_lg = lg; }
  }
  return best_lg;
}

// Slices per center (1..64) of a direct item, n_cl = 64 / n_sl centers per wavefront. A lane
// takes at most kNearLaneSteps sources of the chunk (unless n_sl = 64): for a large box every
// shape costs about the same in total, and without the cap the model picks one or two slices,
// whose wavefronts then run far longer than the rest and set the kernel's length.
constexpr int kNearLaneSteps = 64;

int pick_slices(int64_t nc, int64_t len, double elem_cost) {
  int best_nsl = 64;
  double best = 1e300;
  for (int nsl = 64; nsl >= 1; --nsl) {
    if (nsl < 64 && (len + nsl - 1) / nsl > kNearLaneSteps) continue;
    const int64_t ncl = 64 / nsl;
    int steps = 0;
    while ((1 << steps) < nsl) ++steps;  // reduction steps, ceil(log2 n_sl)
    const double waves = (double)((nc + ncl - 1) / ncl);
    const double cost = waves * ((double)((len + nsl - 1) / nsl) * elem_cost + steps * 60.0 + 150.0);
    if (cost <= best) { best = cost; best_nsl = nsl; }
  }
  return best_nsl;
}

// Work of the per-center stages grouped by QBX order: every box runs at its own order (the
// largest order among its centers, default the build's p_qbx), and the items, rows and centers of
// each compiled order form one contiguous range so that each order is one kernel launch. Device
// contexts upload the lists; host-only contexts keep their counts (gq_get_stats).
gq_status build_near_work(gq_ctx *ctx) {
  const gq::Tree &t = ctx->tree;
  auto &d = ctx->d;
  const int64_t nb = t.n_boxes();
  for (void *p : ctx->nw_allocations) (void)hipFree(p);
  ctx->nw_allocations.clear();
  ctx->generation++;
  std::vector<int32_t> src, bctr0(nb), bctr1(nb), base(nb, 0), nch(nb, 0), nnear(nb, 0), items, fitems, clist, vitems,
      citems;
  std::vector<int32_t> mitems;  // matrix-core direct items: (off, len, first center, first row), (n_ctr <= 4)
  std::vector<int32_t> qwave, qpair, qstage, qunit;
  std::vector<double> qgeo, quz;
  // each center's first target (caller order): a packed unit carries (x - c)/r of its center's
  // target, at which k_m2qbxl_packed evaluates when every center serves at most one target
  std::vector<int64_t> first_tgt(ctx->nc, -1);
  for (int64_t tg = ctx->nt - 1; tg >= 0; --tg)
    for (int sd = 1; sd >= 0; --sd)
      if (ctx->tgt_ctr[2 * tg + sd] >= 0) first_tgt[ctx->tgt_ctr[2 * tg + sd]] = tg;

  std::vector<double> lside = t.level_side_table;
  if (lside.empty())
    for (int l = 0; l < t.n_levels; ++l) lside.push_back(std::ldexp(t.side, -l));
  std::vector<int64_t> box_src_off(nb, 0), box_src_len(nb, 0);
  int64_t rows = 0;
  const int64_t near_chunk = ctx->params.near_chunk > 0 ? ctx->params.near_chunk : kNearChunk;
  const int64_t far_chunk = ctx->params.far_chunk > 0 ? ctx->params.far_chunk : kFarChunk;
  ctx->far_chunk = (int)far_chunk;
  const int far_ppl = ctx->params.far_pairs_per_lane;
  const bool packed = far_ppl == 1;
  const int stage_rows = (int)std::max<int64_t>(kM2qStageRows, far_chunk);
  ctx->m2q_stage_rows = stage_rows;
  // Packed Stage 5b: units (center, chunk of its box's List 3 far boxes) in box order, whole
  // units per wavefront, at most 64 pairs and stage_rows staged multipoles each (a chunk's boxes
  // are staged once per wavefront and shared by the units of its centers)
  int32_t q_pair0 = 0, q_stage0 = 0, q_unit0 = 0;
  auto close_wave = [&]() {
    const int32_t np = (int32_t)qpair.size() / 4 - q_pair0;
    if (np == 0) return;
    const int32_t w[8] = {q_pair0, np, q_stage0, (int32_t)qstage.size() - q_stage0,
                          q_unit0, (int32_t)qunit.size() / 4 - q_unit0, 0, 0};
    qwave.insert(qwave.end(), w, w + 8);
    q_pair0 = (int32_t)qpair.size() / 4;
    q_stage0 = (int32_t)qstage.size();
    q_unit0 = (int32_t)qunit.size() / 4;
  };
  // List 3 far items: with far_ppl > 0 the fewest slices that keep each lane at <= far_ppl
  // boxes (short serial chains, many waves); else the cost model
  auto far_lg = [&](int64_t nc, int64_t clen, int pq) {
    if (far_ppl <= 0) return pick_lg(nc, clen, 200.0 * pq);
    for (int lg = 6; lg > 0; --lg)
      if ((clen + (64 >> lg) - 1) / (64 >> lg) <= far_ppl) return lg;
    return 0;
  };
  auto emit = [](std::vector<int32_t> &out, int64_t off, int64_t clen, int64_t ctr0, int64_t row0,
                 int64_t nc, int lg) {
    const int64_t ncl = int64_t(1) << lg;
    for (int64_t cb = 0; cb < nc; cb += ncl) {
      const int32_t item[8] = {(int32_t)off, (int32_t)clen, (int32_t)(ctr0 + cb), (int32_t)(row0 + cb),
                               (int32_t)std::min<int64_t>(ncl, nc - cb), lg, 0, 0};
      out.insert(out.end(), item, item + 8);
    }
  };
  // direct items record their slice count, n_sl (List 3 far items: log2 of n_cl)
  auto emit_near = [](std::vector<int32_t> &out, int64_t off, int64_t clen, int64_t ctr0,
                      int64_t row0, int64_t nc, int nsl) {
    const int64_t ncl = 64 / nsl;
    for (int64_t cb = 0; cb < nc; cb += ncl) {
      const int32_t item[8] = {(int32_t)off, (int32_t)clen, (int32_t)(ctr0 + cb), (int32_t)(row0 + cb),
                               (int32_t)std::min<int64_t>(ncl, nc - cb), nsl, 0, 0};
      out.insert(out.end(), item, item + 8);
    }
  };
  // direct source lists and row layout (independent of the orders)
  for (int64_t b = 0; b < nb; ++b) {
    bctr0[b] = (int32_t)t.ctr_begin[b];
    bctr1[b] = (int32_t)t.ctr_end[b];
    const int64_t nc = t.ctr_end[b] - t.ctr_begin[b];
    if (nc == 0) continue;
    box_src_off[b] = (int64_t)src.size();
    for (int64_t g = t.near_row[b]; g < t.near_row[b + 1]; ++g)
      for (int64_t s = t.near_lo[g]; s < t.near_hi[g]; ++s) src.push_back((int32_t)s);
    box_src_len[b] = (int64_t)src.size() - box_src_off[b];
    const int64_t nchunks = (box_src_len[b] + near_chunk - 1) / near_chunk;
    const int64_t wlen = t.list3f.start[b + 1] - t.list3f.start[b];
    const int64_t fchunks = (wlen + far_chunk - 1) / far_chunk;
    base[b] = (int32_t)rows;
    nch[b] = (int32_t)(nchunks + fchunks);
    nnear[b] = (int32_t)nchunks;
    rows += (nchunks + fchunks) * nc;
  }
  // items and centers, grouped by order
  ctx->buckets.clear();
  for (int pq : ctx->pq_values) {
    gq::OrderBucket bk;
    bk.pq = pq;
    bk.near0 = (int64_t)items.size() / 8;
    bk.nmf0 = (int64_t)mitems.size() / 8;
    bk.nvf0 = (int64_t)vitems.size() / 8;
    bk.cv0 = (int64_t)citems.size() / 8;
    bk.far0 = (int64_t)fitems.size() / 8;
    bk.m2q0 = (int64_t)qwave.size() / 8;
    bk.ctr0 = (int64_t)clist.size();
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t nc = t.ctr_end[b] - t.ctr_begin[b];
      if (nc == 0) continue;
      // the box's centers of this order: one contiguous group (centers are ordered by QBX order
      // within each box); rows stay those of the whole box, [chunk][center of the box]
      int64_t g0 = t.ctr_begin[b], g1 = t.ctr_end[b];
      if (!ctx->ctr_pq.empty()) {
        while (g0 < g1 && ctx->ctr_pq[g0] != pq) ++g0;
        g1 = g0;
        while (g1 < t.ctr_end[b] && ctx->ctr_pq[g1] == pq) ++g1;
      } else if (ctx->params.p_qbx != pq) {
        continue;
      }
      const int64_t ng = g1 - g0, gl = g0 - t.ctr_begin[b];
      if (ng == 0) continue;
      const int64_t len = box_src_len[b];
      const int64_t nchunks = (len + near_chunk - 1) / near_chunk;
      for (int64_t j = 0; j < nchunks; ++j) {
        const int64_t c0 = j * near_chunk, clen = std::min<int64_t>(near_chunk, len - c0);
        emit_near(items, box_src_off[b] + c0, clen, g0, base[b] + j * nc + gl, ng,
                  pick_slices(ng, clen, 10.0 * pq));
        for (int64_t cb = 0; cb < ng; cb += 4) {
          const int32_t it[8] = {(int32_t)(box_src_off[b] + c0), (int32_t)clen, (int32_t)(g0 + cb),
                                 (int32_t)(base[b] + j * nc + gl + cb),
                                 (int32_t)std::min<int64_t>(4, ng - cb), 0, 0, 0};
          mitems.insert(mitems.end(), it, it + 8);
        }
        for (int64_t cb = 0; cb < ng; cb += 16) {
          const int32_t it[8] = {(int32_t)(box_src_off[b] + c0), (int32_t)clen, (int32_t)(g0 + cb),
                                 (int32_t)(base[b] + j * nc + gl + cb),
                                 (int32_t)std::min<int64_t>(16, ng - cb), 0, 0, 0};
          vitems.insert(vitems.end(), it, it + 8);
        }
      }
      const int64_t woff = t.list3f.start[b], wlen = t.list3f.start[b + 1] - woff;
      for (int64_t cb = 0; cb < ng; cb += 32) {  // k_ctr_val: two row tiles of 16 centers
        const int32_t it[8] = {(int32_t)b, (int32_t)(g0 + cb), (int32_t)std::min<int64_t>(32, ng - cb),
                               (int32_t)woff, (int32_t)wlen, 0, 0, 0};
        citems.insert(citems.end(), it, it + 8);
      }
      for (int64_t j = 0; j * far_chunk < wlen; ++j) {
        const int64_t c0 = j * far_chunk, clen = std::min<int64_t>(far_chunk, wlen - c0);
        if (!packed) {
          emit(fitems, woff + c0, clen, g0, base[b] + (nchunks + j) * nc + gl, ng,
               far_lg(ng, clen, pq));
          continue;
        }
        int32_t slot0 = -1;  // the chunk's first LDS slot in the current wavefront
        for (int64_t c = g0; c < g1; ++c) {
          const int64_t np = (int64_t)qpair.size() / 4 - q_pair0;
          const int64_t nst = (int64_t)qstage.size() - q_stage0;
          if (np + clen > 64 || (slot0 < 0 && nst + clen > stage_rows)) {
            close_wave();
            slot0 = -1;
          }
          if (slot0 < 0) {
            slot0 = (int32_t)qstage.size() - q_stage0;
            for (int64_t e = 0; e < clen; ++e) qstage.push_back(t.list3f.idx[woff + c0 + e]);
          }
          const int32_t lane0 = (int32_t)qpair.size() / 4 - q_pair0;
          const int32_t u[4] = {(int32_t)(base[b] + (nchunks + j) * nc + (c - t.ctr_begin[b])),
                                lane0, (int32_t)clen, 0};
          qunit.insert(qunit.end(), u, u + 4);
          const int64_t co = t.ctr_order[c];
          double zx = 0.0, zy = 0.0;
          if (first_tgt[co] >= 0) {
            const int64_t tg = first_tgt[co];
            const double ir = 1.0 / ctx->ctr_r[co];
            zx = (ctx->tgt_xy[2 * tg] - ctx->ctr_xy[2 * co]) * ir;
            zy = (ctx->tgt_xy[2 * tg + 1] - ctx->ctr_xy[2 * co + 1]) * ir;
          }
          quz.insert(quz.end(), {zx, zy});
          for (int64_t e = 0; e < clen; ++e) {
            const int32_t fb = t.list3f.idx[woff + c0 + e];
            const int32_t pr[4] = {(int32_t)c, fb, slot0 + (int32_t)e, 0};
            qpair.insert(qpair.end(), pr, pr + 4);
            qgeo.insert(qgeo.end(), {ctx->ctr_xy[2 * co] - t.cx[fb], ctx->ctr_xy[2 * co + 1] - t.cy[fb],
                                     lside[t.level[fb]], ctx->ctr_r[co]});
          }
        }
      }
      for (int64_t c = g0; c < g1; ++c) clist.push_back((int32_t)c);
    }
    bk.near1 = (int64_t)items.size() / 8;
    bk.nmf1 = (int64_t)mitems.size() / 8;
    bk.nvf1 = (int64_t)vitems.size() / 8;
    bk.cv1 = (int64_t)citems.size() / 8;
    close_wave();
    bk.far1 = (int64_t)fitems.size() / 8;
    bk.m2q1 = (int64_t)qwave.size() / 8;
    bk.ctr1 = (int64_t)clist.size();
    if (bk.ctr1 > bk.ctr0) ctx->buckets.push_back(bk);
  }
  ctx->n_near_items = (int64_t)items.size() / 8;
  ctx->n_far_items = (int64_t)fitems.size() / 8;
  ctx->n_m2q_waves = (int64_t)qwave.size() / 8;
  // the packed Stage 5b lists must stay inside what k_m2qbxl_packed indexes: 64 lanes, the LDS
  // slots it stages, the rows of the near-row layout
  for (int64_t w = 0; w < ctx->n_m2q_waves; ++w) {
    const int32_t *q = &qwave[8 * w];
    bool ok = q[1] >= 1 && q[1] <= 64 && q[3] >= 1 && q[3] <= stage_rows && q[5] >= 1;
    for (int32_t i = 0; ok && i < q[1]; ++i) {
      const int32_t *pr = &qpair[4 * (q[0] + i)];
      ok = pr[2] >= 0 && pr[2] < q[3] && qstage[q[2] + pr[2]] == pr[1];
    }
    for (int32_t i = 0; ok && i < q[5]; ++i) {
      const int32_t *u = &qunit[4 * (q[4] + i)];
      ok = u[0] >= 0 && u[0] < rows && u[1] >= 0 && u[2] >= 1 && u[1] + u[2] <= q[1];
    }
    if (!ok) return fail(ctx, GQ_EINVAL, "internal: packed List 3 far work list out of bounds");
  }
  ctx->n_near_rows = rows;
  ctx->n_m2q_pairs = (int64_t)qpair.size() / 4;
  ctx->n_m2q_units = (int64_t)qunit.size() / 4;
  if (ctx->device < 0) return GQ_OK;
  // these buffers live in nw_allocations (re-uploaded when the orders change)
  std::vector<void *> saved;
  saved.swap(ctx->allocations);
  gq_status st = GQ_OK;
  if (st == GQ_OK) st = upload(ctx, d.near_src, src.data(), src.size());
  if (st == GQ_OK) st = upload(ctx, d.near_items, items.data(), items.size() / 4);
  if (st == GQ_OK) st = upload(ctx, d.near_mitems, mitems.data(), mitems.size() / 4);
  if (st == GQ_OK) st = upload(ctx, d.near_vitems, vitems.data(), vitems.size() / 4);
  if (st == GQ_OK) st = upload(ctx, d.cval_items, citems.data(), citems.size() / 4);
  if (st == GQ_OK) st = upload(ctx, d.far_items, fitems.data(), fitems.size() / 4);
  if (st == GQ_OK) st = upload(ctx, d.m2q_wave, qwave.data(), qwave.size() / 4);
  std::vector<int32_t> qslot(qpair.size() / 4);
  for (size_t i = 0; i < qslot.size(); ++i) qslot[i] = qpair[4 * i + 2];
  if (st == GQ_OK) st = upload(ctx, d.m2q_slot, qslot.data(), qslot.size());
  if (st == GQ_OK) st = upload(ctx, d.m2q_geo, qgeo.data(), qgeo.size() / 4);
  if (st == GQ_OK) st = upload(ctx, d.m2q_stage, qstage.data(), qstage.size());
  if (st == GQ_OK) st = upload(ctx, d.m2q_unit, qunit.data(), qunit.size() / 4);
  if (st == GQ_OK) st = upload(ctx, d.m2q_uz, quz.data(), quz.size() / 2);
  if (st == GQ_OK) st = upload(ctx, d.bctr0, bctr0.data(), nb);
  if (st == GQ_OK) st = upload(ctx, d.bctr1, bctr1.data(), nb);
  if (st == GQ_OK) st = upload(ctx, d.part_base, base.data(), nb);
  if (st == GQ_OK) st = upload(ctx, d.n_chunks, nch.data(), nb);
  if (st == GQ_OK) st = upload(ctx, d.n_near_chunks, nnear.data(), nb);
  if (st == GQ_OK) st = upload(ctx, d.ctr_list, clist.data(), clist.size());
  ctx->nw_allocations.swap(ctx->allocations);
  ctx->allocations.swap(saved);
  return st;
}

// Center arrays in tree order (positions, radii, caller index) and the CSR map from each center
// to its target slots (slot = 2 target + column).
struct CenterArrays {
  std::vector<double> xy, r;
  std::vector<int32_t> cperm, start, slot;
};

void center_arrays(const gq_ctx *ctx, CenterArrays &a) {
  const gq::Tree &t = ctx->tree;
  const int64_t nc = ctx->nc, nt = ctx->nt;
  a.xy.resize(2 * nc);
  a.r.resize(nc);
  a.cperm.resize(nc);
  std::vector<int64_t> inv(nc);
  for (int64_t k = 0; k < nc; ++k) {
    const int64_t o = t.ctr_order[k];
    inv[o] = k;
    a.cperm[k] = (int32_t)o;
    a.xy[2 * k] = ctx->ctr_xy[2 * o];
    a.xy[2 * k + 1] = ctx->ctr_xy[2 * o + 1];
    a.r[k] = ctx->ctr_r[o];
  }
  a.start.assign(nc + 1, 0);
  for (int64_t tg = 0; tg < nt; ++tg)
    for (int s = 0; s < 2; ++s)
      if (ctx->tgt_ctr[2 * tg + s] >= 0) a.start[inv[ctx->tgt_ctr[2 * tg + s]] + 1]++;
  for (int64_t k = 0; k < nc; ++k) a.start[k + 1] += a.start[k];
  a.slot.assign(a.start[nc], 0);
  std::vector<int32_t> fill(a.start.begin(), a.start.end() - 1);
  for (int64_t tg = 0; tg < nt; ++tg)
    for (int s = 0; s < 2; ++s)
      if (ctx->tgt_ctr[2 * tg + s] >= 0)
        a.slot[fill[inv[ctx->tgt_ctr[2 * tg + s]]]++] = (int32_t)(2 * tg + s);
}

gq_status upload_all(gq_ctx *ctx) {
  const gq::Tree &t = ctx->tree;
  auto &d = ctx->d;
  const int64_t ns = ctx->ns, nc = ctx->nc, nt = ctx->nt, nb = t.n_boxes();
  // sources in tree order
  {
    std::vector<double> xy(2 * ns), nrm(2 * ns), w(ns);
    std::vector<int32_t> perm(ns);
    for (int64_t i = 0; i < ns; ++i) {
      int64_t o = t.src_order[i];
      xy[2 * i] = ctx->src_xy[2 * o]; xy[2 * i + 1] = ctx->src_xy[2 * o + 1];
      nrm[2 * i] = ctx->src_nrm[2 * o]; nrm[2 * i + 1] = ctx->src_nrm[2 * o + 1];
      w[i] = ctx->src_w[o];
      perm[i] = (int32_t)o;
    }
    GQ_TRY(upload(ctx, d.sxy, xy.data(), ns));
    GQ_TRY(upload(ctx, d.snrm, nrm.data(), ns));
    GQ_TRY(upload(ctx, d.sw, w.data(), ns));
    GQ_TRY(upload(ctx, d.sperm, perm.data(), ns));
  }
  // centers in tree order, center -> target slots
  {
    CenterArrays ca;
    center_arrays(ctx, ca);
    GQ_TRY(upload(ctx, d.cxy, ca.xy.data(), nc));
    GQ_TRY(upload(ctx, d.cr, ca.r.data(), nc));
    GQ_TRY(upload(ctx, d.cperm, ca.cperm.data(), nc));
    GQ_TRY(upload(ctx, d.cbox, t.ctr_box.data(), nc));
    GQ_TRY(upload(ctx, d.c2t_start, ca.start.data(), nc + 1));
    GQ_TRY(upload(ctx, d.c2t_slot, ca.slot.data(), ca.slot.size()));
    ctx->one_target_per_center = true;
    for (int64_t k = 0; k < nc; ++k)
      if (ca.start[k + 1] - ca.start[k] > 1) ctx->one_target_per_center = false;
    GQ_TRY(upload(ctx, d.txy, ctx->tgt_xy.data(), nt));
    GQ_TRY(upload(ctx, d.tctr, ctx->tgt_ctr.data(), 2 * nt));
  }
  // boxes
  {
    std::vector<double> bc(2 * nb);
    std::vector<int32_t> s0(nb), s1(nb), tboxes;
    for (int64_t b = 0; b < nb; ++b) {
      bc[2 * b] = t.cx[b]; bc[2 * b + 1] = t.cy[b];
      s0[b] = (int32_t)t.src_begin[b]; s1[b] = (int32_t)t.src_end[b];
      if (t.has_tgt[b]) tboxes.push_back((int32_t)b);
    }
    ctx->n_tboxes = (int64_t)tboxes.size();
    GQ_TRY(upload(ctx, d.bc, bc.data(), nb));
    GQ_TRY(upload(ctx, d.blevel, t.level.data(), nb));
    GQ_TRY(upload(ctx, d.bparent, t.parent.data(), nb));
    GQ_TRY(upload(ctx, d.bchild, t.child.data(), 4 * nb));
    GQ_TRY(upload(ctx, d.bsrc0, s0.data(), nb));
    GQ_TRY(upload(ctx, d.bsrc1, s1.data(), nb));
    // box sides per level (a forest: per virtual level, one per tree and depth)
    std::vector<double> side = t.level_side_table;
    if (side.empty())
      for (int l = 0; l < t.n_levels; ++l) side.push_back(std::ldexp(t.side, -l));
    std::vector<double> iside(side.size()), lside(side.size());
    for (size_t l = 0; l < side.size(); ++l) {
      iside[l] = 1.0 / side[l];
      lside[l] = std::log(side[l]);
    }
    GQ_TRY(upload(ctx, d.level_side, side.data(), side.size()));
    GQ_TRY(upload(ctx, d.level_inv_side, iside.data(), iside.size()));
    GQ_TRY(upload(ctx, d.level_log_side, lside.data(), lside.size()));
  }
  // Stage 7 gather lists: every box owning centers, with its ancestors (top-down) that receive
  // List 2 or List 4 far contributions of their own, and the two shift ratios of each pair; a box
  // without such ancestors gets one empty pair. Cut after whole boxes into runs of at least
  // kM2LRun pairs, one per wavefront.
  {
    std::vector<int32_t> pr, item, chain;
    std::vector<double> tw;
    std::vector<double> side = t.level_side_table;
    if (side.empty())
      for (int l = 0; l < t.n_levels; ++l) side.push_back(std::ldexp(t.side, -l));
    int64_t sinks = 0;
    int32_t first = 0;
    for (int64_t b = 0; b < nb; ++b) {
      if (t.ctr_end[b] <= t.ctr_begin[b]) continue;
      ++sinks;
      chain.clear();
      for (int32_t a = t.parent[b]; a >= 0; a = t.parent[a])
        if (t.list2.row_size(a) > 0 || t.list4f.row_size(a) > 0) chain.push_back(a);
      if (chain.empty()) {
        pr.insert(pr.end(), {-1, (int32_t)b});
        tw.insert(tw.end(), {0.0, 0.0, 1.0, 0.0});
      }
      for (auto it = chain.rbegin(); it != chain.rend(); ++it) {
        const int32_t a = *it;
        const std::complex<double> dc(t.cx[b] - t.cx[a], t.cy[b] - t.cy[a]);
        const std::complex<double> tt = dc / side[t.level[a]], w = side[t.level[b]] / dc;
        tw.insert(tw.end(), {tt.real(), tt.imag(), w.real(), w.imag()});
        pr.insert(pr.end(), {a, (int32_t)b});
      }
      const int32_t n = (int32_t)pr.size() / 2;
      if (n - first >= kM2LRun) {
        item.insert(item.end(), {first, n});
        first = n;
      }
    }
    if ((int32_t)pr.size() / 2 > first) item.insert(item.end(), {first, (int32_t)pr.size() / 2});
    ctx->n_l2g_sinks = sinks;
    ctx->n_l2g_items = (int64_t)item.size() / 2;
    if (!item.empty()) {
      GQ_TRY(upload(ctx, d.l2g_item, item.data(), item.size() / 2));
      GQ_TRY(upload(ctx, d.l2g_pr, pr.data(), pr.size() / 2));
      GQ_TRY(upload(ctx, d.l2g_tw, tw.data(), tw.size() / 4));
    }
  }
  // Stage 2 work: every box whose multipole M2L (List 2) or M2QBXL (List 3 far) reads, its
  // subtree sources in items of at most kMomentChunk; split boxes first, each chunk writing a
  // partial that k_m_reduce sums in order
  {
    std::vector<uint8_t> need(nb, 0);
    for (int32_t x : t.list2.idx) need[x] = 1;
    for (int32_t x : t.list3f.idx) need[x] = 1;
    std::vector<int32_t> item, red;
    int32_t parts = 0;
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t s0 = t.src_begin[b], s1 = t.src_end[b];
      if (!need[b] || s1 - s0 <= kMomentChunk) continue;
      red.insert(red.end(), {(int32_t)b, parts, 0, 0});
      for (int64_t c0 = s0; c0 < s1; c0 += kMomentChunk)
        item.insert(item.end(), {(int32_t)b, (int32_t)c0,
                                 (int32_t)std::min<int64_t>(s1, c0 + kMomentChunk), parts++});
      red[red.size() - 2] = parts;
    }
    for (int64_t b = 0; b < nb; ++b)
      if (need[b] && t.src_end[b] - t.src_begin[b] <= kMomentChunk)
        item.insert(item.end(), {(int32_t)b, (int32_t)t.src_begin[b], (int32_t)t.src_end[b], -1});
    ctx->n_p2m_items = (int64_t)item.size() / 4;
    ctx->n_p2m_red = (int64_t)red.size() / 4;
    ctx->n_p2m_parts = parts;
    if (!item.empty()) GQ_TRY(upload(ctx, d.p2m_item, item.data(), item.size() / 4));
    if (!red.empty()) GQ_TRY(upload(ctx, d.p2m_red, red.data(), red.size() / 4));
  }
  // Stage 4 work: the List 2 pairs of the target-or-ancestor boxes in box order (a box without
  // pairs gets one empty pair so that its local is written), cut after whole boxes into runs of
  // at least kM2LRun pairs, one per wavefront
  {
    std::vector<double> side = t.level_side_table;
    if (side.empty())
      for (int l = 0; l < t.n_levels; ++l) side.push_back(std::ldexp(t.side, -l));
    const std::vector<double> &olog = ctx->tables.ologabs;
    std::vector<int32_t> pr, item;
    std::vector<double> plog;
    int32_t first = 0;
    for (int64_t b = 0; b < nb; ++b) {
      if (!t.has_tgt[b]) continue;
      const double ls = std::log(side[t.level[b]]);
      if (t.list2.row_size(b) == 0) {
        pr.insert(pr.end(), {-1, 0, (int32_t)b, 0});
        plog.push_back(0.0);
      }
      for (int64_t e = t.list2.start[b]; e < t.list2.start[b + 1]; ++e) {
        const int32_t o = t.list2_offset[e];
        pr.insert(pr.end(), {t.list2.idx[e], o, (int32_t)b, 0});
        plog.push_back(ls + olog[o]);
      }
      const int32_t n = (int32_t)plog.size();
      if (n - first >= kM2LRun) {
        item.insert(item.end(), {first, n});
        first = n;
      }
    }
    if ((int32_t)plog.size() > first) item.insert(item.end(), {first, (int32_t)plog.size()});
    ctx->n_m2l_items = (int64_t)item.size() / 2;
    if (!item.empty()) {
      GQ_TRY(upload(ctx, d.m2l_item, item.data(), item.size() / 2));
      GQ_TRY(upload(ctx, d.m2l_pr, pr.data(), pr.size() / 4));
      GQ_TRY(upload(ctx, d.m2l_plog, plog.data(), plog.size()));
    }
    // The same pairs for density batches, grouped by target parent: siblings share most of
    // their List 2 boxes, so every group record is one source box with the offset of each member
    // that lists it (a byte, 0xFF: none), and a source multipole is read once for up to four
    // targets. The offsets are renumbered to the ones List 2 uses (a compact o^-k table).
    std::vector<int32_t> cmap(121, -1), used;
    for (int32_t o : t.list2_offset)
      if (cmap[o] < 0) {
        cmap[o] = (int32_t)used.size();
        used.push_back(o);
      }
    std::vector<int32_t> gkey(nb + 1, -1), grp, rec, gitem;
    std::vector<double> gplog;
    for (int64_t b = 0; b < nb; ++b) {
      if (!t.has_tgt[b]) continue;
      const int64_t key = t.parent[b] >= 0 ? t.parent[b] : nb;
      if (gkey[key] < 0 || grp[4 * gkey[key] + 3] >= 0) {
        gkey[key] = (int32_t)grp.size() / 4;
        grp.insert(grp.end(), {-1, -1, -1, -1});
      }
      int32_t *gm = &grp[4 * gkey[key]];
      int q = 0;
      while (gm[q] >= 0) ++q;
      gm[q] = (int32_t)b;
    }
    const int32_t ngrp = (int32_t)grp.size() / 4;
    std::vector<std::array<int32_t, 3>> ent;  // (d, member, compact offset)
    int32_t gfirst = 0, work = 0;
    for (int32_t gi = 0; gi < ngrp; ++gi) {
      ent.clear();
      for (int q = 0; q < 4; ++q) {
        const int32_t b = grp[4 * gi + q];
        if (b < 0) continue;
        for (int64_t e = t.list2.start[b]; e < t.list2.start[b + 1]; ++e)
          ent.push_back({t.list2.idx[e], q, cmap[t.list2_offset[e]]});
      }
      std::stable_sort(ent.begin(), ent.end(),
                       [](const auto &x, const auto &y) { return x[0] < y[0]; });
      const double ls = std::log(side[t.level[grp[4 * gi]]]);
      if (ent.empty()) {
        rec.insert(rec.end(), {-1, -1, gi, 0});
        gplog.insert(gplog.end(), {0.0, 0.0, 0.0, 0.0});
      }
      for (size_t e0 = 0; e0 < ent.size();) {
        size_t e1 = e0;
        uint32_t packed = 0xFFFFFFFFu;
        double pl[4] = {0.0, 0.0, 0.0, 0.0};
        for (; e1 < ent.size() && ent[e1][0] == ent[e0][0]; ++e1) {
          const int q = ent[e1][1];
          packed = (packed & ~(0xFFu << (8 * q))) | ((uint32_t)ent[e1][2] << (8 * q));
          pl[q] = ls + olog[used[ent[e1][2]]];
        }
        rec.insert(rec.end(), {ent[e0][0], (int32_t)packed, gi, 0});
        gplog.insert(gplog.end(), pl, pl + 4);
        e0 = e1;
      }
      work += std::max<int32_t>(1, (int32_t)ent.size());
      if (work >= kM2LRun) {
        gitem.insert(gitem.end(), {gfirst, (int32_t)rec.size() / 4});
        gfirst = (int32_t)rec.size() / 4;
        work = 0;
      }
    }
    if ((int32_t)rec.size() / 4 > gfirst) gitem.insert(gitem.end(), {gfirst, (int32_t)rec.size() / 4});
    ctx->n_m2g_items = (int64_t)gitem.size() / 2;
    ctx->m2g_n_off = (int32_t)used.size();
    if (!gitem.empty()) {
      const int P1 = ctx->params.p_fmm + 1;
      std::vector<double> op((size_t)used.size() * P1 * 2);
      for (size_t u = 0; u < used.size(); ++u)
        std::copy_n(ctx->tables.opow.begin() + (size_t)used[u] * P1 * 2, (size_t)P1 * 2,
                    op.begin() + u * P1 * 2);
      GQ_TRY(upload(ctx, d.m2g_item, gitem.data(), gitem.size() / 2));
      GQ_TRY(upload(ctx, d.m2g_rec, rec.data(), rec.size() / 4));
      GQ_TRY(upload(ctx, d.m2g_plog, gplog.data(), gplog.size() / 4));
      GQ_TRY(upload(ctx, d.m2g_grp, grp.data(), grp.size() / 4));
      GQ_TRY(upload(ctx, d.m2g_opow, op.data(), op.size() / 2));
      if (ctx->params.precision == GQ_MIXED_FP32) {
        const std::vector<float> opf(op.begin(), op.end());
        GQ_TRY(upload(ctx, d.m2g_opow_f, opf.data(), opf.size() / 2));
      }
    }
  }
  // Stage 6b work: per box, the sources of its List 4 far boxes (tree order, box by box)
  {
    std::vector<int32_t> item, src;
    for (int64_t b = 0; b < nb; ++b) {
      const int32_t first = (int32_t)src.size();
      for (int64_t e = t.list4f.start[b]; e < t.list4f.start[b + 1]; ++e) {
        const int32_t dd = t.list4f.idx[e];
        for (int64_t s = t.src_begin[dd]; s < t.src_end[dd]; ++s) src.push_back((int32_t)s);
      }
      if ((int32_t)src.size() > first)
        item.insert(item.end(), {(int32_t)b, first, (int32_t)src.size(), 0});
    }
    ctx->n_p2l_boxes = (int64_t)item.size() / 4;
    if (!item.empty()) {
      GQ_TRY(upload(ctx, d.p2l_item, item.data(), item.size() / 4));
      GQ_TRY(upload(ctx, d.p2l_src, src.data(), src.size()));
    }
  }
  // lists
  GQ_TRY(upload(ctx, d.wf_idx, t.list3f.idx.data(), t.list3f.idx.size()));
  GQ_TRY(build_near_work(ctx));

  // tables
  const gq::Tables &tb = ctx->tables;
  const int P1 = ctx->params.p_fmm + 1, PQ = ctx->params.p_qbx;
  GQ_TRY(upload(ctx, d.m2l_bt, tb.m2l_bt.data(), tb.m2l_bt.size()));
  if (ctx->params.precision == GQ_MIXED_FP32) {
    auto f32 = [](const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); };
    const std::vector<float> bt = f32(tb.m2l_bt), op = f32(tb.opow);
    GQ_TRY(upload(ctx, d.m2l_bt_f, bt.data(), bt.size()));
    GQ_TRY(upload(ctx, d.opow_f, op.data(), op.size() / 2));
  }
  GQ_TRY(upload(ctx, d.opow, tb.opow.data(), tb.opow.size() / 2));
  {
    const int NB = tb.nbinom;
    auto C = [&](int n, int k) { return (k < 0 || k > n || n >= NB) ? 0.0 : tb.binom[(size_t)n * NB + k]; };
    std::vector<double> l2q((size_t)P1 * (PQ + 1));
    for (int k = 0; k < P1; ++k)
      for (int m = 0; m <= PQ; ++m) l2q[(size_t)k * (PQ + 1) + m] = C(k, m);
    GQ_TRY(upload(ctx, d.l2q_binom, l2q.data(), l2q.size()));
    std::vector<double> m2q((size_t)P1 * (PQ + 1), 0.0);
    for (int k = 1; k < P1; ++k)
      for (int m = 0; m <= PQ; ++m) m2q[(size_t)k * (PQ + 1) + m] = C(k + m - 1, m);
    GQ_TRY(upload(ctx, d.m2q_binom, m2q.data(), m2q.size()));
    std::vector<double> bt((size_t)P1 * P1);
    for (int k = 0; k < P1; ++k)
      for (int m = 0; m < P1; ++m) bt[(size_t)k * P1 + m] = C(k, m);
    GQ_TRY(upload(ctx, d.l2g_binom_t, bt.data(), bt.size()));
  }
  return GQ_OK;
}

// Per-density buffers (strengths, box expansions, center rows, target slots) for nd densities;
// grows on demand (synchronising the context's streams before freeing the old buffers).
gq_status ensure_workspace(gq_ctx *ctx, int nd) {
  if (nd <= ctx->ws_batch) return GQ_OK;
  free_workspace(ctx);
  auto &d = ctx->d;
  const size_t n = (size_t)nd, P1 = ctx->params.p_fmm + 1, nb = ctx->tree.n_boxes();
  GQ_TRY(alloc_ws(ctx, d.sq, n * ctx->ns));
  GQ_TRY(alloc_ws(ctx, d.sdip, n * ctx->ns));
  GQ_TRY(alloc_ws(ctx, d.M, n * nb * P1));
  GQ_TRY(alloc_ws(ctx, d.L, n * nb * P1));
  GQ_TRY(alloc_ws(ctx, d.Lf, n * nb * P1));
  GQ_TRY(alloc_ws(ctx, d.Mp, n * (size_t)std::max<int64_t>(ctx->n_p2m_parts, 1) * 2 * P1));
  GQ_TRY(alloc_ws(ctx, d.anear, n * std::max<int64_t>(ctx->n_near_rows, 1) * (ctx->params.p_qbx + 1)));
  GQ_TRY(alloc_ws(ctx, d.nval, n * std::max<int64_t>(ctx->n_near_rows, 1)));
  GQ_TRY(alloc_ws(ctx, d.tv, n * 2 * ctx->nt));
  ctx->ws_batch = nd;
  return GQ_OK;
}

// ---- scratch of the allocation-free evaluation (gq_eval_noalloc) ----
// A file-scope device array: every GPU the library runs on holds its own copy, from the first
// use of this code object on that device until the process ends. In host code the name
// `scratch` is only a host-side stand-in; kernels get the device address of each GPU's copy,
// taken once per device with hipGetSymbolAddress when a context is created there.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Once per device, with that device current: the address of its copy of `scratch`.
hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

// Bytes of per-density workspace (strengths, box expansions, center rows, target slots) for
// `slots` workspace slots, each buffer rounded up to 256 bytes.
size_t workspace_bytes(const gq_ctx *ctx, int slots) {
  const size_t n = (size_t)slots, P1 = ctx->params.p_fmm + 1, nb = ctx->tree.n_boxes();
  auto r = [](size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; };
  return r(n * ctx->ns * sizeof(double)) + r(n * ctx->ns * sizeof(double2)) +
         3 * r(n * nb * P1 * sizeof(double2)) +
         r(n * (size_t)std::max<int64_t>(ctx->n_p2m_parts, 1) * 2 * P1 * sizeof(double2)) +
         r(n * (size_t)std::max<int64_t>(ctx->n_near_rows, 1) * (ctx->params.p_qbx + 1) *
           sizeof(double2)) +
         r(n * (size_t)std::max<int64_t>(ctx->n_near_rows, 1) * sizeof(double)) +
         r(n * 2 * ctx->nt * sizeof(double));
}

// Point the context's workspace at `base` (workspace_bytes(ctx, slots) bytes, 256-aligned), in
// the order and sizes of workspace_bytes.
void carve_workspace(gq_ctx *ctx, int slots, unsigned char *base) {
  const size_t n = (size_t)slots, P1 = ctx->params.p_fmm + 1, nb = ctx->tree.n_boxes();
  auto r = [](size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; };
  auto take = [&](size_t bytes) {
    unsigned char *p = base;
    base += r(bytes);
    return p;
  };
  auto &d = ctx->d;
  d.sq = reinterpret_cast<double *>(take(n * ctx->ns * sizeof(double)));
  d.sdip = reinterpret_cast<double2 *>(take(n * ctx->ns * sizeof(double2)));
  d.M = reinterpret_cast<double2 *>(take(n * nb * P1 * sizeof(double2)));
  d.L = reinterpret_cast<double2 *>(take(n * nb * P1 * sizeof(double2)));
  d.Lf = reinterpret_cast<double2 *>(take(n * nb * P1 * sizeof(double2)));
  d.Mp = reinterpret_cast<double2 *>(
      take(n * (size_t)std::max<int64_t>(ctx->n_p2m_parts, 1) * 2 * P1 * sizeof(double2)));
  d.anear = reinterpret_cast<double2 *>(
      take(n * (size_t)std::max<int64_t>(ctx->n_near_rows, 1) * (ctx->params.p_qbx + 1) *
           sizeof(double2)));
  d.nval = reinterpret_cast<double *>(
      take(n * (size_t)std::max<int64_t>(ctx->n_near_rows, 1) * sizeof(double)));
  d.tv = reinterpret_cast<double *>(take(n * 2 * ctx->nt * sizeof(double)));
}

bool finite_all(const std::vector<double> &v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

// One kind of a GQ_S_AND_D evaluation on library stream `s` (no side stream), with every
// workspace pointer moved past the first `slot0` densities' workspace.
gq_status launch_kind_on(gq_ctx *ctx, hipStream_t s, int kind, const double *d1, int64_t ld1,
                         double *out, int64_t ld_out, int nd, int slot0, bool direct) {
  gq::DevBuffers saved = ctx->d;
  const hipStream_t st = ctx->stream;
  const int overlap = ctx->params.overlap;
  const int64_t P1 = ctx->params.p_fmm + 1, nb = ctx->tree.n_boxes();
  ctx->d.sq += (int64_t)slot0 * ctx->ns;
  ctx->d.sdip += (int64_t)slot0 * ctx->ns;
  ctx->d.M += (int64_t)slot0 * nb * P1;
  ctx->d.L += (int64_t)slot0 * nb * P1;
  ctx->d.Lf += (int64_t)slot0 * nb * P1;
  ctx->d.anear += (int64_t)slot0 * ctx->n_near_rows * (ctx->params.p_qbx + 1);
  ctx->d.nval += (int64_t)slot0 * ctx->n_near_rows;
  ctx->d.tv += (int64_t)slot0 * 2 * ctx->nt;
  ctx->stream = s;
  ctx->params.overlap = 0;
  hipError_t e = gq::run_eval(ctx, kind, d1, ld1, nullptr, 0, out, ld_out, nd, direct);
  ctx->d = saved;
  ctx->stream = st;
  ctx->params.overlap = overlap;
  if (e != hipSuccess) return fail(ctx, GQ_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return GQ_OK;
}

// GQ_S_AND_D for one batch: S on library stream 1 (workspace slots [0, batch)), D on library
// stream 2 (slots [batch, 2 batch)), both forked from and joined back to the caller's stream.
gq_status ensure_pair_streams(gq_ctx *ctx) {
  if (ctx->main1) return GQ_OK;
  GQ_HIP(ctx, hipStreamCreateWithFlags(&ctx->main1, hipStreamNonBlocking));
  GQ_HIP(ctx, hipStreamCreateWithFlags(&ctx->main2, hipStreamNonBlocking));
  GQ_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_pair_in, hipEventDisableTiming));
  GQ_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_pair_out1, hipEventDisableTiming));
  GQ_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_pair_out2, hipEventDisableTiming));
  return GQ_OK;
}

gq_status launch_s_and_d(gq_ctx *ctx, const double *d1, int64_t ld1, double *out_s,
                         double *out_d, int64_t ld_out, int nd, int batch, bool direct) {
  GQ_TRY(ensure_pair_streams(ctx));
  GQ_HIP(ctx, hipEventRecord(ctx->ev_pair_in, ctx->stream));
  GQ_HIP(ctx, hipStreamWaitEvent(ctx->main1, ctx->ev_pair_in, 0));
  GQ_HIP(ctx, hipStreamWaitEvent(ctx->main2, ctx->ev_pair_in, 0));
  GQ_TRY(launch_kind_on(ctx, ctx->main1, GQ_S, d1, ld1, out_s, ld_out, nd, 0, direct));
  GQ_TRY(launch_kind_on(ctx, ctx->main2, GQ_D, d1, ld1, out_d, ld_out, nd, batch, direct));
  GQ_HIP(ctx, hipEventRecord(ctx->ev_pair_out1, ctx->main1));
  GQ_HIP(ctx, hipEventRecord(ctx->ev_pair_out2, ctx->main2));
  GQ_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_pair_out1, 0));
  GQ_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_pair_out2, 0));
  return GQ_OK;
}

gq_status launch_batches(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1, int64_t ld1,
                         const double *dens2, int64_t ld2, double *out, int64_t ld_out,
                         bool direct) {
  if (kind == GQ_S_AND_D) {
    // FMM: one expansion pipeline over 2 nd workspace slots (S in the first nd, D in the rest);
    // direct QBX: the two kinds on two library streams
    const int batch = (int)std::min<int64_t>(n_dens, gq::kMaxDensBatch / 2);
    for (int64_t j = 0; j < n_dens; j += batch) {
      const int nd = (int)std::min<int64_t>(batch, n_dens - j);
      if (direct) {
        GQ_TRY(launch_s_and_d(ctx, dens1 + j * ld1, ld1, out + j * ld_out,
                              out + (n_dens + j) * ld_out, ld_out, nd, batch, direct));
        continue;
      }
      hipError_t e = gq::run_eval(ctx, 4, dens1 + j * ld1, ld1, nullptr, 0, out + j * ld_out,
                                  ld_out, nd, false, out + (n_dens + j) * ld_out);
      if (e != hipSuccess) return fail(ctx, GQ_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return GQ_OK;
  }
  const int batch = (int)std::min<int64_t>(n_dens, gq::kMaxDensBatch);
  for (int64_t j = 0; j < n_dens; j += batch) {
    const int nd = (int)std::min<int64_t>(batch, n_dens - j);
    hipError_t e = gq::run_eval(ctx, kind, dens1 + j * ld1, ld1, dens2 ? dens2 + j * ld2 : nullptr,
                                ld2, out + j * ld_out, ld_out, nd, direct);
    if (e != hipSuccess) return fail(ctx, GQ_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  }
  return GQ_OK;
}

// Workspace slots an evaluation needs: one per density of a batch, two for GQ_S_AND_D.
int workspace_batch(int kind, int64_t n_dens) {
  if (kind == GQ_S_AND_D) return 2 * (int)std::min<int64_t>(n_dens, gq::kMaxDensBatch / 2);
  return (int)std::min<int64_t>(n_dens, gq::kMaxDensBatch);
}

gq_status check_eval_args(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1,
                          int64_t ld1, const double *dens2, int64_t ld2, const double *out,
                          int64_t ld_out) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (ctx->device < 0) return fail(ctx, GQ_ESTATE, "host-only context cannot evaluate");
  if (!ctx->built) return fail(ctx, GQ_ESTATE, "gq_eval before a successful gq_build");
  if (kind < GQ_S || kind > GQ_SP) return fail(ctx, GQ_EINVAL, "unknown kind");
  if (kind == GQ_SP && !ctx->tnrm_dev)
    return fail(ctx, GQ_ESTATE, "GQ_SP needs the target normals (gq_set_target_normals)");
  if (n_dens < 0) return fail(ctx, GQ_EINVAL, "n_dens < 0");
  if (n_dens == 0) return GQ_OK;
  if (!dens1 || !out) return fail(ctx, GQ_EINVAL, "null density or output");
  if ((kind == GQ_S_MINUS_D) != (dens2 != nullptr))
    return fail(ctx, GQ_EINVAL, "dens2 must be given exactly for GQ_S_MINUS_D");
  if (ld1 < ctx->ns || (dens2 && ld2 < ctx->ns) || ld_out < ctx->nt)
    return fail(ctx, GQ_EINVAL, "leading dimension smaller than the row length");
  return GQ_OK;
}

gq_status eval_common(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1, int64_t ld1,
                      const double *dens2, int64_t ld2, double *out, int64_t ld_out, bool direct) {
  GQ_TRY(check_eval_args(ctx, kind, n_dens, dens1, ld1, dens2, ld2, out, ld_out));
  if (n_dens == 0) return GQ_OK;
  GQ_HIP(ctx, hipSetDevice(ctx->device));
  GQ_TRY(ensure_workspace(ctx, workspace_batch(kind, n_dens)));
  return launch_batches(ctx, kind, n_dens, dens1, ld1, dens2, ld2, out, ld_out, direct);
}

// Shared by gq_set_geometry (n_geom = 1, null offsets) and gq_set_geometry_batch.
gq_status set_geometry_impl(gq_ctx *ctx, int mem, int64_t n_geom, const int64_t *src_off,
                            const int64_t *ctr_off, const int64_t *tgt_off, int64_t n_src,
                            const double *src_xy, const double *src_nrm, const double *src_w,
                            int64_t n_ctr, const double *ctr_xy, const double *ctr_r,
                            int64_t n_tgt, const double *tgt_xy, const int32_t *tgt_ctr) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (mem != GQ_MEM_HOST && mem != GQ_MEM_DEVICE) return fail(ctx, GQ_EINVAL, "mem must be GQ_MEM_HOST or GQ_MEM_DEVICE");
  if (mem == GQ_MEM_DEVICE && ctx->device < 0) return fail(ctx, GQ_ESTATE, "device memory on a host-only context");
  if (n_src <= 0 || n_ctr < 0 || n_tgt < 0) return fail(ctx, GQ_EINVAL, "need n_src > 0, n_ctr >= 0, n_tgt >= 0");
  if (n_src >= (int64_t(1) << 31) || n_ctr >= (int64_t(1) << 31) || 2 * n_tgt >= (int64_t(1) << 31))
    return fail(ctx, GQ_EUNSUP, "sizes beyond 2^31 are not supported");
  if (!src_xy || !src_nrm || !src_w || (n_ctr > 0 && (!ctr_xy || !ctr_r)) ||
      (n_tgt > 0 && (!tgt_xy || !tgt_ctr)))
    return fail(ctx, GQ_EINVAL, "null geometry pointer");
  // geometry offsets (host): start at 0, non-decreasing, end at the totals, >= 1 source each
  std::vector<int64_t> so{0, n_src}, co{0, n_ctr}, to{0, n_tgt};
  if (n_geom != 1 || src_off) {
    if (n_geom < 1 || !src_off || !ctr_off || !tgt_off) return fail(ctx, GQ_EINVAL, "need n_geom >= 1 and three offset arrays");
    so.assign(src_off, src_off + n_geom + 1);
    co.assign(ctr_off, ctr_off + n_geom + 1);
    to.assign(tgt_off, tgt_off + n_geom + 1);
    if (so[0] || co[0] || to[0] || so[n_geom] != n_src || co[n_geom] != n_ctr || to[n_geom] != n_tgt)
      return fail(ctx, GQ_EINVAL, "offsets must start at 0 and end at the totals");
    for (int64_t k = 0; k < n_geom; ++k)
      if (so[k + 1] <= so[k] || co[k + 1] < co[k] || to[k + 1] < to[k])
        return fail(ctx, GQ_EINVAL, "offsets must increase (every geometry needs a source)");
  }
  free_device(ctx);
  drop_target_normals(ctx);
  ctx->have_geom = false;
  ctx->ns = n_src; ctx->nc = n_ctr; ctx->nt = n_tgt;
  ctx->nc_user = n_ctr; ctx->n_pt = 0;
  ctx->n_geom = n_geom;
  ctx->geom_src_off = so; ctx->geom_ctr_off = co; ctx->geom_tgt_off = to;
  ctx->pt_geom.clear();
  try {
    ctx->src_xy.resize(2 * n_src); ctx->src_nrm.resize(2 * n_src); ctx->src_w.resize(n_src);
    ctx->ctr_xy.resize(2 * n_ctr); ctx->ctr_r.resize(n_ctr);
    ctx->tgt_xy.resize(2 * n_tgt); ctx->tgt_ctr.resize(2 * n_tgt);
  } catch (const std::bad_alloc &) {
    return fail(ctx, GQ_ENOMEM, "host copy of the geometry");
  }
  struct { void *dst; const void *src; size_t bytes; } cp[] = {
      {ctx->src_xy.data(), src_xy, sizeof(double) * 2 * n_src},
      {ctx->src_nrm.data(), src_nrm, sizeof(double) * 2 * n_src},
      {ctx->src_w.data(), src_w, sizeof(double) * n_src},
      {ctx->ctr_xy.data(), ctr_xy, sizeof(double) * 2 * n_ctr},
      {ctx->ctr_r.data(), ctr_r, sizeof(double) * n_ctr},
      {ctx->tgt_xy.data(), tgt_xy, sizeof(double) * 2 * n_tgt},
      {ctx->tgt_ctr.data(), tgt_ctr, sizeof(int32_t) * 2 * n_tgt}};
  for (auto &c : cp) {
    if (!c.bytes) continue;
    if (mem == GQ_MEM_HOST) std::memcpy(c.dst, c.src, c.bytes);
    else GQ_HIP(ctx, hipMemcpy(c.dst, c.src, c.bytes, hipMemcpyDeviceToHost));
  }
  if (!finite_all(ctx->src_xy) || !finite_all(ctx->src_nrm) || !finite_all(ctx->src_w) ||
      !finite_all(ctx->ctr_xy) || !finite_all(ctx->ctr_r) || !finite_all(ctx->tgt_xy))
    return fail(ctx, GQ_EINVAL, "non-finite geometry value");
  for (double r : ctx->ctr_r)
    if (!(r > 0)) return fail(ctx, GQ_EINVAL, "center radius must be positive");
  // target -> center indices: local to the target's geometry in a batch, made global here
  std::vector<int64_t> point_targets;
  std::vector<int32_t> point_geom;
  for (int64_t k = 0; k < n_geom; ++k) {
    const int64_t nck = co[k + 1] - co[k];
    for (int64_t t = to[k]; t < to[k + 1]; ++t) {
      int used = 0;
      for (int s = 0; s < 2; ++s) {
        int32_t &c = ctx->tgt_ctr[2 * t + s];
        if (c < -1 || c >= nck) return fail(ctx, GQ_EINVAL, "target-center index out of range");
        if (c >= 0) {
          c = (int32_t)(c + co[k]);
          ++used;
        }
      }
      if (!used) {
        point_targets.push_back(t);
        point_geom.push_back((int32_t)k);
      }
    }
  }
  if (!point_targets.empty()) {
    const int64_t n_pt = (int64_t)point_targets.size();
    if (n_ctr + n_pt >= (int64_t(1) << 31)) return fail(ctx, GQ_EUNSUP, "too many centers and point targets");
    // internal radius: 2^-40 of the extent of all particles, far below any quadrature scale
    double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
    auto grow = [&](const std::vector<double> &xy) {
      for (size_t i = 0; i + 1 < xy.size(); i += 2)
        for (int a = 0; a < 2; ++a) { lo[a] = std::min(lo[a], xy[i + a]); hi[a] = std::max(hi[a], xy[i + a]); }
    };
    grow(ctx->src_xy); grow(ctx->ctr_xy); grow(ctx->tgt_xy);
    const double ext = std::max(hi[0] - lo[0], hi[1] - lo[1]);
    const double r_pt = std::ldexp(ext > 0 ? ext : 1.0, -40);
    try {
      ctx->ctr_xy.resize(2 * (n_ctr + n_pt)); ctx->ctr_r.resize(n_ctr + n_pt);
    } catch (const std::bad_alloc &) {
      return fail(ctx, GQ_ENOMEM, "host copy of the point-target centers");
    }
    for (int64_t j = 0; j < n_pt; ++j) {
      const int64_t t = point_targets[j], c = n_ctr + j;
      ctx->ctr_xy[2 * c] = ctx->tgt_xy[2 * t]; ctx->ctr_xy[2 * c + 1] = ctx->tgt_xy[2 * t + 1];
      ctx->ctr_r[c] = r_pt;
      ctx->tgt_ctr[2 * t] = (int32_t)c;
    }
    ctx->n_pt = n_pt;
    ctx->nc = n_ctr + n_pt;
    ctx->pt_geom = point_geom;
  }
  if (ctx->nc == 0) return fail(ctx, GQ_EINVAL, "need at least one center or point target");
  ctx->have_geom = true;
  return GQ_OK;
}

// One tree per geometry (threads over geometries), merged into a forest.
std::string build_forest(gq_ctx *ctx, const gq::TreeParams &tp) {
  const int64_t K = ctx->n_geom;
  std::vector<std::vector<int64_t>> cglob(K);
  for (int64_t k = 0; k < K; ++k)
    for (int64_t c = ctx->geom_ctr_off[k]; c < ctx->geom_ctr_off[k + 1]; ++c) cglob[k].push_back(c);
  for (int64_t j = 0; j < ctx->n_pt; ++j) cglob[ctx->pt_geom[j]].push_back(ctx->nc_user + j);
  std::vector<gq::Tree> trees(K);
  std::vector<std::string> msg(K);
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    std::vector<double> cxy, cr;
    for (int64_t k; (k = next.fetch_add(1)) < K;) {
      cxy.resize(2 * cglob[k].size());
      cr.resize(cglob[k].size());
      for (size_t i = 0; i < cglob[k].size(); ++i) {
        const int64_t c = cglob[k][i];
        cxy[2 * i] = ctx->ctr_xy[2 * c]; cxy[2 * i + 1] = ctx->ctr_xy[2 * c + 1];
        cr[i] = ctx->ctr_r[c];
      }
      const int64_t s0 = ctx->geom_src_off[k];
      try {
        msg[k] = gq::build_tree(trees[k], ctx->geom_src_off[k + 1] - s0, ctx->src_xy.data() + 2 * s0,
                                (int64_t)cr.size(), cxy.data(), cr.data(), tp);
      } catch (const std::bad_alloc &) {
        msg[k] = "host allocation during tree build";
      }
    }
  };
  const int nthr = (int)std::max<int64_t>(1, std::min<int64_t>(K, std::max(1u, std::thread::hardware_concurrency())));
  std::vector<std::thread> pool;
  for (int i = 1; i < nthr; ++i) pool.emplace_back(work);
  work();
  for (auto &th : pool) th.join();
  for (int64_t k = 0; k < K; ++k)
    if (!msg[k].empty()) return "geometry " + std::to_string(k) + ": " + msg[k];
  std::vector<int64_t> sbase(ctx->geom_src_off.begin(), ctx->geom_src_off.end() - 1);
  gq::merge_forest(trees, sbase, cglob, ctx->tree);
  return "";
}

}  // namespace

extern "C" {

gq_status gq_default_params(gq_params *p) {
  if (!p) return GQ_EINVAL;
  p->p_qbx = 12;
  p->p_fmm = 30;
  p->n_max = 64;
  p->count_mode = 0;
  p->t_f = 0.9;
  p->w3far_min_sources = 15;
  p->precision = GQ_FP64;
  p->max_levels = 24;
  p->overlap = 1;
  p->near_chunk = 0;
  p->far_chunk = 0;
  p->far_pairs_per_lane = 1;
  p->near_dens_group = 0;
  p->eps = 0.0;
  p->tcr_shape = 0;
  p->level_restrict = 0;
  return GQ_OK;
}

gq_status gq_create(gq_ctx **out, int device, void *hip_stream) {
  if (!out) return fail(nullptr, GQ_EINVAL, "null output pointer");
  *out = nullptr;
  if (device < -1) return fail(nullptr, GQ_EINVAL, "device must be >= -1");
  if (device >= 0) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device >= n)
      return fail(nullptr, GQ_EHIP, std::string("no HIP device ") + std::to_string(device));
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, GQ_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  }
  gq_ctx *ctx = new (std::nothrow) gq_ctx();
  if (!ctx) return fail(nullptr, GQ_ENOMEM, "context allocation failed");
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (device >= 0) {
    // default-priority, non-blocking side stream; events carry the fork/join dependencies
    if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_up, hipEventDisableTiming) != hipSuccess) {
      gq_destroy(ctx);
      return fail(nullptr, GQ_EHIP, "stream/event creation failed");
    }
    hipError_t e = gq::upload_log_table();
    if (e != hipSuccess) {
      gq_destroy(ctx);
      return fail(nullptr, GQ_EHIP, std::string("log table upload: ") + hipGetErrorString(e));
    }
    e = scratch_init(device);
    if (e != hipSuccess) {
      gq_destroy(ctx);
      return fail(nullptr, GQ_EHIP, std::string("scratch address (hipGetSymbolAddress): ") +
                                        hipGetErrorString(e));
    }
  }
  gq_default_params(&ctx->params);
  *out = ctx;
  return GQ_OK;
}

gq_status gq_destroy(gq_ctx *ctx) {
  if (!ctx) return GQ_OK;
  if (ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto &r : ctx->prof) {
      ctx->event_pool.push_back(r.a);
      ctx->event_pool.push_back(r.b);
    }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    if (ctx->main1) (void)hipStreamSynchronize(ctx->main1);
    if (ctx->main2) (void)hipStreamSynchronize(ctx->main2);
  }
  free_device(ctx);
  drop_target_normals(ctx);
  if (ctx->device >= 0) {
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->ev_up) (void)hipEventDestroy(ctx->ev_up);
    if (ctx->gev_fork) (void)hipEventDestroy(ctx->gev_fork);
    if (ctx->gev_up) (void)hipEventDestroy(ctx->gev_up);
    if (ctx->gev_join) (void)hipEventDestroy(ctx->gev_join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->main1) (void)hipStreamDestroy(ctx->main1);
    if (ctx->main2) (void)hipStreamDestroy(ctx->main2);
    if (ctx->ev_pair_in) (void)hipEventDestroy(ctx->ev_pair_in);
    if (ctx->ev_pair_out1) (void)hipEventDestroy(ctx->ev_pair_out1);
    if (ctx->ev_pair_out2) (void)hipEventDestroy(ctx->ev_pair_out2);
  }
  delete ctx;
  return GQ_OK;
}

gq_status gq_set_stream(gq_ctx *ctx, void *hip_stream) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return GQ_OK;
}

gq_status gq_set_geometry(gq_ctx *ctx, int mem, int64_t n_src, const double *src_xy,
                          const double *src_nrm, const double *src_w, int64_t n_ctr,
                          const double *ctr_xy, const double *ctr_r, int64_t n_tgt,
                          const double *tgt_xy, const int32_t *tgt_ctr) {
  return set_geometry_impl(ctx, mem, 1, nullptr, nullptr, nullptr, n_src, src_xy, src_nrm, src_w,
                           n_ctr, ctr_xy, ctr_r, n_tgt, tgt_xy, tgt_ctr);
}

gq_status gq_set_geometry_batch(gq_ctx *ctx, int mem, int64_t n_geom, const int64_t *src_off,
                                const int64_t *ctr_off, const int64_t *tgt_off, int64_t n_src,
                                const double *src_xy, const double *src_nrm, const double *src_w,
                                int64_t n_ctr, const double *ctr_xy, const double *ctr_r,
                                int64_t n_tgt, const double *tgt_xy, const int32_t *tgt_ctr) {
  if (!src_off) return fail(ctx, GQ_EINVAL, "null offsets");
  return set_geometry_impl(ctx, mem, n_geom, src_off, ctr_off, tgt_off, n_src, src_xy, src_nrm,
                           src_w, n_ctr, ctr_xy, ctr_r, n_tgt, tgt_xy, tgt_ctr);
}

gq_status gq_get_expansions(gq_ctx *ctx, int what, int64_t slot, double *dst, int64_t *count) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (!count) return fail(ctx, GQ_EINVAL, "null count");
  if (!ctx->built || ctx->device < 0) return fail(ctx, GQ_ESTATE, "no tree built on a device");
  const int64_t n = ctx->tree.n_boxes() * (ctx->params.p_fmm + 1);
  const double2 *src = nullptr;
  switch (what) {
    case GQ_EXP_MULTIPOLE: src = ctx->d.M; break;
    case GQ_EXP_LOCAL: src = ctx->d.L; break;
    case GQ_EXP_LOCAL_COMPLETE: src = ctx->d.Lf; break;
    default: return fail(ctx, GQ_EINVAL, "unknown expansion kind");
  }
  *count = n;
  if (!dst) return GQ_OK;
  if (ctx->params.precision != GQ_FP64)
    return fail(ctx, GQ_EUNSUP, "expansions are read back from FP64 contexts only");
  if (!src || slot < 0 || slot >= ctx->ws_batch)
    return fail(ctx, GQ_ESTATE, "no evaluation has filled this workspace slot");
  GQ_HIP(ctx, hipSetDevice(ctx->device));
  if (ctx->stream) GQ_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->side) GQ_HIP(ctx, hipStreamSynchronize(ctx->side));
  GQ_HIP(ctx, hipMemcpy(dst, src + slot * n, sizeof(double2) * n, hipMemcpyDeviceToHost));
  return GQ_OK;
}

gq_status gq_set_target_normals(gq_ctx *ctx, int mem, int64_t n_tgt, const double *tgt_nrm) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (!ctx->have_geom) return fail(ctx, GQ_ESTATE, "gq_set_target_normals before gq_set_geometry");
  if (mem != GQ_MEM_HOST && mem != GQ_MEM_DEVICE) return fail(ctx, GQ_EINVAL, "mem must be GQ_MEM_HOST or GQ_MEM_DEVICE");
  if (mem == GQ_MEM_DEVICE && ctx->device < 0) return fail(ctx, GQ_ESTATE, "device memory on a host-only context");
  if (n_tgt != ctx->nt) return fail(ctx, GQ_EINVAL, "n_tgt differs from the geometry's target count");
  if (n_tgt > 0 && !tgt_nrm) return fail(ctx, GQ_EINVAL, "null target normals");
  std::vector<double> h((size_t)2 * n_tgt);
  if (n_tgt > 0) {
    if (mem == GQ_MEM_HOST) std::memcpy(h.data(), tgt_nrm, sizeof(double) * h.size());
    else GQ_HIP(ctx, hipMemcpy(h.data(), tgt_nrm, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
  }
  if (!finite_all(h)) return fail(ctx, GQ_EINVAL, "non-finite target normal");
  if (ctx->device >= 0) {
    GQ_HIP(ctx, hipSetDevice(ctx->device));
    if (!ctx->tnrm_dev) {
      void *p = nullptr;
      hipError_t e = hipMalloc(&p, std::max<size_t>(h.size(), 2) * sizeof(double));
      if (e != hipSuccess) return fail(ctx, GQ_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
      ctx->tnrm_dev = static_cast<double2 *>(p);
    }
    if (ctx->stream) GQ_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (n_tgt > 0)
      GQ_HIP(ctx, hipMemcpy(ctx->tnrm_dev, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
  }
  ctx->tgt_nrm.swap(h);
  return GQ_OK;
}

gq_status gq_build(gq_ctx *ctx, const gq_params *params) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (!params) return fail(ctx, GQ_EINVAL, "null params");
  if (!ctx->have_geom) return fail(ctx, GQ_ESTATE, "gq_build before gq_set_geometry");
  gq_params p = *params;
  if (p.p_fmm <= 0) {
    // Sec. 4.1: the FMM error is of order (1/2)^(p_fmm + 1), so p_fmm ~ |log2 eps|
    if (!(p.eps > 0.0 && p.eps < 1.0))
      return fail(ctx, GQ_EINVAL, "p_fmm <= 0 needs 0 < eps < 1 to derive the FMM order");
    p.p_fmm = std::min(GQ_MAX_P_FMM, std::max(1, (int)std::ceil(-std::log2(p.eps) - 1e-9)));
  }
  if (p.p_qbx < 0 || p.p_fmm < 1) return fail(ctx, GQ_EINVAL, "orders must satisfy p_qbx >= 0, p_fmm >= 1");
  if (p.p_fmm > GQ_MAX_P_FMM) return fail(ctx, GQ_EUNSUP, "p_fmm above GQ_MAX_P_FMM");
  if (!gq::pq_supported(p.p_qbx)) return fail(ctx, GQ_EUNSUP, "p_qbx has no compiled kernel in this build");
  if (p.precision != GQ_FP64 && p.precision != GQ_MIXED_FP32)
    return fail(ctx, GQ_EINVAL, "precision must be GQ_FP64 or GQ_MIXED_FP32");
  if (p.count_mode != 0 && p.count_mode != 1) return fail(ctx, GQ_EINVAL, "count_mode must be 0 or 1");
  if (p.w3far_min_sources < 0) return fail(ctx, GQ_EINVAL, "w3far_min_sources must be >= 0");
  if (p.overlap != 0 && p.overlap != 1) return fail(ctx, GQ_EINVAL, "overlap must be 0 or 1");
  if (p.tcr_shape != 0 && p.tcr_shape != 1) return fail(ctx, GQ_EINVAL, "tcr_shape must be 0 or 1");
  if (p.level_restrict != 0 && p.level_restrict != 1)
    return fail(ctx, GQ_EINVAL, "level_restrict must be 0 or 1");
  if (p.near_chunk < 0 || p.near_chunk > (1 << 20) || p.far_chunk < 0 || p.far_chunk > 32 ||
      p.far_pairs_per_lane < 0 || p.far_pairs_per_lane > 64)
    return fail(ctx, GQ_EINVAL, "work-item shape out of range");
  if (p.near_dens_group != 0 && p.near_dens_group != 1 && p.near_dens_group != 2 &&
      p.near_dens_group != 4)
    return fail(ctx, GQ_EINVAL, "near_dens_group must be 0, 1, 2 or 4");
  free_device(ctx);
  ctx->params = p;
  ctx->pq_values.clear();
  for (int q : gq::compiled_pq()) if (q <= p.p_qbx) ctx->pq_values.push_back(q);
  auto t0 = std::chrono::steady_clock::now();
  gq::TreeParams tp;
  tp.n_max = p.n_max; tp.count_mode = p.count_mode; tp.t_f = p.t_f;
  tp.w3far_min_sources = p.w3far_min_sources; tp.max_levels = p.max_levels;
  tp.tcr_shape = p.tcr_shape; tp.level_restrict = p.level_restrict;
  std::string msg;
  try {
    if (ctx->n_geom > 1)
      msg = build_forest(ctx, tp);
    else
      msg = gq::build_tree(ctx->tree, ctx->ns, ctx->src_xy.data(), ctx->nc, ctx->ctr_xy.data(),
                           ctx->ctr_r.data(), tp);
  } catch (const std::bad_alloc &) {
    return fail(ctx, GQ_ENOMEM, "host allocation during tree build");
  }
  if (!msg.empty()) return fail(ctx, GQ_EINVAL, msg);
  gq::build_tables(ctx->tables, p.p_fmm, p.p_qbx);
  ctx->box_pq.assign(ctx->tree.n_boxes(), p.p_qbx);
  ctx->ctr_pq.clear();
  if (ctx->device >= 0) {
    GQ_HIP(ctx, hipSetDevice(ctx->device));
    gq_status st = upload_all(ctx);
    if (st != GQ_OK) {
      free_device(ctx);
      return st;
    }
  } else {
    GQ_TRY(build_near_work(ctx));
  }
  ctx->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ctx->m_c_sum = -1;
  ctx->built = true;
  return GQ_OK;
}

gq_status gq_eval(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1, int64_t ld1,
                  const double *dens2, int64_t ld2, double *out, int64_t ld_out) {
  return eval_common(ctx, kind, n_dens, dens1, ld1, dens2, ld2, out, ld_out, false);
}

gq_status gq_eval_direct(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1, int64_t ld1,
                         const double *dens2, int64_t ld2, double *out, int64_t ld_out) {
  return eval_common(ctx, kind, n_dens, dens1, ld1, dens2, ld2, out, ld_out, true);
}

gq_status gq_eval_noalloc(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1, int64_t ld1,
                          const double *dens2, int64_t ld2, double *out, int64_t ld_out) {
  GQ_TRY(check_eval_args(ctx, kind, n_dens, dens1, ld1, dens2, ld2, out, ld_out));
  if (n_dens == 0) return GQ_OK;
  if (ctx->profiling) return fail(ctx, GQ_ESTATE, "gq_eval_noalloc runs with stage profiling off");
  if (ctx->device >= kMaxDevices || !g_scratch_ptr[ctx->device])
    return fail(ctx, GQ_ESTATE, "no scratch address for this device");
  const int slots = workspace_batch(kind, n_dens);
  const size_t need = workspace_bytes(ctx, slots);
  if (need > kScratchBytes)
    return fail(ctx, GQ_EINVAL, "gq_eval_noalloc: this evaluation needs " + std::to_string(need) +
                                    " bytes of workspace, more than the " +
                                    std::to_string(kScratchBytes) + "-byte scratch");
  GQ_HIP(ctx, hipSetDevice(ctx->device));
  const gq::DevBuffers saved = ctx->d;
  carve_workspace(ctx, slots, static_cast<unsigned char *>(g_scratch_ptr[ctx->device]));
  const gq_status st = launch_batches(ctx, kind, n_dens, dens1, ld1, dens2, ld2, out, ld_out, false);
  ctx->d = saved;
  return st;
}

struct gq_graph {
  gq_ctx *ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t generation = 0;
};

gq_status gq_graph_create(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1, int64_t ld1,
                          const double *dens2, int64_t ld2, double *out, int64_t ld_out,
                          gq_graph **graph) {
  if (!graph) return fail(ctx, GQ_EINVAL, "null graph output");
  *graph = nullptr;
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  GQ_TRY(check_eval_args(ctx, kind, n_dens, dens1, ld1, dens2, ld2, out, ld_out));
  if (n_dens < 1) return fail(ctx, GQ_EINVAL, "a graph needs n_dens >= 1");
  if (n_dens > (kind == GQ_S_AND_D ? gq::kMaxDensBatch / 2 : gq::kMaxDensBatch))
    return fail(ctx, GQ_EUNSUP, "a graph captures one density batch (at most 128 densities, 64 "
                                "for GQ_S_AND_D)");
  if (ctx->profiling) return fail(ctx, GQ_ESTATE, "disable stage profiling before capturing a graph");
  GQ_HIP(ctx, hipSetDevice(ctx->device));
  // Everything the evaluation needs is allocated and created before the capture begins, so the
  // captured calls are launches, event records and stream waits only: the workspace, a stream to
  // capture on (the caller's may be the null stream, which cannot be captured) and fork/join
  // events reserved for captures (the eager evaluations keep their own).
  GQ_TRY(ensure_workspace(ctx, workspace_batch(kind, n_dens)));
  if (!ctx->capture) GQ_HIP(ctx, hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
  for (hipEvent_t *e : {&ctx->gev_fork, &ctx->gev_up, &ctx->gev_join})
    if (!*e) GQ_HIP(ctx, hipEventCreateWithFlags(e, hipEventDisableTiming));
  if (ctx->stream) GQ_HIP(ctx, hipStreamSynchronize(ctx->stream));
  GQ_HIP(ctx, hipStreamSynchronize(ctx->side));
  const hipStream_t saved = ctx->stream;
  const hipEvent_t ev[3] = {ctx->ev_fork, ctx->ev_up, ctx->ev_join};
  ctx->stream = ctx->capture;
  ctx->ev_fork = ctx->gev_fork;
  ctx->ev_up = ctx->gev_up;
  ctx->ev_join = ctx->gev_join;
  hipGraph_t g = nullptr;
  gq_status st = GQ_OK;
  hipError_t e = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    // one density batch: one gq::run_eval, whose only fork is the side stream (joined back
    // before the per-center stage)
    st = launch_batches(ctx, kind, n_dens, dens1, ld1, dens2, ld2, out, ld_out, false);
    // end the capture even after a failed launch, so the stream leaves capture mode
    const hipError_t e2 = hipStreamEndCapture(ctx->capture, &g);
    if (e2 != hipSuccess) e = e2;
  }
  ctx->stream = saved;
  ctx->ev_fork = ev[0];
  ctx->ev_up = ev[1];
  ctx->ev_join = ev[2];
  if (e != hipSuccess || st != GQ_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st != GQ_OK ? st : fail(ctx, GQ_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  gq_graph *h = new (std::nothrow) gq_graph();
  if (!h) {
    (void)hipGraphDestroy(g);
    return fail(ctx, GQ_ENOMEM, "graph handle");
  }
  h->ctx = ctx;
  h->graph = g;
  h->generation = ctx->generation;
  e = hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    delete h;
    return fail(ctx, GQ_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  *graph = h;
  return GQ_OK;
}

gq_status gq_graph_launch(gq_graph *graph) {
  if (!graph || !graph->ctx) return GQ_EINVAL;
  gq_ctx *ctx = graph->ctx;
  if (graph->generation != ctx->generation)
    return fail(ctx, GQ_ESTATE, "graph is stale: the context's buffers changed since capture");
  GQ_HIP(ctx, hipSetDevice(ctx->device));
  GQ_HIP(ctx, hipGraphLaunch(graph->exec, ctx->stream));
  return GQ_OK;
}

gq_status gq_graph_destroy(gq_graph *graph) {
  if (!graph) return GQ_OK;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  return GQ_OK;
}

// Modeled operation counts per GQ_OP_* stage (the per-list-entry cost model): every QBX center
// at its own order, the box sums weighted by the orders of the user centers a box owns.
static void model_ops(const gq_ctx *ctx, int64_t *ops) {
  const gq::Tree &t = ctx->tree;
  const int64_t pf = ctx->params.p_fmm, nb = t.n_boxes();
  auto ns = [&](int32_t d) { return t.n_src_subtree(d); };
  auto sum_src = [&](const gq::Csr &l, int64_t b) {
    int64_t n = 0;
    for (int64_t i = l.start[b]; i < l.start[b + 1]; ++i) n += ns(l.idx[i]);
    return n;
  };
  for (int k = 0; k < GQ_N_OPS; ++k) ops[k] = 0;
  ops[GQ_OP_MULTIPOLES] = pf * ctx->ns;
  for (int64_t b = 0; b < nb; ++b) {
    if (t.parent[b] >= 0 && ns((int32_t)b) > 0) ops[GQ_OP_M2M] += pf * pf;
    if (t.parent[b] >= 0 && t.has_tgt[b]) ops[GQ_OP_L2L] += pf * pf;
    ops[GQ_OP_LIST2] += pf * pf * t.list2.row_size(b);
    ops[GQ_OP_LIST4_FAR] += pf * sum_src(t.list4f, b);
    int64_t pq = 0;  // sum of the QBX orders of the user centers box b owns
    for (int64_t k = t.ctr_begin[b]; k < t.ctr_end[b]; ++k)
      if (t.ctr_order[k] < ctx->nc_user) pq += ctx->ctr_pq.empty() ? ctx->params.p_qbx : ctx->ctr_pq[k];
    if (pq == 0) continue;
    ops[GQ_OP_LIST1] += pq * sum_src(t.list1, b);
    ops[GQ_OP_LIST3_CLOSE] += pq * sum_src(t.list3c, b);
    ops[GQ_OP_LIST4_CLOSE] += pq * sum_src(t.list4c, b);
    ops[GQ_OP_LIST3_FAR] += pf * pq * t.list3f.row_size(b);
    ops[GQ_OP_L2QBXL] += pf * pq;
  }
}

gq_status gq_get_stats(gq_ctx *ctx, gq_stats *out) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (!out) return fail(ctx, GQ_EINVAL, "null output");
  if (!ctx->built) return fail(ctx, GQ_ESTATE, "no tree built");
  const gq::Tree &t = ctx->tree;
  std::memset(out, 0, sizeof(*out));
  out->n_src = ctx->ns; out->n_ctr = ctx->nc_user; out->n_tgt = ctx->nt;
  out->n_point_targets = ctx->n_pt;
  {
    std::vector<uint8_t> need(t.n_boxes(), 0);
    for (int32_t x : t.list2.idx) need[x] = 1;
    for (int32_t x : t.list3f.idx) need[x] = 1;
    for (int64_t b = 0; b < t.n_boxes(); ++b) {
      if (!need[b]) continue;
      const int64_t n = t.src_end[b] - t.src_begin[b];
      out->n_moment_boxes++;
      out->n_moment_pairs += n;
      if (n > kMomentChunk) out->n_moment_parts += (n + kMomentChunk - 1) / kMomentChunk;
    }
  }
  for (int64_t b = 0; b < t.n_boxes(); ++b) {
    if (t.ctr_end[b] <= t.ctr_begin[b]) continue;
    out->n_l2l_sinks++;
    for (int32_t a = t.parent[b]; a >= 0; a = t.parent[a])
      if (t.list2.row_size(a) > 0 || t.list4f.row_size(a) > 0) out->n_l2l_pairs++;
  }
  out->n_boxes = t.n_boxes(); out->n_levels = t.n_levels; out->n_leaves = t.n_leaves;
  out->n_target_boxes = t.n_target_boxes; out->n_suspended_centers = t.n_suspended;
  out->n_list1 = (int64_t)t.list1.idx.size(); out->n_list2 = (int64_t)t.list2.idx.size();
  out->n_list3_close = (int64_t)t.list3c.idx.size(); out->n_list3_far = (int64_t)t.list3f.idx.size();
  out->n_list4_close = (int64_t)t.list4c.idx.size(); out->n_list4_far = (int64_t)t.list4f.idx.size();
  out->near_pairs = t.near_pairs; out->list3_far_pairs = t.list3f_pairs;
  out->n_m2q_waves = ctx->n_m2q_waves;
  out->n_m2q_pairs = ctx->n_m2q_pairs;
  out->n_m2q_units = ctx->n_m2q_units;
  out->list4_far_sources = t.list4f_sources;
  out->near_sources = t.near_sources;
  out->n_local_boxes = t.n_local_boxes;
  for (int64_t b = 0; b < t.n_boxes(); ++b) {
    out->max_list2 = std::max(out->max_list2, t.list2.row_size(b));
    out->max_list4_close = std::max(out->max_list4_close, t.list4c.row_size(b));
    out->max_list4_far = std::max(out->max_list4_far, t.list4f.row_size(b));
  }
  out->max_list4 = t.max_list4;
  if (ctx->m_c_sum < 0)
    ctx->m_c_sum = gq::sources_near_centers(t, ctx->src_xy.data(), ctx->ctr_xy.data(),
                                            ctx->ctr_r.data(), ctx->nc_user, ctx->params.t_f);
  out->m_c_sum = ctx->m_c_sum;
  out->m_c = ctx->nc_user > 0 ? (double)ctx->m_c_sum / (double)ctx->nc_user : 0.0;
  out->root_lo[0] = t.lo[0]; out->root_lo[1] = t.lo[1]; out->root_side = t.side;
  out->build_ms = ctx->build_ms;
  model_ops(ctx, out->model_ops);
  for (int k = 0; k < GQ_N_OPS; ++k) out->model_ops_total += out->model_ops[k];
  return GQ_OK;
}

gq_status gq_get_tree_array(gq_ctx *ctx, int what, void *dst, int64_t *count) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (!count) return fail(ctx, GQ_EINVAL, "null count");
  if (!ctx->built) return fail(ctx, GQ_ESTATE, "no tree built");
  const gq::Tree &t = ctx->tree;
  const void *src = nullptr;
  size_t n = 0, esz = 0;
  std::vector<int64_t> tmp;
  auto pairs = [&](const std::vector<int64_t> &a, const std::vector<int64_t> &b) {
    tmp.resize(2 * a.size());
    for (size_t i = 0; i < a.size(); ++i) { tmp[2 * i] = a[i]; tmp[2 * i + 1] = b[i]; }
    src = tmp.data(); n = tmp.size(); esz = 8;
  };
  const gq::Csr *csr = nullptr;
  bool starts = false;
  switch (what) {
    case GQ_TREE_BOX_LEVEL: src = t.level.data(); n = t.level.size(); esz = 4; break;
    case GQ_TREE_BOX_PARENT: src = t.parent.data(); n = t.parent.size(); esz = 4; break;
    case GQ_TREE_BOX_CHILD: src = t.child.data(); n = t.child.size(); esz = 4; break;
    case GQ_TREE_BOX_IJ: pairs(t.bi, t.bj); break;
    case GQ_TREE_BOX_SRC_RANGE: pairs(t.src_begin, t.src_end); break;
    case GQ_TREE_BOX_CTR_RANGE: pairs(t.ctr_begin, t.ctr_end); break;
    case GQ_TREE_SRC_ORDER: src = t.src_order.data(); n = t.src_order.size(); esz = 8; break;
    case GQ_TREE_CTR_ORDER: src = t.ctr_order.data(); n = t.ctr_order.size(); esz = 8; break;
    case GQ_LIST1_START: starts = true; /* fallthrough */
    case GQ_LIST1: csr = &t.list1; break;
    case GQ_LIST2_START: starts = true; /* fallthrough */
    case GQ_LIST2: csr = &t.list2; break;
    case GQ_LIST3C_START: starts = true; /* fallthrough */
    case GQ_LIST3C: csr = &t.list3c; break;
    case GQ_LIST3F_START: starts = true; /* fallthrough */
    case GQ_LIST3F: csr = &t.list3f; break;
    case GQ_LIST4C_START: starts = true; /* fallthrough */
    case GQ_LIST4C: csr = &t.list4c; break;
    case GQ_LIST4F_START: starts = true; /* fallthrough */
    case GQ_LIST4F: csr = &t.list4f; break;
    default: return fail(ctx, GQ_EINVAL, "unknown tree array");
  }
  if (csr) {
    if (starts) { src = csr->start.data(); n = csr->start.size(); esz = 8; }
    else { src = csr->idx.data(); n = csr->idx.size(); esz = 4; }
  }
  *count = (int64_t)n;
  if (dst && n) std::memcpy(dst, src, n * esz);
  return GQ_OK;
}

gq_status gq_autotune(gq_ctx *ctx, int kind, const double *dens1, int64_t ld1, int reps,
                      double *best_ms) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (kind != GQ_S && kind != GQ_D) return fail(ctx, GQ_EINVAL, "autotune with GQ_S or GQ_D");
  if (reps < 1 || reps > 1000) return fail(ctx, GQ_EINVAL, "reps must be in 1..1000");
  GQ_TRY(check_eval_args(ctx, kind, 1, dens1, ld1, nullptr, 0, dens1, ctx->nt));
  GQ_HIP(ctx, hipSetDevice(ctx->device));
  double *out = nullptr;
  GQ_HIP(ctx, hipMalloc(&out, sizeof(double) * std::max<int64_t>(ctx->nt, 1)));
  hipEvent_t a = nullptr, b = nullptr;
  gq_status st = GQ_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    st = fail(ctx, GQ_EHIP, "hipEventCreate");
  struct Shape { int near_chunk, far_chunk, far_ppl; };
  const Shape cand[] = {{1024, 16, 1}, {512, 16, 1}, {2048, 16, 1}, {1024, 8, 1}, {1024, 16, 2},
                        {1024, 32, 1}, {4096, 16, 1}};
  const gq_params orig = ctx->params;
  double best = 1e300;
  Shape pick = {orig.near_chunk, orig.far_chunk, orig.far_pairs_per_lane};
  for (const Shape &c : cand) {
    if (st != GQ_OK) break;
    ctx->params.near_chunk = c.near_chunk;
    ctx->params.far_chunk = c.far_chunk;
    ctx->params.far_pairs_per_lane = c.far_ppl;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    st = build_near_work(ctx);
    if (st != GQ_OK) break;
    free_workspace(ctx);  // row counts may change with the shape
    st = eval_common(ctx, kind, 1, dens1, ld1, nullptr, 0, out, ctx->nt, false);  // warm-up
    if (st != GQ_OK) break;
    hipError_t e = hipEventRecord(a, ctx->stream);
    for (int r = 0; r < reps && e == hipSuccess && st == GQ_OK; ++r)
      st = eval_common(ctx, kind, 1, dens1, ld1, nullptr, 0, out, ctx->nt, false);
    if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) st = fail(ctx, GQ_EHIP, std::string("autotune timing: ") + hipGetErrorString(e));
    if (st == GQ_OK && ms / reps < best) {
      best = ms / reps;
      pick = c;
    }
  }
  // leave the context with the fastest shape (or the original one after an error)
  const gq_status st_run = st;
  ctx->params = orig;
  if (st_run == GQ_OK) {
    ctx->params.near_chunk = pick.near_chunk;
    ctx->params.far_chunk = pick.far_chunk;
    ctx->params.far_pairs_per_lane = pick.far_ppl;
  }
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  gq_status st2 = build_near_work(ctx);
  free_workspace(ctx);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(out);
  if (st_run != GQ_OK) return st_run;
  if (st2 != GQ_OK) return st2;
  if (best_ms) *best_ms = best;
  return GQ_OK;
}

gq_status gq_get_params(gq_ctx *ctx, gq_params *out) {
  if (!ctx || !out) return fail(ctx, GQ_EINVAL, "null argument");
  *out = ctx->params;
  return GQ_OK;
}

gq_status gq_set_qbx_orders(gq_ctx *ctx, int mem, const int32_t *orders) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (!ctx->built) return fail(ctx, GQ_ESTATE, "gq_set_qbx_orders before a successful gq_build");
  if (mem != GQ_MEM_HOST && mem != GQ_MEM_DEVICE) return fail(ctx, GQ_EINVAL, "bad mem");
  if (mem == GQ_MEM_DEVICE && ctx->device < 0) return fail(ctx, GQ_ESTATE, "device memory on a host-only context");
  gq::Tree &t = ctx->tree;
  const int64_t nc = ctx->nc, nb = t.n_boxes();
  std::vector<int32_t> ord(nc, ctx->params.p_qbx);
  if (orders) {
    if (mem == GQ_MEM_HOST) std::memcpy(ord.data(), orders, sizeof(int32_t) * ctx->nc_user);
    else GQ_HIP(ctx, hipMemcpy(ord.data(), orders, sizeof(int32_t) * ctx->nc_user, hipMemcpyDeviceToHost));
  }
  for (int64_t c = 0; c < ctx->nc_user; ++c)
    if (ord[c] < 0 || ord[c] > ctx->params.p_qbx) return fail(ctx, GQ_EINVAL, "order outside 0..p_qbx");
  // point targets need only the constant term: the lowest compiled order
  for (int64_t c = ctx->nc_user; c < nc; ++c) ord[c] = ctx->pq_values.front();
  // every center runs at the smallest compiled order at least its own; within each box the
  // centers are regrouped by that order (stable), so each order's centers of a box are one
  // contiguous group of tree positions
  auto eff = [&](int q) {
    for (int c : ctx->pq_values)
      if (c >= q) return c;
    return ctx->params.p_qbx;
  };
  std::vector<int32_t> cpq(nc), bp(nb, -1);
  std::vector<std::pair<int32_t, int64_t>> grp;
  for (int64_t b = 0; b < nb; ++b) {
    grp.clear();
    for (int64_t k = t.ctr_begin[b]; k < t.ctr_end[b]; ++k)
      grp.push_back({(int32_t)eff(ord[t.ctr_order[k]]), t.ctr_order[k]});
    std::stable_sort(grp.begin(), grp.end(),
                     [](const std::pair<int32_t, int64_t> &a, const std::pair<int32_t, int64_t> &b2) {
                       return a.first < b2.first;
                     });
    for (size_t i = 0; i < grp.size(); ++i) {
      const int64_t k = t.ctr_begin[b] + (int64_t)i;
      t.ctr_order[k] = grp[i].second;
      cpq[k] = grp[i].first;
      bp[b] = std::max(bp[b], grp[i].first);
    }
    if (bp[b] < 0) bp[b] = eff(0);
  }
  ctx->box_pq = bp;
  if (orders) ctx->ctr_pq = cpq;
  else ctx->ctr_pq.clear();
  if (ctx->device >= 0) {
    GQ_HIP(ctx, hipSetDevice(ctx->device));
    if (ctx->stream) GQ_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->side) GQ_HIP(ctx, hipStreamSynchronize(ctx->side));
    // the center arrays in the new tree order (same sizes, copied into the same buffers)
    CenterArrays ca;
    center_arrays(ctx, ca);
    auto &d = ctx->d;
    GQ_HIP(ctx, hipMemcpy(d.cxy, ca.xy.data(), sizeof(double) * ca.xy.size(), hipMemcpyHostToDevice));
    GQ_HIP(ctx, hipMemcpy(d.cr, ca.r.data(), sizeof(double) * ca.r.size(), hipMemcpyHostToDevice));
    GQ_HIP(ctx, hipMemcpy(d.cperm, ca.cperm.data(), sizeof(int32_t) * ca.cperm.size(), hipMemcpyHostToDevice));
    GQ_HIP(ctx, hipMemcpy(d.c2t_start, ca.start.data(), sizeof(int32_t) * ca.start.size(), hipMemcpyHostToDevice));
    if (!ca.slot.empty())
      GQ_HIP(ctx, hipMemcpy(d.c2t_slot, ca.slot.data(), sizeof(int32_t) * ca.slot.size(), hipMemcpyHostToDevice));
  }
  return build_near_work(ctx);
}

gq_status gq_get_center_orders(gq_ctx *ctx, int32_t *dst) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (!ctx->built) return fail(ctx, GQ_ESTATE, "no tree built");
  if (!dst) return fail(ctx, GQ_EINVAL, "null output");
  const gq::Tree &t = ctx->tree;
  for (int64_t k = 0; k < ctx->nc; ++k) {
    const int64_t c = t.ctr_order[k];
    if (c < ctx->nc_user) dst[c] = ctx->ctr_pq.empty() ? ctx->params.p_qbx : ctx->ctr_pq[k];
  }
  return GQ_OK;
}

gq_status gq_get_box_orders(gq_ctx *ctx, int32_t *dst, int64_t *count) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (!ctx->built || !count) return fail(ctx, GQ_ESTATE, "no tree built or null count");
  *count = (int64_t)ctx->box_pq.size();
  if (dst) std::memcpy(dst, ctx->box_pq.data(), sizeof(int32_t) * ctx->box_pq.size());
  return GQ_OK;
}

gq_status gq_set_profiling(gq_ctx *ctx, int enable) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (ctx->device < 0) return fail(ctx, GQ_ESTATE, "host-only context");
  ctx->profiling = enable != 0;
  return GQ_OK;
}

gq_status gq_get_stage_times(gq_ctx *ctx, double *ms, int64_t *count) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (!ms || !count) return fail(ctx, GQ_EINVAL, "null output");
  if (ctx->device < 0) return fail(ctx, GQ_ESTATE, "host-only context");
  GQ_HIP(ctx, hipSetDevice(ctx->device));
  GQ_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < 3 * GQ_N_STAGES; ++i) { ms[i] = 0.0; count[i] = 0; }
  gq_status st = GQ_OK;
  for (auto &r : ctx->prof) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      ms[r.slot] += t;
      count[r.slot] += 1;
    } else {
      st = fail(ctx, GQ_EHIP, "hipEventElapsedTime failed");
    }
    ctx->event_pool.push_back(r.a);
    ctx->event_pool.push_back(r.b);
  }
  ctx->prof.clear();
  return st;
}

gq_status gq_device_math(gq_ctx *ctx, int fn, int64_t n, const double *x, double *out) {
  if (!ctx) return fail(nullptr, GQ_EINVAL, "null context");
  if (ctx->device < 0) return fail(ctx, GQ_ESTATE, "host-only context");
  if (fn != GQ_MATH_LOG && fn != GQ_MATH_RCP) return fail(ctx, GQ_EINVAL, "unknown function");
  if (n < 0 || n > (int64_t(1) << 38)) return fail(ctx, GQ_EINVAL, "n out of range");
  if (n == 0) return GQ_OK;
  if (!x || !out) return fail(ctx, GQ_EINVAL, "null array");
  GQ_HIP(ctx, hipSetDevice(ctx->device));
  GQ_HIP(ctx, gq::run_math(fn, n, x, out, ctx->stream));
  return GQ_OK;
}

const char *gq_last_error(gq_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
