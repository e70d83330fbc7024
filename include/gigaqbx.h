/*
 * gigaqbx.h -- C ABI of the MI355X (gfx950) QBX-coupled FMM for 2-D Laplace layer potentials.
 *
 * Method: Wala & Kloeckner, "A Fast Algorithm with Error Bounds for Quadrature by Expansion".
 * The library evaluates the QBX approximation (Sec. 2.1, eq. (qbx)) of the single-layer potential
 * (Sec. 1, eq. (slp-definition)) and double-layer potential (eq. (dlp-definition)) at targets that
 * are associated with QBX expansion centers, accelerated by the GIGAQBX FMM (Sec. 4, Algorithm
 * Stages 1-8) on a quadtree with target confinement regions and the modified interaction lists
 * (Sec. 4.3, Definitions 1-9).
 *
 * General conventions
 *   - Every call returns a gq_status; nothing is thrown across the ABI. On failure the context
 *     keeps a message retrievable with gq_last_error().
 *   - Points and vectors are (n, 2) row-major interleaved (x, y) FP64 arrays. Complex values are
 *     (re, im) FP64 pairs.
 *   - The caller owns every input and output pointer; the library owns its internal workspace
 *     (device memory it allocates at gq_build and frees at gq_destroy).
 *   - Potentials include the -1/(2 pi) factor of eqs. (slp-definition)/(dlp-definition).
 *   - A context is bound to one device and one HIP stream; calls on one context must not overlap.
 *     Device work is enqueued on the context's stream and is asynchronous unless stated.
 *   - A context created with device = -1 is host-only: it builds the tree and lists (Stage 1 and
 *     Sec. 4.3) and exposes them for inspection, but cannot evaluate.
 */
#ifndef GIGAQBX_H
#define GIGAQBX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gq_ctx gq_ctx;

typedef enum {
  GQ_OK = 0,
  GQ_EINVAL = -1,  /* invalid argument (null pointer, bad size, non-finite coordinate, ...)   */
  GQ_ENOMEM = -2,  /* host or device allocation failed                                        */
  GQ_EHIP = -3,    /* a HIP runtime call failed (message names it)                            */
  GQ_ESTATE = -4,  /* call out of order (evaluate before build, host-only context, ...)       */
  GQ_EUNSUP = -5   /* valid request this build does not support (order too high, ...)         */
} gq_status;

/* Layer-potential kinds. GQ_S_MINUS_D evaluates S(dens1) - D(dens2), the left side of Green's
 * formula used as the accuracy test in Sec. 5.1. GQ_S_AND_D evaluates both S(dens1) and
 * D(dens1) (two output rows per density). GQ_SP evaluates S'(dens1) = n(x) . grad_x S(dens1)(x),
 * the normal derivative of the single layer potential at the targets (the operator of the
 * exterior Neumann integral equation of Sec. 1, eq. (ext-neumann-ie)), with the target normals
 * of gq_set_target_normals: the same expansions as GQ_S, differentiated where they are evaluated;
 * a target with two centers takes the average of the two one-sided limits (the principal value). */
enum { GQ_S = 1, GQ_D = 2, GQ_S_MINUS_D = 3, GQ_S_AND_D = 4, GQ_SP = 5 };

/* Where the geometry arrays passed to gq_set_geometry live. */
enum { GQ_MEM_HOST = 0, GQ_MEM_DEVICE = 1 };

/* Arithmetic of the box expansions. GQ_MIXED_FP32 stores box multipoles and locals in FP32; every
 * coefficient is scaled by a power of two per tree level (the box side), so the scaling itself is
 * exact. M2L and the downward pass (L2L as the Stage 7 gather) run on the FP32 matrix cores. For
 * density batches (8 or more expansion slots) the moments (P2M; M2M is not launched, the moments
 * are the multipoles it would build) and P2L run on the FP32 matrix cores too, with FP32 products
 * per batch of sources summed in FP64; one density forms them in FP64 and rounds them to FP32.
 * The source-to-center (P2QBXL), multipole-to-center (M2QBXL) and local-to-center (L2QBXL) steps,
 * the pair powers and the evaluation at the targets stay in FP64. Intended for tolerances around
 * 1e-6. */
enum { GQ_FP64 = 0, GQ_MIXED_FP32 = 1 };

typedef struct {
  int p_qbx;              /* QBX expansion order (Sec. 4.1), 0..GQ_MAX_P_QBX                   */
  int p_fmm;              /* FMM expansion order (Sec. 4.1), 1..GQ_MAX_P_FMM                   */
  int n_max;              /* subdivide a box owning more than n_max eligible particles (Stage 1) */
  int count_mode;         /* 0: sources + eligible centers count towards n_max (Sec. 4.3);
                             1: sources only                                                    */
  double t_f;             /* target confinement factor, 0 <= t_f < 1 (Sec. 4.3.1); 0.9 typical  */
  int w3far_min_sources;  /* Remark 1: a List-3-far box with fewer sources is evaluated directly
                             through its leaves; 0 disables                                     */
  int precision;          /* GQ_FP64 or GQ_MIXED_FP32                                           */
  int max_levels;         /* depth guard for coincident particles (not in the paper); <= 28     */
  int overlap;            /* 1: direct and List 3 far work on a second stream, overlapping the
                             tree passes; 0: everything on the caller's stream                  */
  int near_chunk;         /* direct sources per work item (one wavefront), 0: 1024             */
  int far_chunk;          /* List 3 far boxes per work item (1..32), 0: 16                      */
  int far_pairs_per_lane; /* 1 (default): one (center, List 3 far box) pair per lane, pairs of
                             whole (center, far chunk) units packed across boxes; 2..64: items
                             of one box's centers with at most that many pairs per lane;
                             0: such items shaped by a cost model                              */
  int near_dens_group;    /* densities per direct-interaction work item when an evaluation has
                             several (1, 2 or 4): the pair geometry is formed once per group;
                             0: 2                                                              */
  double eps;             /* requested accuracy (Sec. 4.1 input (b)); used when p_fmm <= 0:
                             the FMM error is of order (1/2)^(p_fmm + 1) (Theorem 1), so
                             p_fmm = ceil(|log2 eps|), at most GQ_MAX_P_FMM. 0: unused       */
  int tcr_shape;          /* target confinement region: 0 (default) the closed square of
                             radius |b|(1 + t_f) (Sec. 4.3, Definition 1); 1 the closed disk of
                             that radius, the shape the paper's corrigendum reports its first
                             experiments used; the separation relations of Definition 1 then
                             take the l-inf distance to the disk                              */
  int level_restrict;     /* 1: refine the tree until adjacent leaves differ by at most one
                             level (Remark 2, level-restricted quadtree); 0 (default): as built */
} gq_params;

#define GQ_MAX_P_QBX 20
#define GQ_MAX_P_FMM 63

/* Fill *p with the defaults: p_qbx 12, p_fmm 30, n_max 64, count_mode 0, t_f 0.9,
 * w3far_min_sources 15, GQ_FP64, max_levels 24, overlap 1, work-item shapes 0 (defaults),
 * eps 0, tcr_shape 0, level_restrict 0. */
gq_status gq_default_params(gq_params *p);

/* Create a context on HIP device `device` (>= 0) using `hip_stream` (a hipStream_t, may be NULL for
 * the default stream; borrowed, not owned), or a host-only context with device = -1. */
gq_status gq_create(gq_ctx **out, int device, void *hip_stream);

/* Release the context and all device workspace. Synchronises the context's stream first. */
gq_status gq_destroy(gq_ctx *ctx);

/* Replace the stream later calls enqueue on (borrowed). */
gq_status gq_set_stream(gq_ctx *ctx, void *hip_stream);

/*
 * Geometry (Sec. 4.2 inputs (a) and (d), Sec. 2.2.2 center placement), copied into the context:
 *   src_xy  (n_src, 2)  quadrature nodes y_i
 *   src_nrm (n_src, 2)  unit normals n_i (outward for the sign conventions of eq. (dlp))
 *   src_w   (n_src)     quadrature weights including the arclength element
 *   ctr_xy  (n_ctr, 2)  QBX expansion centers, ctr_r (n_ctr) their radii (> 0); n_ctr may be
 *                       0 when every target is a conventional one
 *   tgt_xy  (n_tgt, 2)  targets; tgt_ctr (n_tgt, 2) int32 indices of the one or two centers
 *                       whose expansions are averaged for the target; -1 marks an unused slot.
 *                       A target with both slots -1 is a conventional (off-surface) target:
 *                       it gets the plain point value of the layer potential (direct sum over
 *                       its near sources, multipole-to-point over List 3 far, its box's local
 *                       expansion: Stages 3a, 5b and 8a) through an internal center at the
 *                       target with radius 2^-40 of the particles' extent, appended after the
 *                       caller's centers (indices >= n_ctr in the tree arrays). Such a target
 *                       must not coincide with a source node.
 * mem says whether all pointers are host (GQ_MEM_HOST) or device (GQ_MEM_DEVICE) memory on the
 * context's device. The call returns after the copy; the arrays may be freed afterwards. It
 * invalidates any previous build. Non-finite coordinates or radii give GQ_EINVAL.
 */
gq_status gq_set_geometry(gq_ctx *ctx, int mem, int64_t n_src, const double *src_xy,
                          const double *src_nrm, const double *src_w, int64_t n_ctr,
                          const double *ctr_xy, const double *ctr_r, int64_t n_tgt,
                          const double *tgt_xy, const int32_t *tgt_ctr);

/*
 * Several independent geometries in one context (a ragged batch): every stage then runs once
 * over the work of all geometries, with no interaction between them. The arrays are the
 * geometries' arrays concatenated; src_off, ctr_off, tgt_off (host, n_geom + 1 each, starting at
 * 0 and ending at n_src, n_ctr, n_tgt) give each geometry's first source, center and target, and
 * every geometry needs at least one source. tgt_ctr holds center indices local to the target's
 * geometry (-1 unused; both -1: conventional target of that geometry). gq_build builds one tree
 * per geometry (host threads) and merges them into one forest; densities and outputs of gq_eval
 * are concatenated in the same order. Tree arrays then describe the forest: boxes are numbered
 * depth-major over all trees and GQ_TREE_BOX_LEVEL holds a per-(tree, depth) level index;
 * gq_stats' root fields describe the first geometry's root. Other arguments as gq_set_geometry.
 */
gq_status gq_set_geometry_batch(gq_ctx *ctx, int mem, int64_t n_geom, const int64_t *src_off,
                                const int64_t *ctr_off, const int64_t *tgt_off, int64_t n_src,
                                const double *src_xy, const double *src_nrm, const double *src_w,
                                int64_t n_ctr, const double *ctr_xy, const double *ctr_r,
                                int64_t n_tgt, const double *tgt_xy, const int32_t *tgt_ctr);

/*
 * Target-to-center association for targets anywhere in the plane (Sec. 2.2.2: identify the
 * targets too close to the curve for plain quadrature and find a QBX center for each). Host
 * arrays, no context. For each of the n_tgt targets, with rho = min over centers of
 * |x - c| / r_c (ties to the lowest center index):
 *   rho <= 1 + slack:           QBX target of that center: tgt_ctr[t] = (c, -1) (one-sided value
 *                               at the center's side of the curve); slack 0.2 is the 20 % the
 *                               paper reports as harmless, 0 admits only targets in a disk;
 *   1 + slack < rho < far_factor: in a coverage gap next to the curve (the paper refines the
 *                               geometry there): tgt_ctr[t] = (-1, -1) like a far target, and
 *                               counted in *n_gap (may be NULL) so the caller can refine;
 *   rho >= far_factor:          conventional target: tgt_ctr[t] = (-1, -1).
 * The output feeds gq_set_geometry's tgt_ctr (centers in the same order). Needs slack >= 0 and a
 * finite far_factor >= 1 + slack, finite coordinates and positive radii (else GQ_EINVAL; message
 * from gq_associate_last_error()). Runs on host threads; the query is an area query on a grid
 * whose cells hold the centers whose disks of radius far_factor r_c they overlap.
 */
gq_status gq_associate_targets(int64_t n_ctr, const double *ctr_xy, const double *ctr_r,
                               int64_t n_tgt, const double *tgt_xy, double slack,
                               double far_factor, int32_t *tgt_ctr, int64_t *n_gap);
const char *gq_associate_last_error(void);

/*
 * Stage 1 and Sec. 4.3: build the quadtree (root square covering every particle and every whole
 * QBX disk; a center stays in a box when its disk does not fit the child's target confinement
 * region), sort particles into tree order, build Lists 1, 2, 3-close/far, 4-close/far, and upload
 * tree, lists and translation tables to the device. Synchronous. Invalid parameters give
 * GQ_EINVAL, orders above the compiled maxima GQ_EUNSUP. With p_fmm <= 0 the FMM order is
 * derived from params->eps (0 < eps < 1, else GQ_EINVAL) as described at gq_params.eps;
 * gq_get_params then shows the order used.
 */
gq_status gq_build(gq_ctx *ctx, const gq_params *params);

/*
 * The box expansions of the last evaluation, for operator-level tests: what = GQ_EXP_MULTIPOLE
 * (every box's multipole, Stage 2), GQ_EXP_LOCAL (every target-or-ancestor box's own local: List 2
 * by M2L plus List 4 far by P2L, Stages 4 and 6b) or GQ_EXP_LOCAL_COMPLETE (the complete local of
 * every box owning centers after the downward pass, Stage 7; other boxes' rows are not written).
 * Layout: n_boxes x (p_fmm + 1) complex values, (re, im) interleaved, boxes in the order of the
 * tree arrays, coefficients scaled by the box side s: a_k / s^k (multipoles, the expansion
 * a_0 log(z - c) + sum_k a_k (z - c)^-k) and b_k s^k (locals, sum_k b_k (z - c)^k). slot selects
 * the density slot of the evaluation (0 for one density; GQ_S_AND_D of n densities uses slots
 * 0..n-1 for S and n..2n-1 for D). *count receives the number of complex values; dst NULL asks
 * for the count only; else dst (host) receives them, after the context's streams have finished.
 * Errors: GQ_ESTATE before a build or an evaluation that filled the slot; GQ_EUNSUP for
 * GQ_MIXED_FP32 contexts (FP32 storage); GQ_EINVAL for an unknown what or a null count.
 */
enum { GQ_EXP_MULTIPOLE = 1, GQ_EXP_LOCAL = 2, GQ_EXP_LOCAL_COMPLETE = 3 };
gq_status gq_get_expansions(gq_ctx *ctx, int what, int64_t slot, double *dst, int64_t *count);

/*
 * Unit normals n(x) of the n_tgt targets for GQ_SP: (n_tgt x 2), (x, y) interleaved, in the
 * caller's target order, host or device memory as mem says; the library copies them. n_tgt must
 * be the geometry's target count (else GQ_EINVAL; non-finite values: GQ_EINVAL). A later call
 * replaces them; gq_set_geometry drops them. Before gq_set_geometry: GQ_ESTATE.
 */
gq_status gq_set_target_normals(gq_ctx *ctx, int mem, int64_t n_tgt, const double *tgt_nrm);

/*
 * Evaluate, by the GIGAQBX FMM (Algorithm Stages 2-8 plus evaluation of the QBX expansions at
 * the targets), n_dens independent potentials:
 *   kind GQ_S:          out[j] = S dens1[j]
 *   kind GQ_D:          out[j] = D dens1[j]
 *   kind GQ_S_MINUS_D:  out[j] = S dens1[j] - D dens2[j]
 *   kind GQ_S_AND_D:    out[j] = S dens1[j] and out[n_dens + j] = D dens1[j]; one expansion
 *                       pipeline over two workspace halves (S, D): the stages that only move
 *                       expansions run once for both kinds, and the direct interactions of both
 *                       kinds share their pair geometry. When every center serves at most one
 *                       target, the direct and List 3 far (M2QBXL) parts of each center's
 *                       expansion (and, for 8 or more densities, its box local, L2QBXL) are
 *                       summed at that target instead of formed as coefficients (GQ_S and GQ_D
 *                       of one density likewise): the same truncated series in another
 *                       order, so S and D agree with GQ_S and GQ_D to rounding (about 1e-14),
 *                       not bitwise. The direct-QBX path (gq_eval_direct) runs the two kinds on
 *                       two library streams forked from and joined back to the context's stream
 *   kind GQ_SP:         out[j] = S' dens1[j] (needs gq_set_target_normals, else GQ_ESTATE)
 * dens1/dens2 are device arrays (n_dens, n_src) with row stride ld1/ld2 (>= n_src) in the
 * caller's source order; out is a device array (n_dens, n_tgt) (GQ_S_AND_D: 2 n_dens rows)
 * with row stride ld_out in the caller's target order. dens2 must be NULL unless kind is
 * GQ_S_MINUS_D. Enqueued on the
 * context's stream; inputs must stay valid and outputs untouched until the stream passes the
 * call. Requires a successful gq_build on a device context (else GQ_ESTATE).
 */
gq_status gq_eval(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1, int64_t ld1,
                  const double *dens2, int64_t ld2, double *out, int64_t ld_out);

/*
 * Same contract as gq_eval, computed by unaccelerated QBX on the GPU: every center's expansion
 * (eq. (qbx)) is formed from all sources directly, without tree or lists (needs only
 * gq_set_geometry and gq_build for the orders). Each center uses the same order as in gq_eval
 * (gq_get_center_orders). O(n_ctr n_src) work; for checking and small
 * problems.
 */
gq_status gq_eval_direct(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1,
                         int64_t ld1, const double *dens2, int64_t ld2, double *out,
                         int64_t ld_out);

/*
 * gq_eval without any device allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Same contract and results as
 * gq_eval (the same kernels in the same order; bitwise equal outputs), but the per-density
 * workspace (strengths, box expansions, center rows, target slots) lives in a fixed scratch
 * array of 256 MiB in device memory that the library holds on each device it runs on until the
 * process ends (its address is taken when the first context is created on that device). An
 * evaluation whose workspace for one density batch exceeds it (about 105 MB per density and kind
 * for 131072 sources at p_fmm 30, p_qbx 12) gives GQ_EINVAL and launches nothing; stage profiling
 * must be off (GQ_ESTATE). The call allocates no device or host memory. Every call on a device
 * shares that device's scratch, so calls that can overlap on one device (on different streams or
 * from different threads, from any context) race and must be ordered by the caller; the scratch
 * keeps the last call's contents, none of which a later call reads.
 */
gq_status gq_eval_noalloc(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1,
                          int64_t ld1, const double *dens2, int64_t ld2, double *out,
                          int64_t ld_out);

/*
 * Per-center QBX orders (the truncation order p of eq. (qbx) may differ between centers; Sec. 4.1
 * chooses it from the truncation error, which depends on the local geometry). orders[c] (n_ctr
 * int32, caller order, host or device memory per mem; NULL restores the uniform p_qbx) must lie in
 * 0..p_qbx of the last gq_build. Every center then runs at the smallest compiled order that is at
 * least its own (gq_get_center_orders): the centers inside each box are regrouped by that order
 * (GQ_TREE_CTR_ORDER changes accordingly) and the direct, List 3 far and per-center work of each
 * group runs at the group's order. Results per center do not depend on the regrouping.
 * Synchronous. Call after gq_build; a new gq_build resets to the uniform order.
 */
gq_status gq_set_qbx_orders(gq_ctx *ctx, int mem, const int32_t *orders);

/* The compiled QBX order each center runs at (n_ctr int32, caller order, host memory `dst`). */
gq_status gq_get_center_orders(gq_ctx *ctx, int32_t *dst);

/* Tune the work-item shapes (gq_params near_chunk, far_chunk, far_pairs_per_lane) for this
 * built context: each of a fixed set of candidate shapes is timed over `reps` evaluations of
 * kind GQ_S or GQ_D of dens1 (device, n_src, row stride ld1) with HIP events on the context's
 * stream, and the context keeps the fastest (gq_get_params shows it; *best_ms, may be NULL,
 * receives its time per evaluation). Synchronous; allocates a temporary output of n_tgt doubles
 * and releases the evaluation workspace (the next gq_eval sizes it again). Results may differ
 * from other shapes by summation order only. On an error the original shape is restored. */
gq_status gq_autotune(gq_ctx *ctx, int kind, const double *dens1, int64_t ld1, int reps,
                      double *best_ms);

/* The parameters of the last gq_build (after gq_autotune: with the chosen shapes). */
gq_status gq_get_params(gq_ctx *ctx, gq_params *out);

/* Copy the largest QBX order run in each box (n_boxes int32, breadth-first box order; the
 * smallest compiled order for a box without centers) to host memory `dst` (NULL to query the
 * count, always written to *count). */
gq_status gq_get_box_orders(gq_ctx *ctx, int32_t *dst, int64_t *count);

/*
 * HIP graph of one evaluation (the build-once / evaluate-many split of Sec. 4.6: the tree and lists
 * are fixed, so the launches of an evaluation can be recorded once and replayed).
 * gq_graph_create records gq_eval(ctx, kind, n_dens, dens1, ld1, dens2, ld2, out, ld_out) (the
 * FMM path, any kind) into a graph without running it; gq_graph_launch replays it on the
 * context's current stream, reading the densities at the recorded addresses and writing the
 * recorded output. One density batch per graph: n_dens in 1..128 (1..64 for GQ_S_AND_D), else
 * GQ_EUNSUP. Synchronous creation (it first sizes the workspace, then synchronises the
 * context's streams); profiling must be off (GQ_ESTATE). The graph refers to the context's
 * workspace: a later gq_eval with more densities, gq_build, gq_set_qbx_orders or gq_autotune
 * replaces it, after which gq_graph_launch returns GQ_ESTATE. Replays and eager evaluations on
 * one context share the workspace and must not overlap on the device (enqueue them on one
 * stream). gq_graph_destroy accepts NULL.
 */
typedef struct gq_graph gq_graph;
gq_status gq_graph_create(gq_ctx *ctx, int kind, int64_t n_dens, const double *dens1,
                          int64_t ld1, const double *dens2, int64_t ld2, double *out,
                          int64_t ld_out, gq_graph **graph);
gq_status gq_graph_launch(gq_graph *graph);
gq_status gq_graph_destroy(gq_graph *graph);

/*
 * Modeled operation counts (Sec. 4.6 and the per-list-entry cost model of Sec. 5): an expansion
 * of order p costs p to form from one source or to evaluate, a translation between orders p and
 * p' costs p p'. With n_s the sources of a source box, n_t the QBX centers owned by a target box
 * (each at its own QBX order p_c, so n_t p_QBX reads as the sum of p_c over them) and N_S the
 * sources, one evaluation of one density is modeled as
 *   GQ_OP_MULTIPOLES  N_S p_FMM                      (Stage 2, forming leaf multipoles)
 *   GQ_OP_M2M         p_FMM^2 per upward shift       (Stage 2: boxes with sources and a parent)
 *   GQ_OP_LIST1       p_QBX n_s n_t per List 1 entry (Stage 3)
 *   GQ_OP_LIST2       p_FMM^2 per List 2 entry       (Stage 4)
 *   GQ_OP_LIST3_CLOSE p_QBX n_s n_t per entry        (Stage 5a)
 *   GQ_OP_LIST3_FAR   p_FMM p_QBX n_t per entry      (Stage 5b)
 *   GQ_OP_LIST4_CLOSE p_QBX n_s n_t per entry        (Stage 6a)
 *   GQ_OP_LIST4_FAR   p_FMM n_s per entry            (Stage 6b)
 *   GQ_OP_L2L         p_FMM^2 per downward shift     (Stage 7: boxes with a local and a parent)
 *   GQ_OP_L2QBXL      p_FMM p_QBX per QBX center     (Stage 8)
 * Conventional (non-QBX) targets and their internal centers are not in the model. The counts
 * describe the method, not the kernels (which form multipoles from whole subtrees, for one).
 */
enum {
  GQ_OP_MULTIPOLES = 0, GQ_OP_M2M, GQ_OP_LIST1, GQ_OP_LIST2, GQ_OP_LIST3_CLOSE, GQ_OP_LIST3_FAR,
  GQ_OP_LIST4_CLOSE, GQ_OP_LIST4_FAR, GQ_OP_L2L, GQ_OP_L2QBXL, GQ_N_OPS
};

/* Sizes of the tree and lists after gq_build (Sec. 4.3, and the stage costs of Table 2). */
typedef struct {
  int64_t n_src, n_ctr, n_tgt;
  int64_t n_boxes, n_levels, n_leaves, n_target_boxes;
  int64_t n_suspended_centers;   /* centers owned by non-leaf boxes                      */
  int64_t n_list1, n_list2, n_list3_close, n_list3_far, n_list4_close, n_list4_far;
  int64_t near_pairs;            /* (center, source) pairs evaluated directly             */
  int64_t list3_far_pairs;       /* (center, box) multipole-to-QBX-local pairs            */
  int64_t list4_far_sources;     /* (box, source) pairs formed into box locals            */
  int64_t near_sources;          /* sum over boxes owning centers of their direct sources  */
  int64_t n_local_boxes;         /* target-or-ancestor boxes (boxes with a local expansion) */
  int64_t max_list2, max_list4, max_list4_close, max_list4_far;  /* largest row of List 2, of
                                    List 4 itself (Definition 7, before the close/far split),
                                    of List 4 close and of List 4 far (Sec. 4.6 bounds them by
                                    75, 21, 42 and 63)                                          */
  double root_lo[2];
  double root_side;
  double build_ms;               /* host time of the last gq_build                        */
  int64_t n_point_targets;       /* conventional targets (each with an internal center)   */
  int64_t n_l2l_sinks;           /* boxes owning centers (they receive complete locals)   */
  int64_t n_l2l_pairs;           /* (box, ancestor with its own local) shifts in Stage 7   */
  int64_t n_moment_boxes;        /* boxes whose multipole M2L or M2QBXL reads (Stage 2)   */
  int64_t n_moment_pairs;        /* (box, subtree source) pairs of their moments          */
  int64_t n_moment_parts;        /* partial moments of boxes split over several items     */
  int64_t n_m2q_waves;           /* Stage 5b wavefronts of (center, List 3 far box) pairs
                                    packed across boxes (far_pairs_per_lane 1; else 0)   */
  int64_t n_m2q_pairs;           /* their pairs (list3_far_pairs when packed)             */
  int64_t n_m2q_units;           /* their rows: (center, chunk of its List 3 far boxes)   */
  double m_c;                    /* M_C of Sec. 4.6.1: the mean over centers c of the number of
                                    sources in the closed square of radius 8 r_c / t_f about c
                                    (every source when t_f = 0); computed on the first
                                    gq_get_stats after a build                                */
  int64_t m_c_sum;               /* the sum behind m_c (N_C m_c)                            */
  int64_t model_ops[GQ_N_OPS];   /* modeled operation counts per GQ_OP_* stage (above), for the
                                    current QBX orders; computed on each gq_get_stats        */
  int64_t model_ops_total;       /* their sum                                               */
} gq_stats;

gq_status gq_get_stats(gq_ctx *ctx, gq_stats *out);

/*
 * Copy one tree or list array to host memory `dst` (may be NULL to query the element count,
 * which is always written to *count). Element types:
 *   GQ_TREE_BOX_LEVEL, GQ_TREE_BOX_PARENT       int32  (n_boxes)      parent -1 for the root
 *   GQ_TREE_BOX_CHILD                           int32  (n_boxes, 4)   quadrant x + 2 y, -1 none
 *   GQ_TREE_BOX_IJ                              int64  (n_boxes, 2)   integer coordinates at level
 *   GQ_TREE_BOX_SRC_RANGE, GQ_TREE_BOX_CTR_RANGE int64 (n_boxes, 2)   [begin, end) in tree order;
 *                                               sources: whole subtree; centers: owned ones
 *   GQ_TREE_SRC_ORDER, GQ_TREE_CTR_ORDER        int64  (n_src | n_ctr) caller index at each
 *                                               tree-order position
 *   GQ_LIST*_START                              int64  (n_boxes + 1)  CSR row starts
 *   GQ_LIST*                                    int32  (entries)      box indices
 */
enum {
  GQ_TREE_BOX_LEVEL = 1, GQ_TREE_BOX_PARENT, GQ_TREE_BOX_CHILD, GQ_TREE_BOX_IJ,
  GQ_TREE_BOX_SRC_RANGE, GQ_TREE_BOX_CTR_RANGE, GQ_TREE_SRC_ORDER, GQ_TREE_CTR_ORDER,
  GQ_LIST1_START, GQ_LIST1, GQ_LIST2_START, GQ_LIST2, GQ_LIST3C_START, GQ_LIST3C,
  GQ_LIST3F_START, GQ_LIST3F, GQ_LIST4C_START, GQ_LIST4C, GQ_LIST4F_START, GQ_LIST4F
};
gq_status gq_get_tree_array(gq_ctx *ctx, int what, void *dst, int64_t *count);

/*
 * Per-stage device timing for profiling. When enabled, every evaluation records a HIP event pair
 * on the context's stream around each stage; gq_get_stage_times synchronises the stream, adds
 * the elapsed times since the last query into ms[(kind - 1) * GQ_N_STAGES + stage] (caller
 * arrays of 3 * GQ_N_STAGES doubles / int64 counts), and clears the records. GQ_S_AND_D
 * evaluations record under GQ_S (each stage interval covers both kinds). Disabled by default.
 */
enum {
  GQ_STAGE_GATHER = 0,   /* densities -> per-source strengths in tree order                */
  GQ_STAGE_P2M,          /* Stage 2a                                                        */
  GQ_STAGE_M2M,          /* Stage 2b (all levels)                                           */
  GQ_STAGE_M2L_P2L,      /* Stages 4 and 6b: box locals from List 2 and List 4 far          */
  GQ_STAGE_L2L,          /* Stage 7 (all levels)                                            */
  GQ_STAGE_NEAR,         /* Stages 3, 5a, 6a: direct sources -> QBX centers (P2QBXL)        */
  GQ_STAGE_M2QBXL,       /* Stage 5b: List 3 far multipoles -> QBX centers                  */
  GQ_STAGE_QBX_CENTER,   /* Stage 8 per center (L2QBXL) and evaluation at the targets      */
  GQ_STAGE_FINALIZE,     /* average of the one or two center values per target              */
  GQ_STAGE_DIRECT,       /* unaccelerated QBX (gq_eval_direct)                              */
  GQ_N_STAGES
};
gq_status gq_set_profiling(gq_ctx *ctx, int enable);
gq_status gq_get_stage_times(gq_ctx *ctx, double *ms, int64_t *count);

/*
 * Diagnostics: the device natural logarithm (GQ_MATH_LOG; x > 0 normal) and reciprocal
 * (GQ_MATH_RCP; x finite, non-zero) that the direct-interaction (P2QBXL), P2L and M2QBXL kernels
 * use, applied elementwise to n device doubles x, written to n device doubles out, enqueued on
 * the context's stream. For testing their accuracy; other inputs give unspecified values.
 */
enum { GQ_MATH_LOG = 1, GQ_MATH_RCP = 2 };
gq_status gq_device_math(gq_ctx *ctx, int fn, int64_t n, const double *x, double *out);

/* Message describing the last failure on this context (or on creation, with ctx NULL). */
const char *gq_last_error(gq_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GIGAQBX_H */
