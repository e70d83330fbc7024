// Per-center geometry features and order prediction for the order-prediction network.
//
// The QBX truncation error at a center is governed by how far the expansion radius is from the
// nearest singularity of the local field (the curve near the center, other parts of the curve or
// other curves) and by how well the quadrature resolves the sources inside a few radii (Sec. 4.1
// discusses both error sources). The features below measure exactly these quantities from the
// sources inside a disk of four expansion radii, found by walking the source tree.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gigaqbx_mlp.h"
#include "context.hpp"

namespace {

constexpr int kStack = 96;  // tree depth <= 28: a depth-first walk holds at most 3 d + 1 boxes

// Visit every source within distance R of x (leaf boxes whose square meets the disk), calling
// f(s) with the tree-order source index. Returns false if the stack would overflow (no source
// is skipped silently: the caller flags the center).
template <typename F>
__device__ bool walk_disk(int32_t root, double2 x, double R, const double2 *__restrict__ bc,
                          const int32_t *__restrict__ blevel, const int32_t *__restrict__ bchild,
                          const int32_t *__restrict__ bsrc0, const int32_t *__restrict__ bsrc1,
                          const double *__restrict__ level_side, F &&f) {
  int32_t stack[kStack];
  int sp = 0;
  stack[sp++] = root;
  const double R2 = R * R;
  while (sp > 0) {
    const int32_t b = stack[--sp];
    const double h = 0.5 * level_side[blevel[b]];
    const double2 c = bc[b];
    const double dx = fmax(fabs(x.x - c.x) - h, 0.0), dy = fmax(fabs(x.y - c.y) - h, 0.0);
    if (dx * dx + dy * dy >= R2) continue;
    const int4 ch = *reinterpret_cast<const int4 *>(bchild + 4 * (int64_t)b);
    if (ch.x < 0 && ch.y < 0 && ch.z < 0 && ch.w < 0) {
      for (int32_t s = bsrc0[b]; s < bsrc1[b]; ++s) f(s);
      continue;
    }
    if (sp + 4 > kStack) return false;
    if (ch.x >= 0) stack[sp++] = ch.x;
    if (ch.y >= 0) stack[sp++] = ch.y;
    if (ch.z >= 0) stack[sp++] = ch.z;
    if (ch.w >= 0) stack[sp++] = ch.w;
  }
  return true;
}

// One thread per tree-order center; writes GQ_N_FEATURES FP32 values at the caller's index.
__global__ void __launch_bounds__(256) k_center_features(
    int64_t nc, const double2 *__restrict__ cxy, const double *__restrict__ cr,
    const int32_t *__restrict__ cperm, const int32_t *__restrict__ cbox,
    const int32_t *__restrict__ bparent, const double2 *__restrict__ bc,
    const int32_t *__restrict__ blevel, const int32_t *__restrict__ bchild,
    const int32_t *__restrict__ bsrc0, const int32_t *__restrict__ bsrc1,
    const double *__restrict__ level_side, const double2 *__restrict__ sxy,
    const double2 *__restrict__ snrm, const double *__restrict__ sw, float *__restrict__ feat,
    int64_t nc_user, int32_t *__restrict__ overflow) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nc || cperm[k] >= nc_user) return;  // internal point-target centers have no row
  const double2 x = cxy[k];
  const double r = cr[k], R = 4.0 * r;
  // the root of this center's own tree (a context may hold several independent geometries)
  int32_t root = cbox[k];
  for (int guard = 0; guard < kStack && bparent[root] >= 0; ++guard) root = bparent[root];
  // pass 1: nearest source and its normal
  double dmin2 = 1e300;
  double2 n0 = make_double2(0.0, 0.0);
  bool ok = walk_disk(root, x, R, bc, blevel, bchild, bsrc0, bsrc1, level_side, [&](int32_t s) {
    const double2 y = sxy[s];
    const double d2 = (y.x - x.x) * (y.x - x.x) + (y.y - x.y) * (y.y - x.y);
    if (d2 < dmin2) { dmin2 = d2; n0 = snrm[s]; }
  });
  // pass 2: arc length, node count, normal coherence, normal offsets, opposite-facing sheet
  double a2 = 0.0, a4 = 0.0, cnt = 0.0, nx = 0.0, ny = 0.0, o1 = 0.0, o2 = 0.0;
  double sheet2 = R * R;
  ok &= walk_disk(root, x, R, bc, blevel, bchild, bsrc0, bsrc1, level_side, [&](int32_t s) {
    const double2 y = sxy[s], n = snrm[s];
    const double ex = y.x - x.x, ey = y.y - x.y, d2 = ex * ex + ey * ey;
    if (d2 >= R * R) return;
    const double w = sw[s];
    if (d2 < 4.0 * r * r) a2 += w;
    a4 += w;
    cnt += 1.0;
    nx += w * n.x;
    ny += w * n.y;
    const double o = (ex * n.x + ey * n.y) / r;
    o1 += w * o;
    o2 += w * o * o;
    if (n.x * n0.x + n.y * n0.y < 0.0) sheet2 = fmin(sheet2, d2);
  });
  float *f = feat + (int64_t)cperm[k] * GQ_N_FEATURES;
  const double inv_a4 = a4 > 0.0 ? 1.0 / a4 : 0.0;
  const double mean_o = o1 * inv_a4;
  f[0] = (float)(a2 / r * 0.25);
  f[1] = (float)(a4 / r * 0.125);
  f[2] = (float)(dmin2 < 1e299 ? sqrt(dmin2) / r : 4.0);
  f[3] = (float)(cnt > 0.0 ? log2(fmax(r * cnt * inv_a4, 1e-3)) : 0.0);
  f[4] = (float)(sqrt(nx * nx + ny * ny) * inv_a4);
  f[5] = (float)sqrt(fmax(o2 * inv_a4 - mean_o * mean_o, 0.0));
  f[6] = (float)mean_o;
  f[7] = (float)(sqrt(sheet2) / R);
  if (!ok) *overflow = 1;  // vector store; only ever set to 1
}

// orders[c] = smallest candidate j whose predicted log10 error (scale y_j + shift) is at most
// limit[j] (the tolerance less that candidate's margin); the largest candidate otherwise (also
// for non-finite predictions).
__global__ void k_choose_orders(int64_t n, int n_out, const float *__restrict__ y, float scale,
                                float shift, const float *__restrict__ limit,
                                const int32_t *__restrict__ cand, int32_t *__restrict__ orders) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int32_t q = cand[n_out - 1];
  for (int j = 0; j < n_out; ++j) {
    const float e = fmaf(scale, y[c * n_out + j], shift);
    if (e == e && e <= limit[j]) { q = cand[j]; break; }
  }
  orders[c] = q;
}

gq_status ofail(gq_ctx *ctx, gq_status st, const std::string &m) {
  if (ctx) ctx->err = m;
  return st;
}

#define GQ_ORD_HIP(ctx, call)                                                                  \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return ofail(ctx, GQ_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

extern "C" {

gq_status gq_center_features(gq_ctx *ctx, float *feat) {
  if (!ctx) return GQ_EINVAL;
  if (!ctx->built || ctx->device < 0)
    return ofail(ctx, GQ_ESTATE, "gq_center_features needs a successful gq_build on a device");
  if (!feat && ctx->nc_user > 0) return ofail(ctx, GQ_EINVAL, "null feature array");
  if (ctx->nc_user == 0) return GQ_OK;
  if (ctx->nc > INT32_MAX) return ofail(ctx, GQ_EUNSUP, "too many centers");
  GQ_ORD_HIP(ctx, hipSetDevice(ctx->device));
  int32_t *flag = nullptr;
  GQ_ORD_HIP(ctx, hipMalloc(&flag, sizeof(int32_t)));
  int32_t h_flag = 0;
  hipError_t e = hipMemcpyAsync(flag, &h_flag, sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream);
  const gq::DevBuffers &d = ctx->d;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_center_features, dim3((unsigned)((ctx->nc + 255) / 256)), dim3(256), 0,
                       ctx->stream, ctx->nc, d.cxy, d.cr, d.cperm, d.cbox, d.bparent, d.bc,
                       d.blevel, d.bchild, d.bsrc0,
                       d.bsrc1, d.level_side, d.sxy, d.snrm, d.sw, feat, ctx->nc_user, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(&h_flag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(flag);
  if (e != hipSuccess) return ofail(ctx, GQ_EHIP, std::string("center features: ") + hipGetErrorString(e));
  if (h_flag) return ofail(ctx, GQ_EUNSUP, "tree walk stack exhausted");
  return GQ_OK;
}

gq_status gq_orders_predict(gq_ctx *ctx, gq_mlp *net, const int32_t *cand, int n_cand,
                            double out_scale, double out_shift, double log10_tol,
                            const double *margins, int32_t *orders, int apply) {
  if (!ctx) return GQ_EINVAL;
  if (!net || !cand || n_cand < 1 || !orders) return ofail(ctx, GQ_EINVAL, "null argument or no candidates");
  int n_in = 0, n_out = 0;
  if (gq_mlp_shape(net, &n_in, nullptr, &n_out) != GQ_OK || n_in != GQ_N_FEATURES || n_out != n_cand)
    return ofail(ctx, GQ_EINVAL, "network inputs must be GQ_N_FEATURES and outputs n_cand");
  if (!ctx->built || ctx->device < 0)
    return ofail(ctx, GQ_ESTATE, "gq_orders_predict needs a successful gq_build on a device");
  for (int j = 0; j < n_cand; ++j)
    if (cand[j] < 0 || cand[j] > ctx->params.p_qbx || (j && cand[j] <= cand[j - 1]))
      return ofail(ctx, GQ_EINVAL, "candidate orders must ascend within 0..p_qbx");
  if (!std::isfinite(out_scale) || !std::isfinite(out_shift) || !std::isfinite(log10_tol))
    return ofail(ctx, GQ_EINVAL, "non-finite scale, shift or tolerance");
  std::vector<float> limit(n_cand);
  for (int j = 0; j < n_cand; ++j) {
    const double m = margins ? margins[j] : 0.0;
    if (!std::isfinite(m)) return ofail(ctx, GQ_EINVAL, "non-finite margin");
    limit[j] = (float)(log10_tol - m);
  }
  const int64_t nc = ctx->nc_user;
  if (nc == 0) return apply ? gq_set_qbx_orders(ctx, GQ_MEM_DEVICE, nullptr) : GQ_OK;
  GQ_ORD_HIP(ctx, hipSetDevice(ctx->device));
  float *feat = nullptr, *y = nullptr, *dlimit = nullptr;
  int32_t *dcand = nullptr;
  gq_status st = GQ_OK;
  if (hipMalloc(&feat, sizeof(float) * nc * GQ_N_FEATURES) != hipSuccess ||
      hipMalloc(&y, sizeof(float) * nc * n_cand) != hipSuccess ||
      hipMalloc(&dcand, sizeof(int32_t) * n_cand) != hipSuccess ||
      hipMalloc(&dlimit, sizeof(float) * n_cand) != hipSuccess)
    st = ofail(ctx, GQ_ENOMEM, "hipMalloc (order prediction)");
  if (st == GQ_OK && (hipMemcpy(dcand, cand, sizeof(int32_t) * n_cand, hipMemcpyHostToDevice) != hipSuccess ||
                      hipMemcpy(dlimit, limit.data(), sizeof(float) * n_cand, hipMemcpyHostToDevice) != hipSuccess))
    st = ofail(ctx, GQ_EHIP, "hipMemcpy (candidates, limits)");
  if (st == GQ_OK) st = gq_center_features(ctx, feat);
  // the network runs on its own stream: gq_center_features returned after its stream drained
  if (st == GQ_OK) {
    st = gq_mlp_forward(net, nc, feat, y);
    if (st != GQ_OK) ctx->err = std::string("network: ") + gq_mlp_last_error(net);
  }
  if (st == GQ_OK) {
    hipStream_t ns = static_cast<hipStream_t>(gq_mlp_stream(net));
    hipLaunchKernelGGL(k_choose_orders, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, ns, nc,
                       n_cand, y, (float)out_scale, (float)out_shift, dlimit, dcand, orders);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(ns);
    if (e != hipSuccess) st = ofail(ctx, GQ_EHIP, std::string("order choice: ") + hipGetErrorString(e));
  }
  (void)hipFree(feat);
  (void)hipFree(y);
  (void)hipFree(dcand);
  (void)hipFree(dlimit);
  if (st == GQ_OK && apply) st = gq_set_qbx_orders(ctx, GQ_MEM_DEVICE, orders);
  return st;
}

}  // extern "C"
