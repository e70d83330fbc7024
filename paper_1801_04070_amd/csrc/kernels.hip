// HIP kernels (gfx950) for the GIGAQBX FMM stages and direct QBX.
//
// Expansion scaling (see tables.hpp): box multipoles are stored as a_k / s^k and box locals as
// b_k s^k with s the box side; QBX local coefficients of a center of radius r are stored as
// alpha_m r^m, so the QBX expansion is evaluated at the target as sum_m alpha_m ((x - c)/r)^m.
//
// Kinds (template KIND): 1 = single layer (charges q = w sigma), 2 = double layer (dipoles
// w tau n), 3 = S(sigma) - D(tau). With z = y - c the source contributions are
//   charge:  alpha_0 += q log|z|,   alpha_m += -q / (m z^m)        (eq. (local), eq. (qbx))
//   dipole:  alpha_m += d / z^(m+1),  d = w tau n                    (Re(n/(y - x)) kernel)
// and the multipole of a box about c_b (eq. (multipole)):
//   charge:  a_0 += q,  a_k += -q z^k / k;   dipole: a_k += -d z^(k-1).
#include "context.hpp"
#include "cplx.hpp"
#include "kernels.hpp"

namespace gq {

namespace {

// Natural log of a positive normal double, table-driven in the manner of P. T. P. Tang, "Table-
// driven implementation of the logarithm function in IEEE floating-point arithmetic" (ACM TOMS
// 16(4), 1990): x = M 2^(e-1) with M in [1, 2); the top 7 bits of M pick j, c_j ~ 1/(1 + (j +
// 1/2)/128) and T_j = -log c_j (both rounded to FP64 on the host in long double, T_j from the
// rounded c_j), so log M = T_j + log1p(r) with r = M c_j - 1 formed by one FMA (exact),
// |r| <= 2^-8, and log1p(r) by its Taylor series through r^7 (the next term is below 2^-64 r).
// (e - 1) log 2 uses a two-part log 2: the head is log 2 rounded to a multiple of 2^-32 (32
// significant bits, so (e - 1) times it is exact for any double exponent) and the tail the
// remainder rounded to FP64; both were derived from a 60-digit value of log 2. Absolute error
// about 1e-16 over the normal doubles (a GPU test sweeps the exponent range against numpy).
constexpr int kLogTab = 128;
constexpr double kLn2Head = 0x1.62e42ffp-1;                 // round(2^32 log 2) / 2^32
constexpr double kLn2Tail = -0x1.718432a1b0e26p-35;          // log 2 - kLn2Head
__device__ double2 g_log_tab[kLogTab];

__device__ __forceinline__ double log_tab(double x, const double2 *__restrict__ tab) {
  int e;
  const double M = 2.0 * frexp(x, &e);
  const double2 ct = tab[(__double2hiint(M) >> 13) & (kLogTab - 1)];
  const double r = fma(M, ct.x, -1.0);
  double p = fma(r, 1.0 / 7.0, -1.0 / 6.0);
  p = fma(p, r, 1.0 / 5.0);
  p = fma(p, r, -0.25);
  p = fma(p, r, 1.0 / 3.0);
  p = fma(p, r, -0.5);
  const double l1 = fma(r * r, p, r);
  const double fe = (double)(e - 1);
  return fma(fe, kLn2Head, fma(fe, kLn2Tail, ct.y) + l1);
}

// The moments, M2L, P2L and the Stage 7 gather run on the caller's stream and form the critical
// path of an evaluation; their waves take issue priority over the direct pass's waves (side
// stream) on a SIMD they share.
__device__ __forceinline__ void critical_path_priority() { __builtin_amdgcn_s_setprio(1); }

constexpr double kInv2Pi = 0.159154943091895335768883763372514362;





// ------------------------------------------------------------------------------------------
// Source strengths in tree order: q = w sigma, dipole d = w tau n (with the minus sign of S - D).
template <int KIND>
__global__ void k_gather(int32_t ns, const int32_t *__restrict__ sperm, const double *__restrict__ sw,
                         const double2 *__restrict__ snrm, const double *__restrict__ d1,
                         int64_t ld1, const double *__restrict__ d2, int64_t ld2,
                         double *__restrict__ sq, double2 *__restrict__ sdip) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int64_t jd = blockIdx.y;  // density of the batch
  d1 += jd * ld1;
  if (KIND == 3) d2 += jd * ld2;
  sq += jd * ns;
  sdip += jd * ns;
  const int32_t o = sperm[i];
  const double w = sw[i];
  if (KIND == 1) sq[i] = w * d1[o];
  if (KIND == 2) sdip[i] = cscale(snrm[i], w * d1[o]);
  if (KIND == 3) {
    sq[i] = w * d1[o];
    sdip[i] = cscale(snrm[i], -w * d2[o]);
  }
  if (KIND == 4) {  // S and D of the same density: charge and dipole from one value
    const double v = w * d1[o];
    sq[i] = v;
    sdip[i] = cscale(snrm[i], v);
  }
}

// ------------------------------------------------------------------------------------------
// A double moved between lanes by one DPP pattern (CTRL), both halves alike; a lane whose source
// lies outside its row reads 0.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// The value of lane + o (o = 1, 2, 4, ... 32) for the group sums below, which need their result
// only in the lowest group of lanes: DPP row shifts (row_shl) within 16-lane rows for o < 16, a
// shuffle across rows otherwise.
__device__ __forceinline__ double lane_down(double v, int o) {
  switch (o) {
    case 1: return dpp_mov<0x101>(v);
    case 2: return dpp_mov<0x102>(v);
    case 4: return dpp_mov<0x104>(v);
    case 8: return dpp_mov<0x108>(v);
    default: return __shfl_down(v, o, 64);
  }
}

// The value of lane ^ 1 (quad_perm 1, 0, 3, 2).
__device__ __forceinline__ double lane_xor1(double v) { return dpp_mov<0xB1>(v); }

// ------------------------------------------------------------------------------------------
// Stage 2 as direct moments: the multipole of every box that M2L or M2QBXL reads is formed from
// the sources of its subtree (contiguous in tree order). In 2-D, M2M keeps the first p + 1
// moments of a box exact (coefficient m of the parent depends only on the children's
// coefficients k <= m), so these are the multipoles the level-by-level pass builds, up to
// rounding. One work item = one box and up to 512 of its sources; a box with more sources is
// split into several items whose partial sums k_m_reduce adds in a fixed order.
// Lanes: NBLK blocks of 8 consecutive orders (k = 8 kb + i) times 64 / NBLK source groups. A lane
// walks the sources of its group, forms y^(8 kb) by repeated squaring and the block's powers by a
// chain of complex multiplies, and accumulates A_k = sum q y^k and B_k = sum d y^k in registers;
// a fixed shift-down tree (lane_down) then sums the groups into lanes 0..NBLK-1. Coefficient k
// of the single layer is A_0 (k = 0) or -A_k / k, of the double layer B_(k-1) (0 at k = 0).
// KIND 3 stores their sum (one expansion), KIND 4 (S and D of one density) both, the D
// multipole d_off coefficients after the S one.
// A split box's items write partial rows [S: P1][D: P1] to Mp for k_m_reduce.
template <int KIND, int NBLK, typename E>
__global__ void __launch_bounds__(64) k_p2m_all(
    const int4 *__restrict__ items, const double2 *__restrict__ bc,
    const int32_t *__restrict__ blevel, const double *__restrict__ level_inv_side,
    const double2 *__restrict__ sxy, const double *__restrict__ sq,
    const double2 *__restrict__ sdip, int P1, E *__restrict__ M, double2 *__restrict__ Mp,
    int64_t src_st, int64_t box_st, int64_t part_st, int64_t d_off) {
  critical_path_priority();
  constexpr bool HQ = (KIND & 1) || KIND == 4, HD = (KIND & 2) || KIND == 4;
  constexpr int G = 64 / NBLK;
  const int4 it = items[blockIdx.x];  // box, first source, end of sources, partial slot or -1
  const int32_t b = it.x;
  const int lane = threadIdx.x;
  const int kb = lane % NBLK, g = lane / NBLK;
  {
    const int64_t jd = blockIdx.y;
    sq += jd * src_st;
    sdip += jd * src_st;
    M += jd * box_st;
    Mp += jd * part_st;
  }
  const double2 c = bc[b];
  const double is = level_inv_side[blevel[b]];
  double2 A[8], B[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    A[i] = make_double2(0.0, 0.0);
    B[i] = make_double2(0.0, 0.0);
  }
  for (int32_t s = it.y + g; s < it.z; s += G) {
    const double2 y = make_double2((sxy[s].x - c.x) * is, (sxy[s].y - c.y) * is);
    const double q = HQ ? sq[s] : 0.0;
    const double2 d = HD ? cscale(sdip[s], -is) : make_double2(0.0, 0.0);
    // y^(8 kb)
    double2 pw = make_double2(1.0, 0.0);
    if (NBLK > 1) {
      const double2 y2 = cmul(y, y), y4 = cmul(y2, y2), y8 = cmul(y4, y4);
      if (kb & 1) pw = y8;
      if (NBLK > 2) {
        const double2 y16 = cmul(y8, y8);
        if (kb & 2) pw = (kb & 1) ? cmul(y16, y8) : y16;
        if (NBLK > 4) {
          const double2 y32 = cmul(y16, y16);
          if (kb & 4) pw = cmul(pw, y32);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (HQ) A[i] = caxpy(q, pw, A[i]);
      if (HD) B[i] = cfma(d, pw, B[i]);
      if (i < 7) pw = cmul(pw, y);
    }
  }
#pragma unroll
  for (int o = NBLK; o < 64; o <<= 1) {  // group g adds group g + o / NBLK: lanes 0..NBLK-1 sum
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (HQ) {
        A[i].x += lane_down(A[i].x, o);
        A[i].y += lane_down(A[i].y, o);
      }
      if (HD) {
        B[i].x += lane_down(B[i].x, o);
        B[i].y += lane_down(B[i].y, o);
      }
    }
  }
  // B_(8 kb - 1) from the lane of the previous block (lanes 0..NBLK-1 hold the sums)
  double2 Bprev = make_double2(0.0, 0.0);
  if (HD) {
    Bprev.x = __shfl(B[7].x, lane - 1, 64);
    Bprev.y = __shfl(B[7].y, lane - 1, 64);
  }
  if (g != 0) return;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = 8 * kb + i;
    if (k >= P1) break;
    double2 sv = make_double2(0.0, 0.0), dv = make_double2(0.0, 0.0);
    if (HQ) sv = k == 0 ? A[0] : cscale(A[i], -1.0 / k);
    if (HD) dv = i > 0 ? B[i - 1] : (kb > 0 ? Bprev : make_double2(0.0, 0.0));
    if (it.w >= 0) {
      double2 *o = Mp + (int64_t)it.w * 2 * P1;
      if (KIND == 4) {
        o[k] = sv;
        o[P1 + k] = dv;
      } else {
        o[k] = KIND == 1 ? sv : KIND == 2 ? dv : cadd(sv, dv);
      }
    } else if (KIND == 4) {
      M[(int64_t)b * P1 + k] = from_d2<E>(sv);
      M[d_off + (int64_t)b * P1 + k] = from_d2<E>(dv);
    } else {
      M[(int64_t)b * P1 + k] = from_d2<E>(KIND == 1 ? sv : KIND == 2 ? dv : cadd(sv, dv));
    }
  }
}

// Sum of a split box's partial moments, one work-group of W wavefronts per box: the partials are
// taken in chunks of 16 (chunk c by wavefront c mod W), each lane holding sixteen running sums of
// one coefficient (one per position in a chunk, their loads issued together, clamped to the last
// partial, extra values unused); the sixteen are combined by a fixed pairwise tree and the
// wavefronts' sums in wavefront order through LDS, so the result is deterministic. W = 4 for one
// density (the largest box waits on a quarter of the dependent loads of one wavefront), 1 for
// batches (grid.y already holds the densities, and most split boxes have few partials).
template <int NK, int W, typename E>
__global__ void __launch_bounds__(64 * W) k_m_reduce(const int4 *__restrict__ red,
                                                            const double2 *__restrict__ Mp,
                                                            int P1, E *__restrict__ M,
                                                            int64_t part_st, int64_t box_st,
                                                            int64_t d_off) {
  critical_path_priority();
  __shared__ double2 wsum[W][64];
  const int4 it = red[blockIdx.x];  // box, first partial, end of partials
  const int64_t jd = blockIdx.y;
  Mp += jd * part_st;
  M += jd * box_st;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int U = 16;
  for (int r0 = 0; r0 < NK * P1; r0 += 64) {
    const int r = r0 + lane;
    double2 a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = make_double2(0.0, 0.0);
    if (r < NK * P1)
      for (int32_t p = it.y + U * wv; p < it.z; p += U * W) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t q = p + u;
          const double2 v = Mp[(int64_t)(q < it.z ? q : it.z - 1) * 2 * P1 + r];
          if (q < it.z) a[u] = cadd(a[u], v);
        }
      }
#pragma unroll
    for (int w = U / 2; w >= 1; w >>= 1)
#pragma unroll
      for (int u = 0; u < w; ++u) a[u] = cadd(a[u], a[u + w]);
    wsum[wv][lane] = a[0];
    __syncthreads();
    if (wv == 0 && r < NK * P1) {
      double2 sum = wsum[0][lane];
#pragma unroll
      for (int w = 1; w < W; ++w) sum = cadd(sum, wsum[w][lane]);
      if (r < P1) M[(int64_t)it.x * P1 + r] = from_d2<E>(sum);
      else M[d_off + (int64_t)it.x * P1 + (r - P1)] = from_d2<E>(sum);
    }
    __syncthreads();  // wsum is written again for the next 64 coefficients
  }
}

// ------------------------------------------------------------------------------------------
// Stages 4 and 6b: box local L_b = M2L over List 2 + P2L over List 4 far.
//
// M2L (eq. (m2l), corrected a_0 sign) in factored form beta_m = o^-m sum_k B[m][k] (a_k o^-k)
// (+ a_0 log|s o| in beta_0) on the matrix cores: the fixed real matrix B is the A operand of
// v_mfma_f64_16x16x4f64 (RT row tiles x 4 RT k-steps, held in registers for the whole wavefront),
// and a batch of 8 List 2 pairs gives the 16 real columns (re/im of a_k o^-k per pair) of the B
// operand. The 16 x 16 results are scaled by o^-m per pair and written to LDS by pair and row,
// where lane m sums row m over the batch (one LDS round trip instead of a shuffle tree per row).
// Operand layout of the FP64 16x16x4 instruction: A[i][k] in lane i + 16 k, B[k][j] in lane
// j + 16 k, D[g + 4 v][j] in element v of lane j + 16 g.
typedef double gq_d4 __attribute__((ext_vector_type(4)));
typedef float gq_f4 __attribute__((ext_vector_type(4)));

// One 16x16x4 matrix-core step in the expansion precision, and the output row held in element v of
// a lane of 16-lane group g (FP64: g + 4 v, FP32: 4 g + v).
__device__ __forceinline__ gq_d4 mfma16(double a, double b, gq_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ gq_f4 mfma16(float a, float b, gq_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename R> struct Mfma16;
template <> struct Mfma16<double> {
  using Acc = gq_d4;
  static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};
template <> struct Mfma16<float> {
  using Acc = gq_f4;
  static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};

// M2L over a flat list of List 2 pairs (one slot per grid row): a wavefront takes a run of whole
// target boxes (about 64 pairs), in batches of 8 consecutive pairs that may span boxes (each
// matrix-core column is its own pair). The next batch's pair records and multipole rows are
// fetched while the current batch runs on the matrix cores; lane m then adds row m of each pair
// in pair order and writes a box's local when the next box starts. Pair record: (source box d,
// offset index, target box, 0), d = -1 for a target box without List 2 pairs (its local is 0);
// plog = log s_b + log|o| for the a_0 term. For FP64 the row factors o^-m a lane needs are the
// o^-k it loaded for its operands (row 16 rt + g + 4 v = order 4 ks + g with ks = 4 rt + v).
template <int RT, typename E>
__global__ void __launch_bounds__(64) k_m2l_mb(
    const int2 *__restrict__ items, const int4 *__restrict__ prs,
    const double *__restrict__ plog, const E *__restrict__ M,
    const typename Scalar<E>::T *__restrict__ Bt, const E *__restrict__ opow, int P1,
    E *__restrict__ L, int64_t box_st) {
  critical_path_priority();
  using R = typename Scalar<E>::T;
  using Acc = typename Mfma16<R>::Acc;
  constexpr int KS = 4 * RT;
  constexpr bool F64 = sizeof(R) == 8;
  __shared__ double2 Pt[8][16 * RT];
  __shared__ int32_t Pb[8];
  const int2 it = items[blockIdx.x];  // first pair, end of pairs
  {
    const int64_t jd = blockIdx.y;
    M += jd * box_st;
    L += jd * box_st;
  }
  const int lane = threadIdx.x;
  const int g = lane >> 4, c16 = lane & 15;
  const int pr = c16 >> 1, comp = c16 & 1;
  R A[RT][KS];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int i = 16 * rt + c16, k = 4 * ks + g;
      A[rt][ks] = (i < P1 && k < P1) ? Bt[k * P1 + i] : R(0);
    }
  // operands of the batch at j: pair record, a_0 log factor, M_d[k] and o^-k for this lane's k
  int4 rec;
  double pl;
  E mdv[KS], opv[KS];
  auto fetch = [&](int32_t j) {
    const int32_t p = j + pr;
    const bool in = p < it.y;
    const int32_t pc = in ? p : it.y - 1;  // in-bounds load, then select
    const int4 rv = prs[pc];
    const double lv = plog[pc];
    rec = in ? rv : make_int4(-1, 0, -1, 0);
    pl = in ? lv : 0.0;
    const bool pv = rec.x >= 0;
    const E *Md = M + (int64_t)(pv ? rec.x : 0) * P1;
    const E *op = opow + (int64_t)rec.y * P1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      // loads from in-bounds addresses, then selects: no branch around each load
      const int k = 4 * ks + g, kc = k < P1 ? k : P1 - 1;
      const E mv = Md[kc], ov = op[kc];
      mdv[ks] = (pv && k < P1) ? mv : mk2<E>(0.0, 0.0);
      opv[ks] = k < P1 ? ov : mk2<E>(0.0, 0.0);
    }
  };
  fetch(it.x);
  double2 acc = make_double2(0.0, 0.0);
  int32_t cur = -1;
  for (int32_t j0 = it.x; j0 < it.y; j0 += 8) {
    const int nbat = min(8, (int)(it.y - j0));
    const int4 rc = rec;
    const double plc = pl;
    E mdc[KS], opc[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      mdc[ks] = mdv[ks];
      opc[ks] = opv[ks];
    }
    if (j0 + 8 < it.y) fetch(j0 + 8);  // in flight during this batch
    R Bf[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const E mk = mdc[ks], ok = opc[ks];
      Bf[ks] = comp ? mk.x * ok.y + mk.y * ok.x : mk.x * ok.x - mk.y * ok.y;
    }
    Acc C[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      C[rt] = Acc{R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) C[rt] = mfma16(A[rt][ks], Bf[ks], C[rt]);
    }
    const E *opr = opow + (int64_t)rc.y * P1;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * rt + Mfma16<R>::row(g, v);
        const double y = C[rt][v];
        const double yo = lane_xor1(y);
        if (!comp && m < P1) {
          const E om = F64 ? opc[4 * rt + v] : opr[m];
          double2 t = cmul(make_double2(y, yo), to_d2(om));
          if (m == 0) t.x = fma((double)mdc[0].x, plc, t.x);  // a_0 log|s o| (lane g = 0)
          Pt[pr][m] = t;
        }
      }
    if (c16 == 2 * pr && g == 0 && !comp) Pb[pr] = rc.z;
    __syncthreads();
    if (lane < P1) {
      // the batch's rows and boxes read together, then summed in pair order
      double2 v[8];
      int32_t bxs[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        v[p] = Pt[p][lane];
        bxs[p] = Pb[p];
      }
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if (p >= nbat) break;
        if (bxs[p] != cur) {
          if (cur >= 0) L[(int64_t)cur * P1 + lane] = from_d2<E>(acc);
          acc = make_double2(0.0, 0.0);
          cur = bxs[p];
        }
        acc = cadd(acc, v[p]);
      }
    }
    __syncthreads();
  }
  if (lane < P1 && cur >= 0) L[(int64_t)cur * P1 + lane] = from_d2<E>(acc);
}

// ------------------------------------------------------------------------------------------
// M2L (Stage 4) and the Stage 7 gather over many workspace slots (a density batch, S and D): the
// pair-dependent factors are diagonal, so every pair is one small GEMM whose columns are the
// slots. A wavefront takes 8 slots (16 real columns: re/im of each), the fixed matrix T is the
// A operand held in registers, and the pair's input rows scaled by the pre-factors f_k are the
// B operand; the products, scaled by the post-factors g_m, accumulate in registers over the pairs
// of a target box (all columns belong to the same pair), and a box's rows are written once, when
// its last pair is done. A work-group takes 8 NW slots (NW wavefronts) of one run of whole boxes
// of the flat pair lists that k_m2l_mb and k_l2l_gather walk.
//   M2L:    f_k = o^-k, g_m = o^-m, T = B (the List 2 offset tables), plus a_0 log|s o| in beta_0;
//   gather: f_k = t^k,  g_m = u^-m, T = C(k, m); a box's own local is added when it is written.
// FP64 rows 16 rt + g + 4 v are the orders 4 (4 rt + v) + g, the orders 4 ks + g of the lane's
// k-steps, so one set of per-lane factors serves both sides; FP32 rows (16 rt + 4 g + v) take
// their post-factors separately. Arithmetic of the products in the expansion precision, of the
// post-scaling and the sums in FP64.
template <typename R>
__device__ __forceinline__ double slot_post(double y, int comp, double2 gm) {
  const double yo = lane_xor1(y);
  const double yr = comp ? yo : y, yi = comp ? y : yo;
  return comp ? fma(gm.x, yi, gm.y * yr) : fma(gm.x, yr, -(gm.y * yi));
}

template <int RT, typename E>
__global__ void __launch_bounds__(256) k_m2l_slots(
    int32_t n_items, const int2 *__restrict__ items, const int4 *__restrict__ prs,
    const double *__restrict__ plog, const E *__restrict__ M,
    const typename Scalar<E>::T *__restrict__ Bt, const E *__restrict__ opow, int P1,
    E *__restrict__ L, int64_t box_st, int n_slots) {
  critical_path_priority();
  using R = typename Scalar<E>::T;
  using Acc = typename Mfma16<R>::Acc;
  constexpr int KS = 4 * RT;
  constexpr bool F64 = sizeof(R) == 8;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int slot0 = (blockIdx.y * (blockDim.x >> 6) + wv) * 8;
  (void)n_items;
  const int g = lane >> 4, c16 = lane & 15, comp = c16 & 1;
  const int slot = slot0 + (c16 >> 1);
  const bool sact = slot < n_slots;
  M += (int64_t)(sact ? slot : slot0) * box_st;
  L += (int64_t)(sact ? slot : slot0) * box_st;
  // the fixed matrix in LDS, in the A-operand order of each (row tile, k-step): one read per
  // matrix-core step instead of RT KS registers per lane
  __shared__ R As[RT][KS][64];
  for (int e = threadIdx.x; e < RT * KS * 64; e += blockDim.x) {
    const int l = e & 63, ks = (e >> 6) % KS, rt = (e >> 6) / KS;
    const int i = 16 * rt + (l & 15), k = 4 * ks + (l >> 4);
    As[rt][ks][l] = (i < P1 && k < P1) ? Bt[k * P1 + i] : R(0);
  }
  __syncthreads();
  // every thread of the work-group has filled the matrix; a wavefront past the last slot stops
  if (slot0 >= n_slots) return;
  const int2 it = items[blockIdx.x];  // first pair, end of pairs
  int4 rec;
  double pl;
  E inv[KS], fv[KS], gv[F64 ? 1 : 4 * RT];
  auto fetch = [&](int32_t j) {
    rec = prs[j];
    pl = plog[j];
    const bool pv = rec.x >= 0;
    const E *Md = M + (int64_t)(pv ? rec.x : 0) * P1;
    const E *op = opow + (int64_t)rec.y * P1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + g, kc = k < P1 ? k : P1 - 1;
      // raw loads (a select here would wait for them at once): orders k >= P1 meet zero columns
      // of the fixed matrix, and a pair without a source box is skipped
      inv[ks] = Md[kc];
      fv[ks] = op[kc];
    }
    if (!F64) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * rt + Mfma16<R>::row(g, v), mc = m < P1 ? m : P1 - 1;
          gv[F64 ? 0 : 4 * rt + v] = op[mc];
        }
    }
  };
  double acc[RT][4];
  auto flush = [&](int32_t b) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * rt + Mfma16<R>::row(g, v);
        if (sact && m < P1) reinterpret_cast<R *>(L + (int64_t)b * P1 + m)[comp] = (R)acc[rt][v];
        acc[rt][v] = 0.0;
      }
  };
  fetch(it.x);
  int32_t cur = rec.z;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[rt][v] = 0.0;
  for (int32_t j = it.x; j < it.y; ++j) {
    // the B operand and the factors this pair needs are taken before the next pair's loads are
    // issued into the same registers
    const int4 rc = rec;
    const double plc = pl;
    const double a0 = (double)inv[0].x;
    R Bf[KS];
    E fc[F64 ? KS : 1], gc[F64 ? 1 : 4 * RT];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const E mk = inv[ks], ok = fv[ks];
      Bf[ks] = comp ? mk.x * ok.y + mk.y * ok.x : mk.x * ok.x - mk.y * ok.y;
      if (F64) fc[F64 ? ks : 0] = ok;
    }
    if (!F64) {
#pragma unroll
      for (int q = 0; q < 4 * RT; ++q) gc[F64 ? 0 : q] = gv[F64 ? 0 : q];
    }
    if (j + 1 < it.y) fetch(j + 1);  // in flight during this pair's matrix-core work
    if (rc.z != cur) {
      flush(cur);
      cur = rc.z;
    }
    if (rc.x < 0) continue;  // a box without List 2 pairs: its local is 0
    Acc C[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      C[rt] = Acc{R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) C[rt] = mfma16(As[rt][ks][lane], Bf[ks], C[rt]);
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * rt + Mfma16<R>::row(g, v);
        const double2 gm = to_d2(F64 ? fc[F64 ? (4 * rt + v) % KS : 0] : gc[F64 ? 0 : 4 * rt + v]);
        double val = slot_post<R>((double)C[rt][v], comp, gm);
        if (m == 0 && !comp) val = fma(a0, plc, val);  // a_0 log|s o|
        acc[rt][v] += val;
      }
  }
  flush(cur);
}

// Direct load from global memory into LDS: every active lane moves N bytes from its own address
// to lds + N * lane (lds is the same for the whole wavefront); counted by vmcnt.
template <int N>
__device__ __forceinline__ void load_to_lds(const void *src, void *lds) {
  static_assert(N == 4 || N == 16, "4 or 16 bytes per lane");
  auto *l = (__attribute__((address_space(3))) void *)lds;
  if constexpr (N == 16)
    __builtin_amdgcn_global_load_lds(src, l, 16, 0, 0);
  else
    __builtin_amdgcn_global_load_lds(src, l, 4, 0, 0);
}

// M2L over a density batch with the target boxes grouped by parent: a record is one source box
// and the offsets of the (up to four) sibling targets that list it, so its multipole rows are
// loaded once and serve every member; each member has its own accumulators, written when the
// group ends. The fixed matrix is held in registers in A-operand order, the o^-k rows of the
// offsets in use sit in LDS, and the next record's multipole rows travel from memory straight
// into a per-wavefront LDS buffer (no registers held while they are in flight). A lane of a real
// column keeps (Re M_k, -Im M_k) and a lane of an imaginary column (Im M_k, Re M_k), so the
// pre-scaled operand is Re or Im of o^-k M_k with one product and one fma; the post-factor o^-m
// enters the same way, with Im o^-m signed by the column.
template <int RT, typename E>
__global__ void __launch_bounds__(256) k_m2l_grp(
    const int2 *__restrict__ items, const int4 *__restrict__ recs,
    const double4 *__restrict__ plog, const int4 *__restrict__ grp, const E *__restrict__ M,
    const typename Scalar<E>::T *__restrict__ Bt, const E *__restrict__ opow, int n_off, int P1,
    E *__restrict__ L, int64_t box_st, int n_slots) {
  critical_path_priority();
  using R = typename Scalar<E>::T;
  using Acc = typename Mfma16<R>::Acc;
  constexpr int KS = 4 * RT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int slot0 = (blockIdx.y * (blockDim.x >> 6) + wv) * 8;
  const int g = lane >> 4, c16 = lane & 15, comp = c16 & 1;
  const int slot = slot0 + (c16 >> 1);
  const bool sact = slot < n_slots;
  const R sgn = comp ? R(1) : R(-1);
  L += (int64_t)(sact ? slot : slot0) * box_st;
  // LDS: the o^-k table [n_off][P1], then per wavefront the staged rows of one record, entry
  // (ks, g, s) = 32 ks + 8 g + s holding M_(4 ks + g) of slot slot0 + s (zero where k >= P1)
  extern __shared__ unsigned char dyn_lds[];
  E *Os = reinterpret_cast<E *>(dyn_lds);
  E *Mb = Os + ((n_off * P1 + 1) & ~1) + wv * (KS * 32);
  for (int e = threadIdx.x; e < n_off * P1; e += blockDim.x) Os[e] = opow[e];
  for (int e = lane; e < KS * 32; e += 64) Mb[e] = mk2<E>(0.0, 0.0);
  __syncthreads();
  // every thread of the work-group has filled the tables; a wavefront past the last slot stops
  if (slot0 >= n_slots) return;
  R A[RT][KS];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int i = 16 * rt + c16, k = 4 * ks + g;
      A[rt][ks] = (i < P1 && k < P1) ? Bt[k * P1 + i] : R(0);
    }
  // the loader lanes: a direct load moves U bytes per lane (a whole FP64 entry, or half of an FP32
  // one), so instruction h fills the EPI entries from EPI h on; entry e is k-step e / 32, order
  // 4 (e / 32) + (e / 8) % 4, slot slot0 + e % 8
  constexpr int U = sizeof(E) == 16 ? 16 : 4, EPI = 64 * U / (int)sizeof(E), NI = KS * 32 / EPI;
  const int le = U == 16 ? lane : lane >> 1, ls = le & 7, lg = (le >> 3) & 3;
  const bool lact = slot0 + ls < n_slots;
  const char *Ml = reinterpret_cast<const char *>(M + (int64_t)(lact ? slot0 + ls : slot0) * box_st) +
                   (U == 16 ? 0 : 4 * (lane & 1));
  auto stage = [&](int32_t src) {  // rows of box src into this wavefront's buffer
    if (src < 0) return;
#pragma unroll
    for (int h = 0; h < NI; ++h) {
      const int k = 4 * ((EPI * h + le) >> 5) + lg;
      if (lact && k < P1)
        load_to_lds<U>(Ml + ((int64_t)src * P1 + k) * (int64_t)sizeof(E),
                       reinterpret_cast<char *>(Mb) + 64 * U * h);
    }
  };
  const int2 it = items[blockIdx.x];  // first record, end of records
  // the records are read two ahead, so that staging the next record's rows waits for nothing
  int4 rec = recs[it.x], rnx = recs[it.x + 1 < it.y ? it.x + 1 : it.x];
  stage(rec.x);
  int32_t cur = rec.z;
  int4 tg = grp[rec.z];
  double acc[4][RT][4];
  auto flush = [&](const int4 &t4) {
    const int32_t tb[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * rt + Mfma16<R>::row(g, v);
          if (tb[q] >= 0 && sact && m < P1)
            reinterpret_cast<R *>(L + (int64_t)tb[q] * P1 + m)[comp] = (R)acc[q][rt][v];
          acc[q][rt][v] = 0.0;
        }
  };
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[q][rt][v] = 0.0;
  const R *Mr = reinterpret_cast<const R *>(Mb + 8 * g + (c16 >> 1));
  for (int32_t j = it.x; j < it.y; ++j) {
    const int4 rc = rec;
    const double4 plc = plog[j];
    // this record's rows have landed (and the stores of a finished group are out)
    __builtin_amdgcn_s_waitcnt(0);
    R m0[KS], m1[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      m0[ks] = Mr[64 * ks + comp];
      const R o1 = Mr[64 * ks + 1 - comp];
      m1[ks] = comp ? o1 : -o1;
    }
    // the reads are complete before the buffer is filled again with the next record's rows
    __builtin_amdgcn_s_waitcnt(0xC07F);
    if (j + 1 < it.y) {
      rec = rnx;
      stage(rec.x);
      if (j + 2 < it.y) rnx = recs[j + 2];
    }
    if (rc.z != cur) {
      flush(tg);
      cur = rc.z;
      tg = grp[rc.z];
    }
    if (rc.x < 0) continue;  // a group without List 2 pairs: its locals are 0
    const double a0 = (double)m0[0];  // Re M_0 on the real columns of lanes g = 0
    const double plq[4] = {plc.x, plc.y, plc.z, plc.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = ((uint32_t)rc.y >> (8 * q)) & 0xFF;
      if (o == 0xFF) continue;
      const E *op = Os + o * P1;
      Acc C[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) C[rt] = Acc{R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + g, kc = k < P1 ? k : P1 - 1;
        const E ok = op[kc];
        const R bf = fma(m0[ks], ok.x, m1[ks] * ok.y);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) C[rt] = mfma16(A[rt][ks], bf, C[rt]);
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * rt + Mfma16<R>::row(g, v);
          const double y = (double)C[rt][v], yo = lane_xor1(y);
          const E om = op[m < P1 ? m : P1 - 1];
          const double px = (double)om.x, py = (double)(sgn * om.y);
          double a = fma(px, y, acc[q][rt][v]);
          if (m == 0 && !comp) a = fma(a0, plq[q], a);  // a_0 log|s o|
          acc[q][rt][v] = fma(py, yo, a);
        }
    }
  }
  flush(tg);
}

template <int RT, typename E>
__global__ void __launch_bounds__(256) k_l2l_slots(
    int32_t n_items, const int2 *__restrict__ items, const int2 *__restrict__ prs,
    const double4 *__restrict__ anc_tw, const double *__restrict__ binom_t, int P1,
    const E *__restrict__ L, E *__restrict__ Lf, int64_t box_st, int n_slots) {
  critical_path_priority();
  using R = typename Scalar<E>::T;
  using Acc = typename Mfma16<R>::Acc;
  constexpr int KS = 4 * RT;
  constexpr bool F64 = sizeof(R) == 8;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int slot0 = (blockIdx.y * (blockDim.x >> 6) + wv) * 8;
  (void)n_items;
  if (slot0 >= n_slots) return;
  const int2 it = items[blockIdx.x];
  const int g = lane >> 4, c16 = lane & 15, comp = c16 & 1;
  const int slot = slot0 + (c16 >> 1);
  const bool sact = slot < n_slots;
  L += (int64_t)(sact ? slot : slot0) * box_st;
  Lf += (int64_t)(sact ? slot : slot0) * box_st;
  // C(k, i) vanishes below the diagonal: row tile rt needs only k-steps ks >= 4 rt
  R A[RT][KS];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int i = 16 * rt + c16, k = 4 * ks + g;
      A[rt][ks] = (ks >= 4 * rt && i < P1 && k < P1) ? (R)binom_t[k * P1 + i] : R(0);
    }
  // the pairs are read two ahead, so that the loads of the next pair's rows wait for nothing
  int2 rec = prs[it.x], rnx = prs[it.x + 1 < it.y ? it.x + 1 : it.x];
  double4 tw;
  E inv[KS];
  auto fetch = [&](int32_t j) {
    tw = anc_tw[j];
    const bool pv = rec.x >= 0;
    const E *La = L + (int64_t)(pv ? rec.x : 0) * P1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + g, kc = k < P1 ? k : P1 - 1;
      inv[ks] = La[kc];  // raw: orders k >= P1 meet zero columns, a pair without ancestor is skipped
    }
  };
  double acc[RT][4];
  auto flush = [&](int32_t b) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * rt + Mfma16<R>::row(g, v);
        if (sact && m < P1) {
          const int64_t o = (int64_t)b * P1 + m;
          const double own = (double)reinterpret_cast<const R *>(L + o)[comp];
          reinterpret_cast<R *>(Lf + o)[comp] = (R)(own + acc[rt][v]);
        }
        acc[rt][v] = 0.0;
      }
  };
  fetch(it.x);
  int32_t cur = rec.y;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[rt][v] = 0.0;
  for (int32_t j = it.x; j < it.y; ++j) {
    const int2 rc = rec;
    const double4 twc = tw;
    E inc[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) inc[ks] = inv[ks];
    if (j + 1 < it.y) {
      rec = rnx;
      fetch(j + 1);
      if (j + 2 < it.y) rnx = prs[j + 2];
    }
    if (rc.y != cur) {
      flush(cur);
      cur = rc.y;
    }
    if (rc.x < 0) continue;  // no ancestor with a local of its own: Lf = L
    const double2 t = make_double2(twc.x, twc.y), w = make_double2(twc.z, twc.w);
    // pre-factors t^k, k = 4 ks + g
    double2 pw = make_double2(1.0, 0.0);
    for (int e = 0; e < g; ++e) pw = cmul(pw, t);
    const double2 t2 = cmul(t, t), t4 = cmul(t2, t2);
    R Bf[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const double2 x = cmul(pw, to_d2(inc[ks]));
      Bf[ks] = (R)(comp ? x.y : x.x);
      pw = cmul(pw, t4);
    }
    Acc C[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      C[rt] = Acc{R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int ks = 4 * rt; ks < KS; ++ks) C[rt] = mfma16(A[rt][ks], Bf[ks], C[rt]);
    }
    // post-factors u^-m for rows m = 16 rt + row(g, v)
    const double2 w2 = cmul(w, w), w4 = cmul(w2, w2), w8 = cmul(w4, w4), w16 = cmul(w8, w8);
    double2 wr = make_double2(1.0, 0.0);
    const int g0 = F64 ? g : 4 * g;  // order of row (g, 0) in the first tile
    for (int e = 0; e < g0; ++e) wr = cmul(wr, w);
    const double2 wstep = F64 ? w4 : w;  // from row (g, v) to (g, v + 1)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      double2 wv2 = wr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[rt][v] += slot_post<R>((double)C[rt][v], comp, wv2);
        wv2 = cmul(wv2, wstep);
      }
      wr = cmul(wr, w16);
    }
  }
  flush(cur);
}

// ------------------------------------------------------------------------------------------
// Stage 2 (direct moments, MODE 0) and Stage 6b (P2L, MODE 1) for S and D of a batch of
// densities on the matrix cores. For one box and its sources the coefficients of every density
// are one real GEMM: rows are the real and imaginary parts of the powers of the scaled offset
// (MODE 0: y^k for S, -n y^(k-1)/s for D; MODE 1: v^k with v = 1/y, log|s y| in row 0, for S and
// n v^(k+1)/s for D; the dipole is the charge times the normal), the k dimension the sources and
// the columns 64 densities; the charges q^(j) = w mu^(j) are the B operand for both kinds. The
// S rows (RTS tiles of 16) and D rows (RTD tiles) are spread over the four wavefronts of a
// work-group, TPW tiles each; the item's sources and the strengths of the 64 densities are
// staged in LDS 32 sources at a time. Row 16 rt + i of either block is power 8 rt + i/2 (MODE 1
// D: one more), so a lane forms x^(i/2) once per source and steps by x^8 between its tiles.
// Coefficients as k_p2m_all / k_p2l write them: S a_0 = sum q, a_k = -A_k / k (MODE 0), the log
// sum and -A_k / k (MODE 1); D from its rows directly. MODE 0 items of split boxes write partial
// rows for k_m_reduce; MODE 1 adds to the box locals that M2L wrote.
template <int MODE, int TPW, typename E>
__global__ void __launch_bounds__(256, 2) k_p2x_mfma(
    int32_t n_items, const int4 *__restrict__ items, const int32_t *__restrict__ src_idx,
    const double2 *__restrict__ bc, const int32_t *__restrict__ blevel,
    const double *__restrict__ level_inv_side, const double *__restrict__ level_log_side,
    const double2 *__restrict__ sxy, const double2 *__restrict__ snrm,
    const double *__restrict__ sq, int P1, E *__restrict__ Out,
    double2 *__restrict__ Mp, int64_t src_st, int64_t box_st, int64_t part_st, int nd,
    int64_t d_off) {
  critical_path_priority();
  using R = typename Scalar<E>::T;
  using Acc = typename Mfma16<R>::Acc;
  constexpr bool F64 = sizeof(R) == 8;
  constexpr int NT = 4, NDB = 64, SB = 32, SST = SB + 4;
  __shared__ double t_q[NDB][SST];
  __shared__ double2 t_y[SB], t_n[SB];
  __shared__ double2 t_log[kLogTab];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  (void)n_items;
  const int4 it = items[blockIdx.x];
  const int32_t b = it.x;
  const int d0 = blockIdx.y * NDB;
  const int lev = blevel[b];
  const double2 c = bc[b];
  const double is = level_inv_side[lev];
  const double logs = MODE == 1 ? level_log_side[lev] : 0.0;
  if (MODE == 1 && tid < kLogTab) t_log[tid] = g_log_tab[tid];
  const double2 *lt = t_log;
  const int RTS = (2 * P1 + 15) / 16;
  const int RTD = (2 * (MODE == 0 ? P1 - 1 : P1) + 15) / 16;
  const int i = lane & 15, kk = lane >> 4, h = i >> 1, comp = i & 1;
  const int ss = tid % SB, sd = tid / SB;
  const int32_t len = it.z - it.y;
  double rq[NDB / 8];
  double2 ry = make_double2(0.0, 0.0), rn = make_double2(0.0, 0.0);
  // a batch's source indices are read one batch ahead of its strengths, and the strengths are
  // kept raw until they are written to LDS (a select at the load would wait for it at once)
  auto index = [&](int32_t base) {
    const int nb = min(SB, (int)(len - base));
    const int32_t e = it.y + base + (ss < nb ? ss : 0);
    return MODE == 0 ? e : src_idx[e];
  };
  auto load = [&](int32_t src) {
    if (sd == 0) {
      ry = sxy[src];
      rn = snrm[src];
    }
#pragma unroll
    for (int q = 0; q < NDB / 8; ++q) {
      const int dj = d0 + sd + 8 * q;
      rq[q] = sq[(int64_t)(dj < nd ? dj : 0) * src_st + src];
    }
  };
  // this wavefront's tiles: t = wv TPW + u; S tile t < RTS, else D tile t - RTS
  int trt[TPW];
  bool tis_d[TPW], tact[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = wv * TPW + u;
    tis_d[u] = t >= RTS;
    trt[u] = tis_d[u] ? t - RTS : t;
    tact[u] = t < RTS + RTD;
  }
  // FP32 products are summed over one batch on the matrix cores, then into FP64 sums
  Acc C[TPW][NT];
  double Cd[F64 ? 1 : TPW][F64 ? 1 : NT][4];
#pragma unroll
  for (int u = 0; u < TPW; ++u)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      C[u][nt] = Acc{R(0), R(0), R(0), R(0)};
      if (!F64)
#pragma unroll
        for (int v = 0; v < 4; ++v) Cd[F64 ? 0 : u][F64 ? 0 : nt][v] = 0.0;
    }
  load(index(0));
  int32_t snx = SB < len ? index(SB) : 0;
  for (int32_t base = 0; base < len; base += SB) {
    const int nb = min(SB, (int)(len - base));
    __syncthreads();
    if (sd == 0) {
      t_y[ss] = ry;
      t_n[ss] = rn;
    }
#pragma unroll
    for (int q = 0; q < NDB / 8; ++q)
      t_q[sd + 8 * q][ss] = (ss < nb && d0 + sd + 8 * q < nd) ? rq[q] : 0.0;
    __syncthreads();
    if (base + SB < len) {
      load(snx);
      if (base + 2 * SB < len) snx = index(base + 2 * SB);
    }
    if (!tact[0]) continue;
    const int nks = (nb + 3) >> 2;
    for (int ks = 0; ks < nks; ++ks) {
      const int sl = 4 * ks + kk;
      const bool valid = sl < nb;
      const double2 yy = t_y[sl], nv = t_n[sl];
      const double2 y = make_double2((yy.x - c.x) * is, (yy.y - c.y) * is);
      double2 x = y;
      double lg = 0.0;
      if (MODE == 1) {
        const double r2 = valid ? cnorm2(y) : 1.0;
        const double ir2 = rcp_nr(r2);
        x = make_double2(y.x * ir2, -y.y * ir2);
        if (i == 0 && wv == 0) lg = fma(0.5, log_tab(r2, lt), logs);
      }
      const double2 one = make_double2(1.0, 0.0);
      const double2 x2 = cmul(x, x), x4 = cmul(x2, x2), x8 = cmul(x4, x4);
      const double2 xh = cmul(cmul((h & 1) ? x : one, (h & 2) ? x2 : one), (h & 4) ? x4 : one);
      const double2 nd_s = make_double2(nv.x * is, nv.y * is);  // n / s
      R a[TPW];
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        double2 p = xh;
        for (int q = 0; q < trt[u]; ++q) p = cmul(p, x8);
        const int k = 8 * trt[u] + h;
        double val;
        if (!tis_d[u]) {
          val = comp ? p.y : p.x;
          if (MODE == 1 && k == 0) val = comp ? 0.0 : lg;
          if (k >= P1) val = 0.0;
        } else {
          // MODE 0: row k is coefficient k + 1, -n y^k / s; MODE 1: row k, n v^(k+1) / s
          const double2 w = MODE == 0 ? cmul(make_double2(-nd_s.x, -nd_s.y), p)
                                      : cmul(nd_s, cmul(p, x));
          val = comp ? w.y : w.x;
          if (k >= (MODE == 0 ? P1 - 1 : P1)) val = 0.0;
        }
        a[u] = (R)((valid && tact[u]) ? val : 0.0);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const R bq = (R)t_q[16 * nt + i][sl];
#pragma unroll
        for (int u = 0; u < TPW; ++u) C[u][nt] = mfma16(a[u], bq, C[u][nt]);
      }
    }
    if (!F64) {
#pragma unroll
      for (int u = 0; u < TPW; ++u)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
          for (int v = 0; v < 4; ++v) Cd[F64 ? 0 : u][F64 ? 0 : nt][v] += (double)C[u][nt][v];
          C[u][nt] = Acc{R(0), R(0), R(0), R(0)};
        }
    }
  }
  // lane (column j, group g) holds rows 16 rt + row(g, v): order 8 rt + row/2, part row & 1
  const int g = kk, j = i;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int dj = d0 + 16 * nt + j;
    if (dj >= nd) continue;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      if (!tact[u]) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rin = Mfma16<R>::row(g, v);
        const int k = 8 * trt[u] + (rin >> 1), gc = rin & 1;
        const double y = F64 ? (double)C[u][nt][v] : Cd[F64 ? 0 : u][F64 ? 0 : nt][v];
        int coef;
        double val;
        if (!tis_d[u]) {
          if (k >= P1) continue;
          coef = k;
          val = k == 0 ? y : -y * (1.0 / k);
        } else {
          coef = MODE == 0 ? k + 1 : k;
          if (coef >= P1) continue;
          val = y;
        }
        if (MODE == 0) {
          if (it.w >= 0) {
            double *o = reinterpret_cast<double *>(Mp + (int64_t)dj * part_st +
                                                   (int64_t)it.w * 2 * P1);
            o[2 * ((tis_d[u] ? P1 : 0) + coef) + gc] = val;
            if (!tis_d[u] && k == 0) o[2 * P1 + gc] = 0.0;  // D coefficient 0
          } else {
            R *o = reinterpret_cast<R *>(Out + (int64_t)dj * box_st + (tis_d[u] ? d_off : 0) +
                                         (int64_t)b * P1);
            o[2 * coef + gc] = (R)val;
            if (!tis_d[u] && k == 0)
              reinterpret_cast<R *>(Out + (int64_t)dj * box_st + d_off + (int64_t)b * P1)[gc] = R(0);
          }
        } else {
          R *o = reinterpret_cast<R *>(Out + (int64_t)dj * box_st + (tis_d[u] ? d_off : 0) +
                                       (int64_t)b * P1);
          o[2 * coef + gc] = (R)((double)o[2 * coef + gc] + val);
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Stage 6b, P2L (eq. (local) about c_b) for the sources of a box's List 4 far boxes, added to the
// box local that k_m2l wrote. One wavefront per box with such sources (their indices flattened
// on the host). With v = 1/y, coefficient 0 is q log|s y| + d v and coefficient k >= 1 is
// -q v^k / k + d v^(k+1). Lanes: NBLK blocks of 8 consecutive powers (j = 8 kb + i, covering
// j = 0..P1) times 64 / NBLK source groups; a lane forms v^(8 kb) by squaring and the block by a
// multiply chain, accumulates A_j = sum q v^j and B_j = sum d v^j in registers (and the log sum
// on the lanes of block 0), and a fixed shift-down tree (lane_down) adds the groups into lanes
// 0..NBLK-1. Single layer row j = -A_j / j (the log sum at j = 0), double layer row
// j = B_(j+1) (the next block's first power from the neighbouring lane, or for the last block
// one extra power). KIND 4 (S and D of one density) adds the D rows d_off coefficients further.
template <int KIND, int NBLK, typename E>
__global__ void __launch_bounds__(64) k_p2l(
    const int4 *__restrict__ items, const int32_t *__restrict__ src_idx,
    const double2 *__restrict__ bc, const int32_t *__restrict__ blevel,
    const double *__restrict__ level_inv_side, const double *__restrict__ level_log_side,
    const double2 *__restrict__ sxy, const double *__restrict__ sq,
    const double2 *__restrict__ sdip, int P1, E *__restrict__ L, int64_t src_st,
    int64_t box_st, int64_t d_off) {
  critical_path_priority();
  constexpr bool HQ = (KIND & 1) || KIND == 4, HD = (KIND & 2) || KIND == 4;
  constexpr int G = 64 / NBLK;
  const int4 it = items[blockIdx.x];  // box, first source, end of sources
  const int32_t b = it.x;
  const int lane = threadIdx.x;
  const int kb = lane % NBLK, g = lane / NBLK;
  {
    const int64_t jd = blockIdx.y;
    sq += jd * src_st;
    sdip += jd * src_st;
    L += jd * box_st;
  }
  const int lev = blevel[b];
  const double2 c = bc[b];
  const double is = level_inv_side[lev];
  const double logs = level_log_side[lev];
  const double2 *lt = g_log_tab;
  double2 A[8], B[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    A[i] = make_double2(0.0, 0.0);
    B[i] = make_double2(0.0, 0.0);
  }
  double lsum = 0.0;
  double2 Bx = make_double2(0.0, 0.0);  // d v^(8 NBLK), on the last block's lanes
  for (int32_t j = it.y + g; j < it.z; j += G) {
    const int32_t s = src_idx[j];
    const double2 y = make_double2((sxy[s].x - c.x) * is, (sxy[s].y - c.y) * is);
    const double r2 = cnorm2(y);
    const double ir2 = rcp_nr(r2);
    const double2 v = make_double2(y.x * ir2, -y.y * ir2);
    const double q = HQ ? sq[s] : 0.0;
    const double2 d = HD ? cscale(sdip[s], is) : make_double2(0.0, 0.0);
    if (HQ && kb == 0) lsum = fma(q, fma(0.5, log_tab(r2, lt), logs), lsum);
    double2 pw = make_double2(1.0, 0.0);  // v^(8 kb)
    if (NBLK > 1) {
      const double2 v2 = cmul(v, v), v4 = cmul(v2, v2), v8 = cmul(v4, v4);
      if (kb & 1) pw = v8;
      if (NBLK > 2) {
        const double2 v16 = cmul(v8, v8);
        if (kb & 2) pw = (kb & 1) ? cmul(v16, v8) : v16;
        if (NBLK > 4) {
          const double2 v32 = cmul(v16, v16);
          if (kb & 4) pw = cmul(pw, v32);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (HQ) A[i] = caxpy(q, pw, A[i]);
      if (HD) B[i] = cfma(d, pw, B[i]);
      if (i < 7) pw = cmul(pw, v);
    }
    if (HD && kb == NBLK - 1) Bx = cfma(d, cmul(pw, v), Bx);
  }
#pragma unroll
  for (int o = NBLK; o < 64; o <<= 1) {  // group g adds group g + o / NBLK: lanes 0..NBLK-1 sum
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (HQ) {
        A[i].x += lane_down(A[i].x, o);
        A[i].y += lane_down(A[i].y, o);
      }
      if (HD) {
        B[i].x += lane_down(B[i].x, o);
        B[i].y += lane_down(B[i].y, o);
      }
    }
    if (HQ) lsum += lane_down(lsum, o);
    if (HD) {
      Bx.x += lane_down(Bx.x, o);
      Bx.y += lane_down(Bx.y, o);
    }
  }
  // B_(8 kb + 8) from the lane of the next block (lanes 0..NBLK-1 hold the sums)
  double2 Bnext = make_double2(0.0, 0.0);
  if (HD) {
    Bnext.x = __shfl(B[0].x, lane + 1, 64);
    Bnext.y = __shfl(B[0].y, lane + 1, 64);
  }
  if (g != 0) return;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = 8 * kb + i;
    if (k >= P1) break;
    double2 sv = make_double2(0.0, 0.0), dv = make_double2(0.0, 0.0);
    if (HQ) sv = k == 0 ? make_double2(lsum, 0.0) : cscale(A[i], -1.0 / k);
    if (HD) dv = i < 7 ? B[i + 1] : (kb + 1 < NBLK ? Bnext : Bx);
    if (KIND == 4) {
      E *o = L + (int64_t)b * P1 + k;
      *o = from_d2<E>(cadd(to_d2(*o), sv));
      E *od = L + d_off + (int64_t)b * P1 + k;
      *od = from_d2<E>(cadd(to_d2(*od), dv));
    } else {
      // the same expression per kind as above, so each kind rounds as in KIND 4
      E *o = L + (int64_t)b * P1 + k;
      const double2 val = KIND == 1 ? sv : KIND == 2 ? dv : cadd(sv, dv);
      *o = from_d2<E>(cadd(to_d2(*o), val));
    }
  }
}

// ------------------------------------------------------------------------------------------
// Stage 7 as one gather: the local of a box b that owns centers is its own local (M2L + P2L)
// plus every ancestor a's own local shifted to c_b (eq. (l2l) applied across the level gap in
// one step; translations compose, so this equals the level-by-level pass).
//
// With t = (c_b - c_a)/s_a, u = (c_b - c_a)/s_b and alpha the scaled coefficients of a,
//   beta_m = sum_{j>=m} C(j,m) t^(j-m) (s_b/s_a)^m alpha_j = u^-m sum_{j>=m} C(j,m) (t^j alpha_j),
// so the pair-dependent parts are diagonal and the fixed binomial matrix runs on the FP64 matrix
// cores, 8 pairs (16 real columns) per step, as in M2L. |t| < 2^-1/2 and |u| > 2^-1/2 for every
// ancestor: t^j only underflows where its term is negligible and u^-m < 2^(m/2). The products run
// on the matrix cores in the expansion precision (FP32 for mixed-precision expansions), the
// diagonal factors and the sums in FP64.
// The (box, ancestor) pairs of all boxes owning centers are one flat list in box order; a
// wavefront takes a run of whole boxes (about 64 pairs) in batches of 8 consecutive pairs, which
// may span boxes (each matrix-core column is its own pair), fetching the next batch's records and
// coefficients during the current one. Lane m adds row m of each pair in pair order and, when the
// next box starts, writes the finished box's own local plus its sum. Pair record: (ancestor, box),
// ancestor -1 for a box without ancestors of its own local (one empty pair per such box).
template <int RT, typename E>
__global__ void __launch_bounds__(64) k_l2l_gather(
    const int2 *__restrict__ items, const int2 *__restrict__ prs,
    const double4 *__restrict__ anc_tw, const double *__restrict__ binom_t, int P1,
    const E *__restrict__ L, E *__restrict__ Lf, int64_t box_st) {
  critical_path_priority();
  using R = typename Scalar<E>::T;
  using Acc = typename Mfma16<R>::Acc;
  constexpr int KS = 4 * RT;
  constexpr bool F64 = sizeof(R) == 8;
  __shared__ double2 Pt[8][16 * RT];  // one batch's shifted rows, per pair
  __shared__ int32_t Pb[8];
  const int2 it = items[blockIdx.x];  // first pair, end of pairs
  {
    const int64_t jd = blockIdx.y;
    L += jd * box_st;
    Lf += jd * box_st;
  }
  const int lane = threadIdx.x;
  const int g = lane >> 4, c16 = lane & 15;
  const int pr = c16 >> 1, comp = c16 & 1;
  // C(k, i) is zero below the diagonal: row tile rt only needs k-steps ks >= 4 rt
  R A[RT][KS];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int i = 16 * rt + c16, k = 4 * ks + g;
      A[rt][ks] = (ks >= 4 * rt && i < P1 && k < P1) ? (R)binom_t[k * P1 + i] : R(0);
    }
  int2 rec;
  double4 tw;
  double2 lav[KS];
  const double4 unit = make_double4(0.0, 0.0, 1.0, 0.0);  // an idle column: t = 0, 1/u = 1
  auto fetch = [&](int32_t j) {
    const int32_t p = j + pr;
    const bool in = p < it.y;
    const int32_t pc = in ? p : it.y - 1;  // in-bounds loads, then selects
    const int2 rv = prs[pc];
    const double4 tv = anc_tw[pc];
    rec = in ? rv : make_int2(-1, -1);
    const bool pv = rec.x >= 0;
    tw = pv ? tv : unit;
    const E *La = L + (int64_t)(pv ? rec.x : 0) * P1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + g, kc = k < P1 ? k : P1 - 1;  // in-bounds load, then select
      const double2 lv = to_d2(La[kc]);
      lav[ks] = (pv && k < P1) ? lv : make_double2(0.0, 0.0);
    }
  };
  fetch(it.x);
  double2 acc = make_double2(0.0, 0.0);  // lane m: coefficient m of the current box
  double2 own = make_double2(0.0, 0.0);  // lane m: coefficient m of that box's own local
  int32_t cur = -1;
  for (int32_t j0 = it.x; j0 < it.y; j0 += 8) {
    const int nbat = min(8, (int)(it.y - j0));
    const int2 rc = rec;
    const double4 twc = tw;
    double2 lac[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) lac[ks] = lav[ks];
    if (j0 + 8 < it.y) fetch(j0 + 8);  // in flight during this batch
    const double2 t = make_double2(twc.x, twc.y), w = make_double2(twc.z, twc.w);
    // t^k alpha_k for k = g, g + 4, ...
    double2 pw = make_double2(1.0, 0.0);
    for (int e = 0; e < g; ++e) pw = cmul(pw, t);
    const double2 t2 = cmul(t, t), t4 = cmul(t2, t2);
    R Bf[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const double2 v = cmul(pw, lac[ks]);
      Bf[ks] = (R)(comp ? v.y : v.x);
      pw = cmul(pw, t4);
    }
    Acc C[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      C[rt] = Acc{R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int ks = 4 * rt; ks < KS; ++ks) C[rt] = mfma16(A[rt][ks], Bf[ks], C[rt]);
    }
    // row m = 16 rt + g + 4 v of column pair pr: times u^-m, into Pt[pr][m]
    // FP64 rows 16 rt + g + 4 v, FP32 rows 16 rt + 4 g + v: u^-m from u^-(row of v = 0)
    double2 wg = make_double2(1.0, 0.0);
    for (int e = 0; e < (F64 ? g : 4 * g); ++e) wg = cmul(wg, w);
    const double2 w2 = cmul(w, w), w4 = cmul(w2, w2), w8 = cmul(w4, w4), w16 = cmul(w8, w8);
    const double2 wstep = F64 ? w4 : w;
    double2 wr = wg;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      double2 wv = wr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * rt + Mfma16<R>::row(g, v);
        const double y = (double)C[rt][v];
        const double yo = lane_xor1(y);
        if (!comp) Pt[pr][m] = cmul(make_double2(y, yo), wv);
        wv = cmul(wv, wstep);
      }
      wr = cmul(wr, w16);
    }
    if (g == 0 && !comp) Pb[pr] = rc.y;
    __syncthreads();
    if (lane < P1) {
      // the batch's rows and boxes read together, then summed in pair order; a box's own local
      // is loaded when its first pair arrives and added when the box is written
      double2 v[8];
      int32_t bxs[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        v[p] = Pt[p][lane];
        bxs[p] = Pb[p];
      }
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if (p >= nbat) break;
        if (bxs[p] != cur) {
          if (cur >= 0) Lf[(int64_t)cur * P1 + lane] = from_d2<E>(cadd(own, acc));
          acc = make_double2(0.0, 0.0);
          cur = bxs[p];
          own = to_d2(L[(int64_t)cur * P1 + lane]);
        }
        acc = cadd(acc, v[p]);
      }
    }
    __syncthreads();
  }
  if (lane < P1 && cur >= 0) Lf[(int64_t)cur * P1 + lane] = from_d2<E>(cadd(own, acc));
}

// ------------------------------------------------------------------------------------------
// Near-field accumulation of one source into a center's QBX coefficients (P2QBXL), in the
// unscaled offset z = y - c and unscaled dipole d: the sums are taken in z^-m and multiplied by
// r^m once per center (finish), which gives the coefficients in (x - c)/r; the log term
// sum q log|z| needs no log r correction then. Charge part: a_m = sum q z^-m (m >= 1), normalised
// by -1/m in finish.
template <int KIND, int PQ>
struct NearAcc {
  double2 a[PQ + 1];   // KIND 1: a_m = sum q z^-m (m>=1); KIND 2/3: unscaled coefficients
  double logsum;       // sum q log|z|^2
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int m = 0; m <= PQ; ++m) a[m] = make_double2(0.0, 0.0);
    logsum = 0.0;
  }
  __device__ __forceinline__ void add(double2 z, double q, double2 dr, const double2 *lt) {
    const double r2 = cnorm2(z);
    const double ir2 = rcp_nr(r2);
    const double2 inv = make_double2(z.x * ir2, -z.y * ir2);
    if (KIND == 1) {
      logsum = fma(q, log_tab(r2, lt), logsum);
      double2 pw = inv;
#pragma unroll
      for (int m = 1; m <= PQ; ++m) {
        a[m] = caxpy(q, pw, a[m]);
        if (m < PQ) pw = cmul(pw, inv);
      }
    } else if (KIND == 2) {
      double2 pw = cmul(dr, inv);
#pragma unroll
      for (int m = 0; m <= PQ; ++m) {
        a[m] = cadd(a[m], pw);
        if (m < PQ) pw = cmul(pw, inv);
      }
    } else {
      logsum = fma(q, log_tab(r2, lt), logsum);
      const double2 e = cmul(dr, inv);
      a[0] = cadd(a[0], e);
      double2 pw = inv;
#pragma unroll
      for (int m = 1; m <= PQ; ++m) {
        const double2 coef = make_double2(fma(-q, 1.0 / m, e.x), e.y);
        a[m] = cfma(pw, coef, a[m]);
        if (m < PQ) pw = cmul(pw, inv);
      }
    }
  }
  // Add the finished near-field coefficients into alpha, scaled by r^m.
  __device__ __forceinline__ void finish(double2 *alpha, double r) const {
    if (KIND & 1) alpha[0].x += 0.5 * logsum;
    if (KIND != 1) alpha[0] = cadd(alpha[0], a[0]);
    double rp = 1.0;
#pragma unroll
    for (int m = 1; m <= PQ; ++m) {
      rp *= r;
      if (KIND == 1) alpha[m] = caxpy(-(rp * (1.0 / m)), a[m], alpha[m]);
      else alpha[m] = cadd(alpha[m], cscale(a[m], rp));
    }
  }
};

// The same P2QBXL accumulation for DG densities at once: the pair geometry (reciprocal, log,
// powers of 1/z) is formed once and applied to every density's charge and dipole.
template <int KIND, int PQ, int DG>
struct NearAccMD {
  double2 a[DG][PQ + 1];
  double logsum[DG];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int g = 0; g < DG; ++g) {
#pragma unroll
      for (int m = 0; m <= PQ; ++m) a[g][m] = make_double2(0.0, 0.0);
      logsum[g] = 0.0;
    }
  }
  __device__ __forceinline__ void add(double2 z, const double *q, const double2 *dr,
                                      const double2 *lt) {
    const double r2 = cnorm2(z);
    const double ir2 = rcp_nr(r2);
    const double2 inv = make_double2(z.x * ir2, -z.y * ir2);
    if (KIND & 1) {
      const double lr = log_tab(r2, lt);
#pragma unroll
      for (int g = 0; g < DG; ++g) logsum[g] = fma(q[g], lr, logsum[g]);
    }
    if (KIND == 1) {
      double2 pw = inv;
#pragma unroll
      for (int m = 1; m <= PQ; ++m) {
#pragma unroll
        for (int g = 0; g < DG; ++g) a[g][m] = caxpy(q[g], pw, a[g][m]);
        if (m < PQ) pw = cmul(pw, inv);
      }
    } else if (KIND == 2) {
      // the running product dr / z^(m+1) per density, in the single-density order of operations
      double2 pw[DG];
#pragma unroll
      for (int g = 0; g < DG; ++g) pw[g] = cmul(dr[g], inv);
#pragma unroll
      for (int m = 0; m <= PQ; ++m) {
#pragma unroll
        for (int g = 0; g < DG; ++g) {
          a[g][m] = cadd(a[g][m], pw[g]);
          if (m < PQ) pw[g] = cmul(pw[g], inv);
        }
      }
    } else {
      double2 e[DG];
#pragma unroll
      for (int g = 0; g < DG; ++g) {
        e[g] = cmul(dr[g], inv);
        a[g][0] = cadd(a[g][0], e[g]);
      }
      double2 pw = inv;
#pragma unroll
      for (int m = 1; m <= PQ; ++m) {
#pragma unroll
        for (int g = 0; g < DG; ++g) {
          const double2 coef = make_double2(fma(-q[g], 1.0 / m, e[g].x), e[g].y);
          a[g][m] = cfma(pw, coef, a[g][m]);
        }
        if (m < PQ) pw = cmul(pw, inv);
      }
    }
  }
  __device__ __forceinline__ void finish(int g, double2 *alpha, double r) const {
    if (KIND & 1) alpha[0].x += 0.5 * logsum[g];
    if (KIND != 1) alpha[0] = cadd(alpha[0], a[g][0]);
    double rp = 1.0;
#pragma unroll
    for (int m = 1; m <= PQ; ++m) {
      rp *= r;
      if (KIND == 1) alpha[m] = caxpy(-(rp * (1.0 / m)), a[g][m], alpha[m]);
      else alpha[m] = cadd(alpha[m], cscale(a[g][m], rp));
    }
  }
};

// QBX expansion of a center evaluated at its targets (QBXL2P), written to the target slots.
// With target normals (tnrm, the normal derivative S' of GQ_SP): u = Re F with F analytic, so
// n . grad u = Re(F'(x) nu), nu = n_x + i n_y; the scaled expansion sum_m a_m z^m, z = (x - c)/r,
// has F' = (1/r) sum_{m>=1} m a_m z^(m-1), formed by the same Horner.
template <int PQ>
__device__ __forceinline__ void eval_targets(int32_t c, double2 cc, double r, const double2 *alpha,
                                             const int32_t *__restrict__ c2t_start,
                                             const int32_t *__restrict__ c2t_slot,
                                             const double2 *__restrict__ txy, double *__restrict__ tv,
                                             const double2 *__restrict__ tnrm) {
  const double ir = 1.0 / r;
  for (int32_t g = c2t_start[c]; g < c2t_start[c + 1]; ++g) {
    const int32_t slot = c2t_slot[g];
    const double2 x = txy[slot >> 1];
    const double2 z = make_double2((x.x - cc.x) * ir, (x.y - cc.y) * ir);
    if (tnrm) {
      double2 s = cscale(alpha[PQ], (double)PQ);
#pragma unroll
      for (int m = PQ - 1; m >= 1; --m) s = cfma(s, z, cscale(alpha[m], (double)m));
      const double2 d = cmul(s, tnrm[slot >> 1]);
      tv[slot] = -kInv2Pi * ir * d.x;
      continue;
    }
    double2 s = alpha[PQ];
#pragma unroll
    for (int m = PQ - 1; m >= 0; --m) s = cfma(s, z, alpha[m]);
    tv[slot] = -kInv2Pi * s.x;
  }
}

// ------------------------------------------------------------------------------------------
// Stages 3, 5a, 6a: P2QBXL from the direct sources (List 1, List 3 close, List 4 close) of a box
// into its centers. One wavefront per work item (box, source chunk, block of n_cl centers): lane
// = (center, slice), n_sl slices per center (any n_sl <= 64, n_cl n_sl <= 64 lanes busy) striding
// over the chunk's sources, then a fixed-order shuffle reduction over the slices (slice_add).
// The result row holds the scaled coefficients.
constexpr int kNearBatch = 128;  // sources staged in LDS per step (two per lane)
static_assert(kNearBatch == 128, "k_near_sd stages two sources per lane");

// One step of the slice reduction over n_sl slices of a center (lanes cl n_sl + sl): at step o
// (1, 2, 4, ...) slice sl adds slice sl + o when sl is a multiple of 2 o and sl + o < n_sl, so
// after ceil(log2 n_sl) steps slice 0 holds the sum, in a fixed order. Every lane joins the
// shuffle.
__device__ __forceinline__ void slice_add(double &v, int o, bool take) {
  const double t = __shfl_down(v, o, 64);
  if (take) v += t;
}

template <int KIND, int PQ>
__global__ void __launch_bounds__(64) k_near(
    int32_t n_items, const int4 *__restrict__ items, const int32_t *__restrict__ near_src,
    const double2 *__restrict__ cxy, const double *__restrict__ cr,
    const double2 *__restrict__ sxy, const double *__restrict__ sq,
    const double2 *__restrict__ sdip, double2 *__restrict__ anear, int rs, int64_t src_st,
    int64_t row_st) {
  __shared__ double2 t_xy[kNearBatch];
  __shared__ double t_q[(KIND & 1) ? kNearBatch : 1];
  __shared__ double2 t_d[(KIND & 2) ? kNearBatch : 1];
  const int32_t w = (int32_t)blockIdx.x;  // one wavefront per work-group and per item
  const int lane = threadIdx.x;
  {
    const int64_t jd = blockIdx.y;
    sq += jd * src_st;
    sdip += jd * src_st;
    anear += jd * row_st;
  }
  const int4 i0 = items[2 * w], i1 = items[2 * w + 1];
  const int32_t off = i0.x, len = i0.y, ctr_first = i0.z, row_first = i0.w;
  const int n_ctr = i1.x, nsl = i1.y;  // centers, slices per center
  const int cl = lane / nsl;
  const int sl = lane - cl * nsl;
  const bool active = cl < n_ctr;
  const int32_t c = ctr_first + (active ? cl : 0);
  const double2 cc = cxy[c];
  const double r = cr[c];
  const double2 *lt = g_log_tab;
  NearAcc<KIND, PQ> acc;
  acc.zero();
  for (int32_t base = 0; base < len; base += kNearBatch) {
    const int nb = min(kNearBatch, (int)(len - base));
    __syncthreads();
#pragma unroll
    for (int j = lane; j < kNearBatch; j += 64) {
      if (j < nb) {
        const int32_t s = near_src[off + base + j];
        t_xy[j] = sxy[s];
        if (KIND & 1) t_q[j] = sq[s];
        if (KIND & 2) t_d[j] = sdip[s];
      }
    }
    __syncthreads();
    if (active) {
      for (int j = sl; j < nb; j += nsl) {
        const double2 z = make_double2(t_xy[j].x - cc.x, t_xy[j].y - cc.y);
        acc.add(z, (KIND & 1) ? t_q[j] : 0.0, (KIND & 2) ? t_d[j] : make_double2(0.0, 0.0), lt);
      }
    }
  }
  for (int o = 1; o < nsl; o <<= 1) {
    const bool take = (sl & (2 * o - 1)) == 0 && sl + o < nsl;
#pragma unroll
    for (int m = 0; m <= PQ; ++m) {
      slice_add(acc.a[m].x, o, take);
      slice_add(acc.a[m].y, o, take);
    }
    if (KIND & 1) slice_add(acc.logsum, o, take);
  }
  if (active && sl == 0) {
    double2 alpha[PQ + 1];
#pragma unroll
    for (int m = 0; m <= PQ; ++m) alpha[m] = make_double2(0.0, 0.0);
    acc.finish(alpha, r);
    double2 *row = anear + (int64_t)(row_first + cl) * rs;
#pragma unroll
    for (int m = 0; m <= PQ; ++m) row[m] = alpha[m];
  }
}

// S and D of one density in one pass (the pair geometry, the log and the powers of 1/z formed
// once): the single-layer sums as in NearAcc<1>, and the double-layer sums d z^-(m+1) taken from
// the same powers, d z^-(m+1) = d (1/z)^(m+1) (NearAcc<2> runs its own product chain, so these D
// rows agree with a GQ_D evaluation to rounding, not bitwise). Rows: S into the first slot, D into
// the slot d_slot rows of row_st further.
template <int PQ>
struct NearAccSD {
  double2 as[PQ + 1], ad[PQ + 1];
  double logsum;
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int m = 0; m <= PQ; ++m) {
      as[m] = make_double2(0.0, 0.0);
      ad[m] = make_double2(0.0, 0.0);
    }
    logsum = 0.0;
  }
  __device__ __forceinline__ void add(double2 z, double q, double2 dr, const double2 *lt) {
    const double r2 = cnorm2(z);
    const double ir2 = rcp_nr(r2);
    const double2 inv = make_double2(z.x * ir2, -z.y * ir2);
    logsum = fma(q, log_tab(r2, lt), logsum);
    double2 pw = inv;  // z^-(m+1) in step m: D coefficient m, S coefficient m + 1
#pragma unroll
    for (int m = 0; m <= PQ; ++m) {
      ad[m] = cfma(dr, pw, ad[m]);
      if (m < PQ) {
        as[m + 1] = caxpy(q, pw, as[m + 1]);
        pw = cmul(pw, inv);
      }
    }
  }
};

// Up to order 12 the accumulators fit three waves per SIMD (168 registers, no spill), which
// measured 10 % faster than two; higher orders keep two.
template <int PQ>
__global__ void __launch_bounds__(64, PQ <= 12 ? 3 : 2) k_near_sd(
    int32_t n_items, const int4 *__restrict__ items, const int32_t *__restrict__ near_src,
    const double2 *__restrict__ cxy, const double *__restrict__ cr,
    const double2 *__restrict__ sxy, const double *__restrict__ sq,
    const double2 *__restrict__ sdip, double2 *__restrict__ anear, int rs, int64_t src_st,
    int64_t row_st, int64_t d_slot) {
  __shared__ double2 t_xy[kNearBatch];
  __shared__ double t_q[kNearBatch];
  __shared__ double2 t_d[kNearBatch];
  const int32_t w = (int32_t)blockIdx.x;
  const int lane = threadIdx.x;
  {
    const int64_t jd = blockIdx.y;
    sq += jd * src_st;
    sdip += jd * src_st;
    anear += jd * row_st;
  }
  const int4 i0 = items[2 * w], i1 = items[2 * w + 1];
  const int32_t off = i0.x, len = i0.y, ctr_first = i0.z, row_first = i0.w;
  const int n_ctr = i1.x, nsl = i1.y;  // centers, slices per center
  const int cl = lane / nsl;
  const int sl = lane - cl * nsl;
  const bool active = cl < n_ctr;
  const int32_t c = ctr_first + (active ? cl : 0);
  const double2 cc = cxy[c];
  const double r = cr[c];
  const double2 *lt = g_log_tab;
  NearAccSD<PQ> acc;
  acc.zero();
  // the indices of a batch's sources are fetched during the previous batch's pairs (clamped to
  // the item's last source, extra values unused)
  const int32_t last = off + len - 1;
  auto idx = [&](int32_t k) { return near_src[k < last ? k : last]; };
  int32_t nx0 = idx(off + lane), nx1 = idx(off + lane + 64);
  for (int32_t base = 0; base < len; base += kNearBatch) {
    const int nb = min(kNearBatch, (int)(len - base));
    const int32_t s0 = nx0, s1 = nx1;
    __syncthreads();
    if (lane < nb) {
      t_xy[lane] = sxy[s0];
      t_q[lane] = sq[s0];
      t_d[lane] = sdip[s0];
    }
    if (lane + 64 < nb) {
      t_xy[lane + 64] = sxy[s1];
      t_q[lane + 64] = sq[s1];
      t_d[lane + 64] = sdip[s1];
    }
    nx0 = idx(off + base + kNearBatch + lane);
    nx1 = idx(off + base + kNearBatch + lane + 64);
    __syncthreads();
    if (active) {
      for (int j = sl; j < nb; j += nsl) {
        const double2 z = make_double2(t_xy[j].x - cc.x, t_xy[j].y - cc.y);
        acc.add(z, t_q[j], t_d[j], lt);
      }
    }
  }
  for (int o = 1; o < nsl; o <<= 1) {
    const bool take = (sl & (2 * o - 1)) == 0 && sl + o < nsl;
#pragma unroll
    for (int m = 0; m <= PQ; ++m) {
      slice_add(acc.as[m].x, o, take);
      slice_add(acc.as[m].y, o, take);
      slice_add(acc.ad[m].x, o, take);
      slice_add(acc.ad[m].y, o, take);
    }
    slice_add(acc.logsum, o, take);
  }
  if (active && sl == 0) {
    // the finish of NearAcc<1> and NearAcc<2> written out for both rows
    double2 *row = anear + (int64_t)(row_first + cl) * rs;
    double2 *rowd = row + d_slot * row_st;
    row[0] = make_double2(0.0 + 0.5 * acc.logsum, 0.0);
    rowd[0] = acc.ad[0];
    double rp = 1.0;
#pragma unroll
    for (int m = 1; m <= PQ; ++m) {
      rp *= r;
      row[m] = caxpy(-(rp * (1.0 / m)), acc.as[m], make_double2(0.0, 0.0));
      rowd[m] = cscale(acc.ad[m], rp);
    }
  }
}

// The direct part of one density evaluated at the centers' own targets (KIND 4: S and D, two
// values; 1, 2, 3: S, D or S - D, one value), for geometries in which every center serves at
// most one target (a target on the curve takes one center on each side). The
// direct part of a center's expansion is then needed at one point only, x, and is summed there:
// for a source y of charge q and dipole strength d, with z = y - c and rho = (x - c)/z,
//   S: q (log|z| - Re sum_{k=1..p} rho^k / k),   D: Re((d / z) sum_{k=0..p} rho^k),
// the truncated series of the coefficient rows of k_near / k_near_sd, summed in another order. Both
// polynomials have real coefficients, so each is evaluated at the complex point rho by the
// second-order recurrence for real polynomials at a complex argument (Knuth, The Art of
// Computer Programming, vol. 2, Sec. 4.6.4): with r1 = 2 Re rho and s = |rho|^2,
// b_k = a_k + r1 b_(k+1) - s b_(k+2) downwards from b_p = a_p, and P(rho) = b_1 rho + a_0 - s b_2;
// two fused multiply-adds per order and polynomial, against a complex product and a complex
// accumulation per order for the coefficients. Each (center, chunk) row's value goes to the dense
// value array nval (S; D d_off entries further, one slot on), which the center stage adds to the
// constant term of the center's expansion.
template <int KIND, int PQ>
__global__ void __launch_bounds__(64) k_near_sd_t(
    int32_t n_items, const int4 *__restrict__ items, const int32_t *__restrict__ near_src,
    const double2 *__restrict__ cxy, const double2 *__restrict__ sxy,
    const double *__restrict__ sq, const double2 *__restrict__ sdip,
    const int32_t *__restrict__ c2t_start, const int32_t *__restrict__ c2t_slot,
    const double2 *__restrict__ txy, double *__restrict__ nval, int64_t d_off) {
  static_assert(PQ >= 2, "the recurrences start at b_p and b_(p-1)");
  constexpr bool HS = KIND != 2, HD = KIND != 1;  // single / double layer terms
  __shared__ double2 t_xy[kNearBatch];
  __shared__ double t_q[HS ? kNearBatch : 1];
  __shared__ double2 t_d[HD ? kNearBatch : 1];
  const int32_t w = (int32_t)blockIdx.x;
  const int lane = threadIdx.x;
  const int4 i0 = items[2 * w], i1 = items[2 * w + 1];
  const int32_t off = i0.x, len = i0.y, ctr_first = i0.z, row_first = i0.w;
  const int n_ctr = i1.x, nsl = i1.y;  // centers, slices per center
  const int cl = lane / nsl;
  const int sl = lane - cl * nsl;
  const bool active = cl < n_ctr;
  const int32_t c = ctr_first + (active ? cl : 0);
  const double2 cc = cxy[c];
  // x - c for the center's target (zero for a center without one: rho = 0, value unused)
  double2 tz = make_double2(0.0, 0.0);
  {
    const int32_t g = c2t_start[c];
    if (c2t_start[c + 1] > g) {
      const double2 x = txy[c2t_slot[g] >> 1];
      tz = make_double2(x.x - cc.x, x.y - cc.y);
    }
  }
  const double tz2 = cnorm2(tz);
  const double2 *lt = g_log_tab;
  double logsum = 0.0, fsum = 0.0, dsum = 0.0;
  const int32_t last = off + len - 1;
  auto idx = [&](int32_t k) { return near_src[k < last ? k : last]; };
  int32_t nx0 = idx(off + lane), nx1 = idx(off + lane + 64);
  for (int32_t base = 0; base < len; base += kNearBatch) {
    const int nb = min(kNearBatch, (int)(len - base));
    const int32_t s0 = nx0, s1 = nx1;
    __syncthreads();
    if (lane < nb) {
      t_xy[lane] = sxy[s0];
      if (HS) t_q[lane] = sq[s0];
      if (HD) t_d[lane] = sdip[s0];
    }
    if (lane + 64 < nb) {
      t_xy[lane + 64] = sxy[s1];
      if (HS) t_q[lane + 64] = sq[s1];
      if (HD) t_d[lane + 64] = sdip[s1];
    }
    nx0 = idx(off + base + kNearBatch + lane);
    nx1 = idx(off + base + kNearBatch + lane + 64);
    __syncthreads();
    if (active) {
      for (int j = sl; j < nb; j += nsl) {
        const double2 y = t_xy[j];
        const double dx = y.x - cc.x, dy = y.y - cc.y;
        const double n2 = fma(dx, dx, dy * dy);
        const double ir2 = rcp_nr(n2);
        // rho = (x - c) conj(z) / |z|^2
        const double ux = fma(tz.x, dx, tz.y * dy) * ir2;
        const double uy = fma(tz.y, dx, -(tz.x * dy)) * ir2;
        const double r1 = 2.0 * ux, s = tz2 * ir2;
        double b2 = 1.0 / PQ, b1 = fma(r1, b2, 1.0 / (PQ - 1));  // S: a_k = 1/k, a_0 = 0
        double e2 = 1.0, e1 = 1.0 + r1;                           // D: a_k = 1
#pragma unroll
        for (int k = PQ - 2; k >= 1; --k) {
          if (HS) {
            const double b0 = fma(r1, b1, fma(-s, b2, 1.0 / k));
            b2 = b1;
            b1 = b0;
          }
          if (HD) {
            const double e0 = fma(r1, e1, fma(-s, e2, 1.0));
            e2 = e1;
            e1 = e0;
          }
        }
        if (HS) {
          const double q = t_q[j];
          logsum = fma(q, log_tab(n2, lt), logsum);
          fsum = fma(q, fma(b1, ux, -(s * b2)), fsum);
        }
        if (HD) {
          const double gx = fma(e1, ux, fma(-s, e2, 1.0)), gy = e1 * uy;
          // Re(d conj(z) g) / |z|^2
          const double hx = fma(dx, gx, dy * gy), hy = fma(dx, gy, -(dy * gx));
          const double2 dr = t_d[j];
          dsum = fma(ir2, fma(dr.x, hx, -(dr.y * hy)), dsum);
        }
      }
    }
  }
  // S and D of one density: two values (D d_off further); one kind, or S - D (the dipoles carry
  // the sign): one value
  double vs = fma(0.5, logsum, -fsum);
  if (KIND != 4) vs += dsum;
  for (int o = 1; o < nsl; o <<= 1) {
    const bool take = (sl & (2 * o - 1)) == 0 && sl + o < nsl;
    slice_add(vs, o, take);
    if (KIND == 4) slice_add(dsum, o, take);
  }
  if (active && sl == 0) {
    nval[row_first + cl] = vs;
    if (KIND == 4) nval[d_off + row_first + cl] = dsum;
  }
}

// Stages 3, 5a, 6a for S and D of many densities (GQ_S_AND_D, a batch of nd densities) on the
// matrix cores. For a center c and a source y of strength q^(j) = w mu^(j) in density j, the
// charge part adds q z^-m (m >= 1) and q log|z|^2, the dipole part q n z^-(m+1) (the dipole is
// the charge times the normal for S and D of one density), z = y - c. Over the sources of a chunk
// and the densities this is one real GEMM per center: rows are the real and imaginary parts of
// z^-m (S, m = 1..PQ, then log|z|^2) and of n z^-(m+1) (D, m = 0..PQ), the k dimension the
// sources, the columns the densities. A work-group of four wavefronts takes up to four centers of
// a box (one per wavefront) and one chunk of its direct sources; the chunk's positions, normals
// and the strengths of 16 NT densities are staged in LDS 64 sources at a time (the next batch's
// loads in flight during the current one), and each lane forms the pair's powers for its rows:
// row 16 rt + i of either block is order 8 rt + i/2 + 1, so one chain of products serves both.
// The finished rows are the scaled coefficients of k_near / k_near_sd (times r^m, S by -1/m),
// written to the same (center, chunk) rows: S of density j in slot j, D in slot d_slot + j.
template <int PQ, int NT>
__global__ void __launch_bounds__(256, 2) k_near_mfma(
    int32_t n_items, const int4 *__restrict__ items, const int32_t *__restrict__ near_src,
    const double2 *__restrict__ cxy, const double *__restrict__ cr,
    const double2 *__restrict__ sxy, const double2 *__restrict__ snrm,
    const double *__restrict__ sq, double2 *__restrict__ anear, int rs, int64_t src_st,
    int64_t row_st, int nd, int64_t d_slot) {
  constexpr int RTS = (2 * PQ + 1 + 15) / 16, RTD = (2 * PQ + 2 + 15) / 16;
  constexpr int RT = RTS > RTD ? RTS : RTD;
  constexpr int LI = (2 * PQ) % 16, LRT = (2 * PQ) / 16;  // lane row and tile of the log row
  constexpr int NDB = 16 * NT;                            // densities per work-group
  constexpr int SB = 32;                                  // sources staged per batch
  // LDS strides chosen so that the k-step reads (4 sources x 16 columns) hit distinct banks
  constexpr int QST = NDB + 1;  // strengths: source-major rows of the batch's densities
  constexpr int PST = 9;        // powers: 8 per source and one pad
  __shared__ double t_q[SB][QST];
  __shared__ double2 t_y[SB], t_n[SB];
  __shared__ double2 t_log[kLogTab];
  __shared__ double2 t_pw[4][SB][PST];  // per wavefront (center): z^-1 .. z^-8 of the batch
  __shared__ double t_lg[4][SB];      // and log|z|^2
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  (void)n_items;
  const int4 i0 = items[2 * blockIdx.x], i1 = items[2 * blockIdx.x + 1];
  const int32_t off = i0.x, len = i0.y, ctr_first = i0.z, row_first = i0.w;
  const int n_ctr = i1.x;
  const int d0 = blockIdx.y * NDB;
  const bool active = wv < n_ctr;
  const int32_t c = ctr_first + (active ? wv : 0);
  const double2 cc = cxy[c];
  const double rad = cr[c];
  if (tid < kLogTab) t_log[tid] = g_log_tab[tid];  // the log table from LDS in the loop
  const double2 *lt = t_log;
  const int i = lane & 15, kk = lane >> 4, h = i >> 1, comp = i & 1;
  // staging: thread (source tid % SB, density rows tid / SB + 8 q) of an SB-source batch
  const int ss = tid % SB, sd = tid / SB;
  double rq[NDB / 8];
  double2 ry = make_double2(0.0, 0.0), rn = make_double2(0.0, 0.0);
  // a batch's source indices are read one batch ahead of its strengths, and the strengths are
  // kept raw until they are written to LDS (a select at the load would wait for it at once)
  auto index = [&](int32_t base) {
    const int nb = min(SB, (int)(len - base));
    return near_src[off + base + (ss < nb ? ss : 0)];
  };
  auto load = [&](int32_t src) {
    if (sd == 0) {
      ry = sxy[src];
      rn = snrm[src];
    }
#pragma unroll
    for (int q = 0; q < NDB / 8; ++q) {
      const int dj = d0 + sd + 8 * q;
      rq[q] = sq[(int64_t)(dj < nd ? dj : 0) * src_st + src];
    }
  };
  gq_d4 CS[RTS][NT], CD[RTD][NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
    for (int rt = 0; rt < RTS; ++rt) CS[rt][nt] = gq_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rt = 0; rt < RTD; ++rt) CD[rt][nt] = gq_d4{0.0, 0.0, 0.0, 0.0};
  }
  load(index(0));
  int32_t snx = SB < len ? index(SB) : 0;
  for (int32_t base = 0; base < len; base += SB) {
    const int nb = min(SB, (int)(len - base));
    __syncthreads();  // the previous batch is no longer read
    if (sd == 0) {
      t_y[ss] = ry;
      t_n[ss] = rn;
    }
#pragma unroll
    for (int q = 0; q < NDB / 8; ++q)
      t_q[ss][sd + 8 * q] = (ss < nb && d0 + sd + 8 * q < nd) ? rq[q] : 0.0;
    __syncthreads();
    if (base + SB < len) {  // in flight during this batch
      load(snx);
      if (base + 2 * SB < len) snx = index(base + 2 * SB);
    }
    if (active) {
      // the pair geometry of the batch, once per (center, source): lane l takes source l % 32
      // and powers 1..4 (l < 32, with the log) or 5..8 of 1/z; zeros past the batch
      const int sa = lane & 31, half = lane >> 5;
      const bool va = sa < nb;
      const double2 ya = t_y[sa];
      const double2 za = make_double2(ya.x - cc.x, ya.y - cc.y);
      const double r2 = va ? cnorm2(za) : 1.0;
      const double ir2 = rcp_nr(r2);
      const double2 inv = make_double2(za.x * ir2, -za.y * ir2);
      const double2 i2 = cmul(inv, inv), i3 = cmul(i2, inv), i4 = cmul(i2, i2);
      const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
      const double2 b4 = half ? i4 : one;  // z^-(4 half)
      double2 *pw = &t_pw[wv][sa][4 * half];
      pw[0] = va ? cmul(b4, inv) : zero;
      pw[1] = va ? cmul(b4, i2) : zero;
      pw[2] = va ? cmul(b4, i3) : zero;
      pw[3] = va ? cmul(b4, i4) : zero;
      if (half == 0) t_lg[wv][sa] = va ? log_tab(r2, lt) : 0.0;
    }
    __syncthreads();
    if (!active) continue;
    const int nks = (nb + 3) >> 2;
    for (int ks = 0; ks < nks; ++ks) {
      const int sl = 4 * ks + kk;
      const double2 nv = t_n[sl];
      double2 pwr = t_pw[wv][sl][h];         // z^-(h + 1)
      const double2 i8 = t_pw[wv][sl][7];   // z^-8
      const double lg = t_lg[wv][sl];
      double aS[RTS], aD[RTD];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int r = 16 * rt + i;
        if (rt < RTS) {
          double a = comp ? pwr.y : pwr.x;
          if (r >= 2 * PQ) a = (rt == LRT && i == LI) ? lg : 0.0;
          aS[rt < RTS ? rt : 0] = a;
        }
        if (rt < RTD) {
          const double2 w = cmul(nv, pwr);
          aD[rt < RTD ? rt : 0] = r < 2 * PQ + 2 ? (comp ? w.y : w.x) : 0.0;
        }
        if (rt + 1 < RT) pwr = cmul(pwr, i8);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const double b = t_q[sl][16 * nt + i];  // B[kk][j]: column j = lane & 15 = i
#pragma unroll
        for (int rt = 0; rt < RTS; ++rt) CS[rt][nt] = mfma16(aS[rt], b, CS[rt][nt]);
#pragma unroll
        for (int rt = 0; rt < RTD; ++rt) CD[rt][nt] = mfma16(aD[rt], b, CD[rt][nt]);
      }
    }
  }
  if (!active) return;
  // lane (column j = lane & 15, group g = lane >> 4) holds rows 16 rt + g + 4 v
  const int g = kk, j = i;
  const int64_t row = row_first + wv;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int dj = d0 + 16 * nt + j;
    if (dj >= nd) continue;
    double *os = reinterpret_cast<double *>(anear + (int64_t)dj * row_st + row * rs);
    double *od = reinterpret_cast<double *>(anear + (d_slot + dj) * row_st + row * rs);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * rt + g + 4 * v;
        if (rt < RTS) {
          const double y = CS[rt < RTS ? rt : 0][nt][v];
          if (r < 2 * PQ) {
            const int m = r / 2 + 1;
            double rp = rad;
            for (int q = 1; q < m; ++q) rp *= rad;
            os[2 * m + (r & 1)] = -(rp * (1.0 / m)) * y;
          } else if (r == 2 * PQ) {
            os[0] = 0.5 * y;
          } else if (r == 2 * PQ + 1) {
            os[1] = 0.0;
          }
        }
        if (rt < RTD && r < 2 * PQ + 2) {
          const double y = CD[rt < RTD ? rt : 0][nt][v];
          const int m = r / 2;
          double rp = 1.0;
          for (int q = 0; q < m; ++q) rp *= rad;
          od[r] = rp * y;
        }
      }
  }
}

// S and D of a batch of densities at the centers' own targets (every center serving at most one
// target) on the matrix cores. At a center's target x the direct part of its expansion is, for
// density j, sum_y q_y^(j) A(c, y) (S) and sum_y q_y^(j) B(c, y) (D), the dipole being the charge
// times the normal: with z = y - c and rho = (x - c)/z,
//   A = log|z| - Re sum_{k=1..p} rho^k / k,   B = Re(n conj(z) sum_{k=0..p} rho^k) / |z|^2,
// pair weights that do not depend on the density (the polynomials by the recurrence of
// k_near_sd_t). Over a chunk of a box's sources this is one real GEMM per block of 16 centers:
// rows the centers, k the sources, columns the densities, S and D two accumulators. A work-group
// of four wavefronts takes one (chunk, block of up to 16 centers) item and 16 NT densities; the
// chunk is staged 64 sources at a time (positions, normals and the strengths of the densities,
// the next batch's loads in flight during the current one), each wavefront takes 16 of them
// (four k-steps, lane (row i, k kk) forming the weights of one pair), and the four partial
// products are summed through LDS at the end. Values go to the dense value array as in
// k_near_sd_t: S of density j in slot j, D in slot d_slot + j.
template <int PQ, int NT>
__global__ void __launch_bounds__(256, 2) k_near_val_mfma(
    const int4 *__restrict__ items, const int32_t *__restrict__ near_src,
    const double2 *__restrict__ cxy, const double2 *__restrict__ sxy,
    const double2 *__restrict__ snrm, const double *__restrict__ sq,
    const int32_t *__restrict__ c2t_start, const int32_t *__restrict__ c2t_slot,
    const double2 *__restrict__ txy, double *__restrict__ nval, int64_t src_st, int64_t nv_st,
    int nd, int64_t d_slot) {
  static_assert(PQ >= 2, "the recurrences start at b_p and b_(p-1)");
  constexpr int NDB = 16 * NT;  // densities per work-group
  constexpr int SB = 64;        // sources staged per batch, 16 per wavefront
  constexpr int QST = NDB + 1;  // strengths: source-major rows of the batch's densities (padded)
  constexpr int NQ = NDB / 4;   // strengths staged per thread and batch
  constexpr int RED = 3 * 64 * 4 * NT;  // one accumulator set of waves 1..3 (doubles)
  static_assert(RED <= SB * QST, "the wave reduction reuses the strength buffer");
  __shared__ double t_q[SB * QST];
  __shared__ double2 t_y[SB], t_n[SB];
  __shared__ double2 t_log[kLogTab];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int4 i0 = items[2 * blockIdx.x], i1 = items[2 * blockIdx.x + 1];
  const int32_t off = i0.x, len = i0.y, ctr_first = i0.z, row_first = i0.w;
  const int n_ctr = i1.x;
  const int d0 = blockIdx.y * NDB;
  if (tid < kLogTab) t_log[tid] = g_log_tab[tid];
  const int i = lane & 15, kk = lane >> 4;
  // the A-operand row of this lane: center i of the block and the offset of its target
  const bool row_on = i < n_ctr;
  const int32_t c = ctr_first + (row_on ? i : 0);
  const double2 cc = cxy[c];
  double2 tz = make_double2(0.0, 0.0);
  {
    const int32_t g = c2t_start[c];
    if (c2t_start[c + 1] > g) {
      const double2 x = txy[c2t_slot[g] >> 1];
      tz = make_double2(x.x - cc.x, x.y - cc.y);
    }
  }
  const double tz2 = cnorm2(tz);
  // staging: thread (source tid % SB, densities tid / SB + 4 q) of a batch
  const int ss = tid % SB, sd = tid / SB;
  double rq[NQ];
  double2 ry = make_double2(0.0, 0.0), rn = make_double2(0.0, 0.0);
  auto index = [&](int32_t base) {
    const int nb = min(SB, (int)(len - base));
    return near_src[off + base + (ss < nb ? ss : 0)];
  };
  auto load = [&](int32_t src) {
    if (sd == 0) {
      ry = sxy[src];
      rn = snrm[src];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int dj = d0 + sd + 4 * q;
      rq[q] = sq[(int64_t)(dj < nd ? dj : 0) * src_st + src];
    }
  };
  gq_d4 CS[NT], CD[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    CS[nt] = gq_d4{0.0, 0.0, 0.0, 0.0};
    CD[nt] = gq_d4{0.0, 0.0, 0.0, 0.0};
  }
  load(index(0));
  int32_t snx = SB < len ? index(SB) : 0;
  for (int32_t base = 0; base < len; base += SB) {
    const int nb = min(SB, (int)(len - base));
    __syncthreads();  // the previous batch is no longer read
    if (sd == 0) {
      t_y[ss] = ry;
      t_n[ss] = rn;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      t_q[ss * QST + sd + 4 * q] = (ss < nb && d0 + sd + 4 * q < nd) ? rq[q] : 0.0;
    __syncthreads();
    if (base + SB < len) {  // in flight during this batch
      load(snx);
      if (base + 2 * SB < len) snx = index(base + 2 * SB);
    }
#pragma unroll 1
    for (int ks = 0; ks < 4; ++ks) {
      const int sl = 16 * wv + 4 * ks + kk;
      if (16 * wv + 4 * ks >= nb) break;  // uniform over the wavefront
      const double2 y = t_y[sl], nv = t_n[sl];
      const double dx = y.x - cc.x, dy = y.y - cc.y;
      const bool on = row_on && sl < nb;
      const double n2 = on ? fma(dx, dx, dy * dy) : 1.0;
      const double ir2 = rcp_nr(n2);
      const double lg = log_tab(n2, t_log);
      const double ux = fma(tz.x, dx, tz.y * dy) * ir2;
      const double uy = fma(tz.y, dx, -(tz.x * dy)) * ir2;
      const double r1 = 2.0 * ux, s = tz2 * ir2;
      double b2 = 1.0 / PQ, b1 = fma(r1, b2, 1.0 / (PQ - 1));
      double e2 = 1.0, e1 = 1.0 + r1;
#pragma unroll
      for (int k = PQ - 2; k >= 1; --k) {
        const double b0 = fma(r1, b1, fma(-s, b2, 1.0 / k));
        const double e0 = fma(r1, e1, fma(-s, e2, 1.0));
        b2 = b1;
        b1 = b0;
        e2 = e1;
        e1 = e0;
      }
      const double gx = fma(e1, ux, fma(-s, e2, 1.0)), gy = e1 * uy;
      const double hx = fma(dx, gx, dy * gy), hy = fma(dx, gy, -(dy * gx));
      const double aS = on ? fma(0.5, lg, -fma(b1, ux, -(s * b2))) : 0.0;
      const double aD = on ? ir2 * fma(nv.x, hx, -(nv.y * hy)) : 0.0;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const double b = t_q[sl * QST + 16 * nt + i];  // B[kk][j]: column j = lane & 15 = i
        CS[nt] = mfma16(aS, b, CS[nt]);
        CD[nt] = mfma16(aD, b, CD[nt]);
      }
    }
  }
  // sum the four wavefronts' products (S, then D) in wavefront 0 through the strength buffer
  double *red = t_q;
  auto reduce = [&](gq_d4 (&C)[NT]) {
    __syncthreads();
    if (wv > 0) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(((wv - 1) * NT + nt) * 4 + v) * 64 + lane] = C[nt][v];
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) C[nt][v] += red[((w * NT + nt) * 4 + v) * 64 + lane];
    }
  };
  reduce(CS);
  reduce(CD);
  if (wv != 0) return;
  // lane (column j = lane & 15, group g = lane >> 4) holds rows (centers) g + 4 v
  const int g = kk, j = i;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int dj = d0 + 16 * nt + j;
    if (dj >= nd) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ci = g + 4 * v;
      if (ci >= n_ctr) continue;
      const int64_t row = row_first + ci;
      nval[(int64_t)dj * nv_st + row] = CS[nt][v];
      nval[(d_slot + dj) * nv_st + row] = CD[nt][v];
    }
  }
}

// k_near for a block of DG densities per work-group (grid.y = density blocks): same items and
// lanes, the sources' charges and dipoles of the DG densities staged together, one pair geometry
// for all of them. Densities past n_dens (a last partial block) get zero strengths and no rows.
template <int KIND, int PQ, int DG>
__global__ void __launch_bounds__(64) k_near_md(
    int32_t n_items, const int4 *__restrict__ items, const int32_t *__restrict__ near_src,
    const double2 *__restrict__ cxy, const double *__restrict__ cr,
    const double2 *__restrict__ sxy, const double *__restrict__ sq,
    const double2 *__restrict__ sdip, double2 *__restrict__ anear, int rs, int64_t src_st,
    int64_t row_st, int n_dens) {
  __shared__ double2 t_xy[kNearBatch];
  __shared__ double t_q[(KIND & 1) ? DG : 1][(KIND & 1) ? kNearBatch : 1];
  __shared__ double2 t_d[(KIND & 2) ? DG : 1][(KIND & 2) ? kNearBatch : 1];
  const int32_t w = (int32_t)blockIdx.x;
  const int lane = threadIdx.x;
  const int jd0 = (int)blockIdx.y * DG;
  const int ng = min(DG, n_dens - jd0);
  const int4 i0 = items[2 * w], i1 = items[2 * w + 1];
  const int32_t off = i0.x, len = i0.y, ctr_first = i0.z, row_first = i0.w;
  const int n_ctr = i1.x, nsl = i1.y;  // centers, slices per center
  const int cl = lane / nsl;
  const int sl = lane - cl * nsl;
  const bool active = cl < n_ctr;
  const int32_t c = ctr_first + (active ? cl : 0);
  const double2 cc = cxy[c];
  const double r = cr[c];
  const double2 *lt = g_log_tab;
  NearAccMD<KIND, PQ, DG> acc;
  acc.zero();
  for (int32_t base = 0; base < len; base += kNearBatch) {
    const int nb = min(kNearBatch, (int)(len - base));
    __syncthreads();
    for (int j = lane; j < nb; j += 64) {
      const int32_t s = near_src[off + base + j];
      t_xy[j] = sxy[s];
#pragma unroll
      for (int g = 0; g < DG; ++g) {
        const int64_t o = (int64_t)(jd0 + g) * src_st + s;
        if (KIND & 1) t_q[g][j] = g < ng ? sq[o] : 0.0;
        if (KIND & 2) t_d[g][j] = g < ng ? sdip[o] : make_double2(0.0, 0.0);
      }
    }
    __syncthreads();
    if (active) {
      for (int j = sl; j < nb; j += nsl) {
        const double2 z = make_double2(t_xy[j].x - cc.x, t_xy[j].y - cc.y);
        double q[DG];
        double2 dr[DG];
#pragma unroll
        for (int g = 0; g < DG; ++g) {
          q[g] = (KIND & 1) ? t_q[g][j] : 0.0;
          dr[g] = (KIND & 2) ? t_d[g][j] : make_double2(0.0, 0.0);
        }
        acc.add(z, q, dr, lt);
      }
    }
  }
  for (int o = 1; o < nsl; o <<= 1) {
    const bool take = (sl & (2 * o - 1)) == 0 && sl + o < nsl;
#pragma unroll
    for (int g = 0; g < DG; ++g) {
#pragma unroll
      for (int m = 0; m <= PQ; ++m) {
        slice_add(acc.a[g][m].x, o, take);
        slice_add(acc.a[g][m].y, o, take);
      }
      if (KIND & 1) slice_add(acc.logsum[g], o, take);
    }
  }
  if (active && sl == 0) {
#pragma unroll
    for (int g = 0; g < DG; ++g) {
      if (g >= ng) break;
      double2 alpha[PQ + 1];
#pragma unroll
      for (int m = 0; m <= PQ; ++m) alpha[m] = make_double2(0.0, 0.0);
      acc.finish(g, alpha, r);
      double2 *row = anear + (int64_t)(jd0 + g) * row_st + (int64_t)(row_first + cl) * rs;
#pragma unroll
      for (int m = 0; m <= PQ; ++m) row[m] = alpha[m];
    }
  }
}

// ------------------------------------------------------------------------------------------
// Stage 5b, M2QBXL: the multipole of a List 3 far box d taken to the QBX local expansion of a
// center c (eq. (m2l) with the corrected a_0 sign, truncated at order PQ), y = c - c_d:
//   alpha_0 += a_0 log|y| + sum_k a_k (s_d/y)^k
//   alpha_m += (-r/y)^m [-a_0/m + sum_k C(m+k-1,k-1) a_k (s_d/y)^k]
//
// The binomial-weighted sums V_m = sum_k C(m+k-1, k-1) T_k, T_k = a_k (s_d/y)^k, are formed without
// binomials: since C(m+k-1, m) = sum_{j<=k} C(m+j-2, m-1), V_m is the (m+1)-fold suffix sum of T.
// Walking k downwards with running sums S_0 += T_k, S_1 += S_0, ..., S_PQ += S_{PQ-1} leaves
// V_m = S_m. The powers w^k are produced downwards from w^p by multiplications with 1/w.
// Pair geometry: y = c - c_d, the side s_d of box d and the radius r of center c.
template <int PQ, typename E>
__device__ __forceinline__ void m2qbxl_add_geo(double2 *alpha, double2 y, double sd, double r,
                                               const E *__restrict__ Md, int P1,
                                               const double2 *__restrict__ lt) {
  const double2 iy = cinv(y);
  const double2 w = cscale(iy, sd);
  const double2 iw = make_double2(y.x / sd, y.y / sd);
  const double2 u = cscale(iy, -r);
  const double a0 = Md[0].x;
  double2 S[PQ + 1];
#pragma unroll
  for (int m = 0; m <= PQ; ++m) S[m] = make_double2(0.0, 0.0);
  double2 wk = cpowi(w, P1 - 1);
  for (int k = P1 - 1; k >= 1; --k) {
    S[0] = cfma(to_d2(Md[k]), wk, S[0]);
#pragma unroll
    for (int m = 1; m <= PQ; ++m) S[m] = cadd(S[m], S[m - 1]);
    wk = cmul(wk, iw);
  }
  // alpha_0 += a_0 log|y| + V_0;  alpha_m += u^m (V_m - a_0/m)
  alpha[0].x += a0 * 0.5 * log_tab(cnorm2(y), lt);
  alpha[0] = cadd(alpha[0], S[0]);
  double2 pm = u;
#pragma unroll
  for (int m = 1; m <= PQ; ++m) {
    alpha[m] = cfma(pm, make_double2(S[m].x - a0 / m, S[m].y), alpha[m]);
    pm = cmul(pm, u);
  }
}

template <int PQ, typename E>
__device__ __forceinline__ void m2qbxl_add(double2 *alpha, double2 cc, double r, int32_t d,
                                           const double2 *__restrict__ bc,
                                           const int32_t *__restrict__ blevel,
                                           const double *__restrict__ level_side,
                                           const E *__restrict__ Md, int P1,
                                           const double2 *__restrict__ lt) {
  m2qbxl_add_geo<PQ, E>(alpha, make_double2(cc.x - bc[d].x, cc.y - bc[d].y),
                        level_side[blevel[d]], r, Md, P1, lt);
}

// Work items for Stage 5b, same item layout and lane mapping as k_near, the slices striding over
// the chunk's List 3 far boxes. One wavefront per work-group; the chunk's multipoles are staged
// in LDS first (dynamic LDS of far_chunk x P1 coefficients), so the serial recurrence over k
// reads LDS instead of waiting on global memory at every step.
template <int PQ, typename E>
__global__ void __launch_bounds__(64) k_m2qbxl(
    int32_t n_items, const int4 *__restrict__ items, const int32_t *__restrict__ wf_idx,
    const double2 *__restrict__ cxy, const double *__restrict__ cr,
    const double2 *__restrict__ bc, const int32_t *__restrict__ blevel,
    const double *__restrict__ level_side, const E *__restrict__ M, int P1,
    double2 *__restrict__ anear, int rs, int64_t box_st, int64_t row_st) {
  HIP_DYNAMIC_SHARED(unsigned char, m2q_lds)
  E *Ms = reinterpret_cast<E *>(m2q_lds);
  const int32_t w = (int32_t)blockIdx.x;
  const double2 *lt = g_log_tab;
  const int lane = threadIdx.x;
  M += (int64_t)blockIdx.y * box_st;
  anear += (int64_t)blockIdx.y * row_st;
  const int4 i0 = items[2 * w], i1 = items[2 * w + 1];
  const int32_t off = i0.x, len = i0.y, ctr_first = i0.z, row_first = i0.w;
  const int n_ctr = i1.x, lg = i1.y;
  for (int i = lane; i < len * P1; i += 64) {
    const int e = i / P1, k = i - e * P1;
    Ms[i] = M[(int64_t)wf_idx[off + e] * P1 + k];
  }
  __syncthreads();
  const int nsl = 64 >> lg;
  const int cl = lane >> (6 - lg);
  const int sl = lane & (nsl - 1);
  const bool active = cl < n_ctr;
  const int32_t c = ctr_first + (active ? cl : 0);
  const double2 cc = cxy[c];
  const double r = cr[c];
  double2 alpha[PQ + 1];
#pragma unroll
  for (int m = 0; m <= PQ; ++m) alpha[m] = make_double2(0.0, 0.0);
  if (active)
    for (int32_t e = sl; e < len; e += nsl)
      m2qbxl_add<PQ, E>(alpha, cc, r, wf_idx[off + e], bc, blevel, level_side, Ms + e * P1, P1,
                        lt);
  for (int o = nsl >> 1; o >= 1; o >>= 1) {
#pragma unroll
    for (int m = 0; m <= PQ; ++m) {
      alpha[m].x += __shfl_xor(alpha[m].x, o, 64);
      alpha[m].y += __shfl_xor(alpha[m].y, o, 64);
    }
  }
  if (active && sl == 0) {
    double2 *row = anear + (int64_t)(row_first + cl) * rs;
#pragma unroll
    for (int m = 0; m <= PQ; ++m) row[m] = alpha[m];
  }
}

// Stage 5b over (center, List 3 far box) pairs packed across boxes, one pair per lane: a
// wavefront holds whole units (a center and one chunk of its box's List 3 far boxes, one row),
// so boxes with few centers or few far boxes no longer leave most lanes idle. The multipoles of
// the wavefront's chunks and its unit records are staged in LDS, and each pair's geometry
// (y = c - c_d, s_d, r; fixed by the build) comes as one record, so a lane waits on no chain of
// dependent loads. Each lane forms its pair's coefficients, then the units' lanes are summed in
// lane order through LDS, kM2qBlock coefficients per pass, and every unit writes its row.
// VAL (every center serves at most one target, no derivative at the targets): each lane
// evaluates its pair's coefficients at the center's target instead (Horner in (x - c)/r, the
// series k_qbx_center evaluates), and every unit writes the sum of its lanes' values, in lane
// order, to nval: one double per (center, far chunk) row instead of p + 1 complex coefficients.
constexpr int kM2qBlock = 8;

template <int PQ, typename E, bool VAL>
__global__ void __launch_bounds__(64) k_m2qbxl_packed(
    const int4 *__restrict__ waves, const int32_t *__restrict__ slots,
    const double4 *__restrict__ geo, const int32_t *__restrict__ stage,
    const int4 *__restrict__ units, const E *__restrict__ M, int P1,
    double2 *__restrict__ anear, int rs, int64_t box_st, int64_t row_st,
    const double2 *__restrict__ uz, double *__restrict__ nval, int64_t nv_st) {
  HIP_DYNAMIC_SHARED(unsigned char, m2q_lds)
  int4 *us = reinterpret_cast<int4 *>(m2q_lds);                       // [64] unit records
  double2 *zl = reinterpret_cast<double2 *>(m2q_lds + 64 * sizeof(int4));  // VAL: [64] per lane
  unsigned char *body = m2q_lds + 64 * sizeof(int4) + (VAL ? 64 * sizeof(double2) : 0);
  E *Ms = reinterpret_cast<E *>(body);                                // staged multipoles
  double2 *red = reinterpret_cast<double2 *>(body);                   // then [kM2qBlock][64]
  const double2 *lt = g_log_tab;
  const int lane = threadIdx.x;
  M += (int64_t)blockIdx.y * box_st;
  anear += (int64_t)blockIdx.y * row_st;
  const int4 w0 = waves[2 * blockIdx.x], w1 = waves[2 * blockIdx.x + 1];
  const int32_t pair0 = w0.x, npairs = w0.y, stage0 = w0.z, nstage = w0.w;
  const int32_t unit0 = w1.x, nunits = w1.y;
  if (lane < nunits) {
    const int4 un = units[unit0 + lane];
    us[lane] = un;
    if constexpr (VAL) {
      // (x - c)/r of the unit's center's target (fixed by the build): where its lanes evaluate
      const double2 z = uz[unit0 + lane];
      for (int l = 0; l < un.z; ++l) zl[un.y + l] = z;
    }
  }
  for (int i = lane; i < nstage * P1; i += 64) {
    const int e = i / P1, k = i - e * P1;
    Ms[i] = M[(int64_t)stage[stage0 + e] * P1 + k];
  }
  __syncthreads();
  double2 alpha[PQ + 1];
#pragma unroll
  for (int m = 0; m <= PQ; ++m) alpha[m] = make_double2(0.0, 0.0);
  if (lane < npairs) {
    const int slot = slots[pair0 + lane];
    const double4 g = geo[pair0 + lane];
    m2qbxl_add_geo<PQ, E>(alpha, make_double2(g.x, g.y), g.z, g.w, Ms + slot * P1, P1, lt);
  }
  if constexpr (VAL) {
    double v = 0.0;
    if (lane < npairs) {
      const double2 z = zl[lane];
      double2 sv = alpha[PQ];
#pragma unroll
      for (int m = PQ - 1; m >= 0; --m) sv = cfma(sv, z, alpha[m]);
      v = sv.x;
    }
    double *rv = reinterpret_cast<double *>(body);
    __syncthreads();  // the staged multipoles are no longer read
    rv[lane] = v;
    __syncthreads();
    if (lane < nunits) {
      const int4 un = us[lane];
      double acc = rv[un.y];
      for (int l = 1; l < un.z; ++l) acc += rv[un.y + l];
      nval[(int64_t)blockIdx.y * nv_st + un.x] = acc;
    }
    return;
  }
#pragma unroll
  for (int m0 = 0; m0 <= PQ; m0 += kM2qBlock) {
    constexpr int kLast = PQ + 1;
    const int mcount = kLast - m0 < kM2qBlock ? kLast - m0 : kM2qBlock;
    __syncthreads();  // the staged multipoles / the previous block are no longer read
#pragma unroll
    for (int mm = 0; mm < kM2qBlock; ++mm)
      if (mm < mcount) red[mm * 64 + lane] = alpha[m0 + mm];
    __syncthreads();
    for (int o = lane; o < nunits * mcount; o += 64) {
      const int u = o / mcount, mm = o - u * mcount;
      const int4 un = us[u];
      double2 acc = red[mm * 64 + un.y];
      for (int l = 1; l < un.z; ++l) acc = cadd(acc, red[mm * 64 + un.y + l]);
      anear[(int64_t)un.x * rs + m0 + mm] = acc;
    }
  }
}

// ------------------------------------------------------------------------------------------
// Stage 8 per center: L2QBXL (box local -> center), plus the direct and List 3 far rows from
// k_near and k_m2qbxl, then QBXL2P at its targets.
// One thread per center (tree order, so a wave covers centers of a few neighbouring boxes), one
// wavefront per work-group: the complete locals of the wave's first kCenterStage boxes are
// staged in LDS, so the serial shift loop reads its coefficients from LDS instead of waiting on
// global memory at every step (a further box reads them from global memory).
constexpr int kCenterStage = 8;

template <int KIND, int PQ, typename E>
__global__ void __launch_bounds__(64) k_qbx_center(
    int32_t nc, const int32_t *__restrict__ clist, int rs, int ls,
    const double2 *__restrict__ cxy, const double *__restrict__ cr,
    const int32_t *__restrict__ cbox, const double2 *__restrict__ bc,
    const int32_t *__restrict__ blevel, const double *__restrict__ level_side,
    const E *__restrict__ L, int P1, const double *__restrict__ l2q_binom,
    const int32_t *__restrict__ bctr0, const int32_t *__restrict__ bctr1,
    const int32_t *__restrict__ part_base, const int32_t *__restrict__ n_chunks,
    const int32_t *__restrict__ n_val_chunks, const double *__restrict__ nval,
    const double2 *__restrict__ anear,
    const int32_t *__restrict__ c2t_start, const int32_t *__restrict__ c2t_slot,
    const double2 *__restrict__ txy, double *__restrict__ tv, int64_t box_st, int64_t row_st,
    int64_t tv_st, const double2 *__restrict__ tnrm, int64_t nv_st) {
  HIP_DYNAMIC_SHARED(unsigned char, ctr_lds)
  E *Ls = reinterpret_cast<E *>(ctr_lds);  // [kCenterStage][P1]
  __shared__ int32_t sbox[kCenterStage];
  const int lane = threadIdx.x;
  const int32_t ic = blockIdx.x * 64 + lane;
  const bool active = ic < nc;
  const int32_t c = clist[active ? ic : nc - 1];
  {
    const int64_t jd = blockIdx.y;
    L += jd * box_st;
    anear += jd * row_st;
    tv += jd * tv_st;
    if (nval) nval += jd * nv_st;
  }
  const int32_t b = cbox[c];
  // runs of equal boxes across the wave's lanes; run j < kCenterStage is staged in LDS row j
  const int32_t bprev = __shfl_up(b, 1, 64);
  const uint64_t runs = __ballot(lane == 0 || bprev != b);
  const int rank = __popcll(runs & (~0ull >> (63 - lane))) - 1;
  const int nst = min(__popcll(runs), kCenterStage);
  {
    uint64_t m = runs;
    for (int j = 0; j < nst; ++j) {
      const int l = __ffsll((long long)m) - 1;
      m &= m - 1;
      const int32_t bx = __shfl(b, l, 64);
      if (lane == 0) sbox[j] = bx;
    }
  }
  __syncthreads();
  for (int i = lane; i < nst * P1; i += 64) {
    const int j = i / P1, k = i - j * P1;
    Ls[i] = L[(int64_t)sbox[j] * P1 + k];
  }
  __syncthreads();
  if (!active) return;
  const double2 cc = cxy[c];
  const double r = cr[c];
  double2 alpha[PQ + 1];

  // L2QBXL: alpha_m = (r/s)^m sum_{k>=m} C(k,m) b_k t^(k-m), t = (c - c_b)/s.
  // With a_k = b_k t^k the sums sum_k C(k,m) a_k are the coefficients of sum_k a_k (1+h)^k in h,
  // formed by Horner in (1+h): per k (downwards) S_m += S_(m-1) for m = PQ..1, then S_0 += a_k,
  // additions only; then alpha_m = S_m (r/(c - c_b))^m. The powers t^k run downwards from t^p by
  // multiplications with 1/t. Where t^p could underflow (|t| below 2^(-900/p)), the plain Horner
  // in t (a complex product per coefficient and step) is used instead.
  {
    const double s = level_side[blevel[b]];
    const double is = 1.0 / s;
    const double2 d = make_double2(cc.x - bc[b].x, cc.y - bc[b].y);
    const double2 t = make_double2(d.x * is, d.y * is);
#pragma unroll
    for (int m = 0; m <= PQ; ++m) alpha[m] = make_double2(0.0, 0.0);
    const E *Lb = rank < kCenterStage ? Ls + rank * P1 : L + (int64_t)b * P1;
    const double t2 = cnorm2(t);
    const bool shift1 = t2 >= ldexp(1.0, -1800 / (P1 > 1 ? P1 - 1 : 1));
    if (shift1) {
      const double it2 = 1.0 / t2;
      const double2 it = make_double2(t.x * it2, -t.y * it2);
      double2 pw = cpowi(t, P1 - 1);
#pragma unroll 4
      for (int k = P1 - 1; k >= 0; --k) {
        const double2 a = cmul(to_d2(Lb[k]), pw);
#pragma unroll
        for (int m = PQ; m >= 1; --m) alpha[m] = cadd(alpha[m], alpha[m - 1]);
        alpha[0] = cadd(alpha[0], a);
        pw = cmul(pw, it);
      }
      const double2 rho = cscale(cinv(d), r);
      double2 f = rho;
#pragma unroll
      for (int m = 1; m <= PQ; ++m) {
        alpha[m] = cmul(alpha[m], f);
        f = cmul(f, rho);
      }
    }
#pragma unroll 4
    for (int k = shift1 ? -1 : P1 - 1; k >= 0; --k) {
      const double2 bk = to_d2(Lb[k]);
      const double *Ck = l2q_binom + (int64_t)k * ls;
#pragma unroll
      for (int m = 0; m <= PQ; ++m)
        if (m <= k) alpha[m] = caxpy(Ck[m], bk, cmul(alpha[m], t));
    }
    if (!shift1) {
      const double rs = r * is;
      double f = rs;
#pragma unroll
      for (int m = 1; m <= PQ; ++m) {
        alpha[m] = cscale(alpha[m], f);
        f *= rs;
      }
    }
  }

  // direct (P2QBXL) and List 3 far (M2QBXL) rows of this center, in chunk order; with
  // n_val_chunks the box's first n_val_chunks[b] rows are values at the center's target in nval:
  // the direct rows (k_near_sd_t), or every row (the far ones from k_m2qbxl_packed, VAL)
  {
    const int32_t nbc = bctr1[b] - bctr0[b];
    const int32_t loc = c - bctr0[b];
    const int32_t nch = n_chunks[b];
    const int32_t nvc = n_val_chunks ? n_val_chunks[b] : 0;
    for (int32_t j = 0; j < nch; ++j) {
      const int64_t r = (int64_t)part_base[b] + j * nbc + loc;
      if (j < nvc) {
        alpha[0].x += nval[r];
        continue;
      }
      const double2 *row = anear + r * rs;
#pragma unroll
      for (int m = 0; m <= PQ; ++m) alpha[m] = cadd(alpha[m], row[m]);
    }
  }
  eval_targets<PQ>(c, cc, r, alpha, c2t_start, c2t_slot, txy, tv, tnrm);
}

// Stage 8 and the List 3 far part of Stage 5 summed at the centers' targets, for centers that
// serve at most one target (with the direct values of k_near_sd_t / k_near_val_mfma). For a
// center c of box b with target x, zeta = x - c, the box parts of its QBX expansion at x are:
//   L2QBXL: Re sum_k b_k U_k, U_k = sum_{m <= min(k, p)} C(k, m) t^(k-m) w^m, t = (c - c_b)/s_b,
//     w = zeta/s_b: the box local (a series in (x - c_b)/s_b) shifted to c and truncated at the
//     QBX order p, by U_0 = 1, U_k = (t + w) U_(k-1) - [k > p] C(k-1, p) t^(k-1-p) w^(p+1);
//   M2QBXL from a List 3 far box d: a_0 (log|y| - Re sum_{m=1..p} rho^m / m)
//     + Re sum_{k>=1} M_k W_k, W_k = (s_d/y)^k P_k(rho), y = c - c_d, rho = -zeta/y,
//     P_k(rho) = sum_{m<=p} C(k+m-1, m) rho^m: the multipole's Taylor series about c truncated
//     at p, evaluated at x.
// These are the coefficient forms of k_qbx_center and k_m2qbxl evaluated at x, summed in another
// order. The weights U_k, W_k do not depend on the density: one wavefront per (box, block of up
// to 16 RT centers) forms them for one segment at a time (the box local, then each List 3 far
// box) in LDS and contracts them with the segment's expansion over the slots on the matrix cores:
// rows the centers (RT tiles of 16, each B operand serving all of them), k the real and imaginary
// parts of the coefficients (Re(b U) = b.x U.x - b.y U.y), columns 16 NT slots. Then the center's
// direct values (nval) are added and its target written.
template <int PQ, int NT, int RT, typename E>
__global__ void __launch_bounds__(64) k_ctr_val(
    const int4 *__restrict__ items, const int32_t *__restrict__ wf_idx,
    const double2 *__restrict__ cxy, const double2 *__restrict__ bc,
    const int32_t *__restrict__ blevel, const double *__restrict__ level_side,
    const E *__restrict__ M, const E *__restrict__ L, int P1,
    const double *__restrict__ m2q_binom, int ls,
    const int32_t *__restrict__ bctr0, const int32_t *__restrict__ bctr1,
    const int32_t *__restrict__ part_base, const int32_t *__restrict__ n_near_chunks,
    const double *__restrict__ nval, const int32_t *__restrict__ c2t_start,
    const int32_t *__restrict__ c2t_slot, const double2 *__restrict__ txy,
    double *__restrict__ tv, int64_t box_st, int64_t nv_st, int64_t tv_st, int nslots) {
  HIP_DYNAMIC_SHARED(unsigned char, cv_lds)
  // k order of a segment: coefficient k = 4 j + r sits at entry 8 j + r (real part, k-step 2 j,
  // B row r) and 8 j + 4 + r (imaginary part, k-step 2 j + 1), so that lane r of a B column loads
  // coefficient 4 j + r whole and uses its two parts in consecutive k-steps
  const int nks = 2 * ((P1 + 3) >> 2);  // k-steps of one segment
  const int ke = 4 * nks;               // real entries of a segment (zero-padded)
  constexpr int RS = 16 * RT + 1;       // LDS row stride of the weights, [entry][center]
  double *As = reinterpret_cast<double *>(cv_lds);  // [ke][RS]
  double *Cb = As + ke * RS;                         // [P1][PQ + 1] C(k+m-1, m)
  constexpr int kFarStage = 64;                      // List 3 far boxes staged per item
  __shared__ double4 fgeo[kFarStage];                // center, side of each far box
  __shared__ int32_t fidx[kFarStage];
  const int lane = threadIdx.x;
  const int4 i0 = items[2 * blockIdx.x], i1 = items[2 * blockIdx.x + 1];
  const int32_t b = i0.x, cfirst = i0.y, n_ctr = i0.z, far0 = i0.w, nfar = i1.x;
  const int d0 = blockIdx.y * 16 * NT;
  const int nrt = (n_ctr + 15) >> 4;  // row tiles in use (uniform)
  for (int e = lane; e < ke * RS; e += 64) As[e] = 0.0;
  for (int e = lane; e < P1 * (PQ + 1); e += 64) Cb[e] = m2q_binom[(e / (PQ + 1)) * ls + e % (PQ + 1)];
  if (lane < nfar && lane < kFarStage) {
    const int32_t d = wf_idx[far0 + lane];
    fidx[lane] = d;
    fgeo[lane] = make_double4(bc[d].x, bc[d].y, level_side[blevel[d]], 0.0);
  }
  // the geometry of far box f (staged for the first kFarStage)
  auto far_box = [&](int f, int32_t &d, double2 &cd, double &sd) {
    if (f < kFarStage) {
      d = fidx[f];
      const double4 g4 = fgeo[f];
      cd = make_double2(g4.x, g4.y);
      sd = g4.z;
    } else {
      d = wf_idx[far0 + f];
      cd = bc[d];
      sd = level_side[blevel[d]];
    }
  };
  const int i = lane & 15, q = lane >> 4;
  // the weight rows of this lane: center 16 r + i of the block (row tile r) and its target offset
  bool row_on[RT];
  double2 cc[RT], tz[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    row_on[r] = 16 * r + i < n_ctr;
    const int32_t c = cfirst + (row_on[r] ? 16 * r + i : 0);
    cc[r] = cxy[c];
    tz[r] = make_double2(0.0, 0.0);
    const int32_t g = c2t_start[c];
    if (c2t_start[c + 1] > g) {
      const double2 x = txy[c2t_slot[g] >> 1];
      tz[r] = make_double2(x.x - cc[r].x, x.y - cc[r].y);
    }
  }
  gq_d4 C[RT][NT];
  // this lane's B-operand columns: offsets of its slots (-1: past the last slot)
  int64_t so[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
    for (int r = 0; r < RT; ++r) C[r][nt] = gq_d4{0.0, 0.0, 0.0, 0.0};
    const int sl = d0 + 16 * nt + i;
    so[nt] = sl < nslots ? (int64_t)sl * box_st : -1;
  }
  auto ent = [](int k) { return 8 * (k >> 2) + (k & 3); };  // entry of the real part
  const int kq = (P1 + 3) >> 2;  // coefficients per lane group q in a far segment
  // B operands in groups of 2 GH k-steps (GH coefficients per column and lane, 16 values in
  // flight), the next group (or the next segment's first) loaded while the current one is on
  // the matrix cores; kept in the storage type until used (a conversion at the load would wait
  // for it at once). One B load serves the RT row tiles.
  constexpr int GH = 8 / NT;
  const int ngr = (nks / 2 + GH - 1) / GH;
  E bcur[GH][NT], bnext[GH][NT];
  auto seg_ptr = [&](int32_t bx, bool local) { return (local ? L : M) + (int64_t)bx * P1; };
  auto load_group = [&](const E *X, int gi, E (&bv)[GH][NT]) {
#pragma unroll
    for (int jj = 0; jj < GH; ++jj) {
      const int k = 4 * (gi * GH + jj) + q;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int64_t o = so[nt] + (k < P1 ? k : 0);
        bv[jj][nt] = X[o < 0 ? 0 : o];  // masked at use
      }
    }
  };
  const E *X = seg_ptr(b, true);
  load_group(X, 0, bcur);
  __syncthreads();  // the staged far boxes
  for (int sg = 0; sg <= nfar; ++sg) {
    __syncthreads();  // the previous segment's weights are no longer read
    if (sg == 0) {
      // lane group q < RT forms the local weights of row tile q
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        if (q != r || r >= nrt) continue;
        const double is = 1.0 / level_side[blevel[b]];
        const double2 t = make_double2((cc[r].x - bc[b].x) * is, (cc[r].y - bc[b].y) * is);
        const double2 w = make_double2(tz[r].x * is, tz[r].y * is);
        const double2 tw = cadd(t, w);
        double2 u = make_double2(1.0, 0.0);
        double2 tp = make_double2(1.0, 0.0);    // t^(k-1-p)
        double cb = 1.0;                        // C(k-1, p), exact integers
        const double2 wp1 = cpowi(w, PQ + 1);
        for (int k = 0; k < P1; ++k) {
          if (k > 0) {
            u = cmul(tw, u);
            if (k > PQ) {
              if (k > PQ + 1) cb = cb * (double)(k - 1) / (double)(k - 1 - PQ);
              u = csub(u, cscale(cmul(tp, wp1), cb));
              tp = cmul(tp, t);
            }
          }
          As[ent(k) * RS + 16 * r + i] = row_on[r] ? u.x : 0.0;
          As[(ent(k) + 4) * RS + 16 * r + i] = row_on[r] ? -u.y : 0.0;
        }
      }
    } else {
      int32_t box;
      double2 cd;
      double sd;
      far_box(sg - 1, box, cd, sd);
      const int k0 = q * kq, k1 = min(P1, k0 + kq);
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        if (r >= nrt) continue;
        const double2 y = make_double2(cc[r].x - cd.x, cc[r].y - cd.y);
        const double2 iy = cinv(y);
        const double2 w = cscale(iy, sd);
        const double2 rho = make_double2(-(tz[r].x * iy.x - tz[r].y * iy.y),
                                         -(tz[r].x * iy.y + tz[r].y * iy.x));
        if (q == 0) {
          // a_0 weight: log|y| - Re sum_{m=1..p} rho^m / m
          const double r1 = 2.0 * rho.x, s2 = cnorm2(rho);
          double b2 = 1.0 / PQ, b1 = fma(r1, b2, 1.0 / (PQ - 1));
#pragma unroll
          for (int m = PQ - 2; m >= 1; --m) {
            const double b0 = fma(r1, b1, fma(-s2, b2, 1.0 / m));
            b2 = b1;
            b1 = b0;
          }
          const double a0w = 0.5 * log_tab(cnorm2(y), g_log_tab) - fma(b1, rho.x, -(s2 * b2));
          As[ent(0) * RS + 16 * r + i] = row_on[r] ? a0w : 0.0;
          As[(ent(0) + 4) * RS + 16 * r + i] = 0.0;
        }
        double2 wk = cpowi(w, k0 > 1 ? k0 : 1);
        for (int k = k0 > 1 ? k0 : 1; k < k1; ++k) {
          const double *ck = Cb + k * (PQ + 1);
          double2 h = make_double2(ck[PQ], 0.0);
#pragma unroll
          for (int m = PQ - 1; m >= 0; --m)
            h = make_double2(fma(h.x, rho.x, fma(-h.y, rho.y, ck[m])), fma(h.x, rho.y, h.y * rho.x));
          const double2 wv = cmul(wk, h);
          As[ent(k) * RS + 16 * r + i] = row_on[r] ? wv.x : 0.0;
          As[(ent(k) + 4) * RS + 16 * r + i] = row_on[r] ? -wv.y : 0.0;
          wk = cmul(wk, w);
        }
      }
    }
    __syncthreads();
    for (int gi = 0; gi < ngr; ++gi) {
      if (gi + 1 < ngr) {
        load_group(X, gi + 1, bnext);
      } else if (sg < nfar) {
        int32_t nb2;
        double2 cd2;
        double sd2;
        far_box(sg, nb2, cd2, sd2);
        X = seg_ptr(nb2, false);
        load_group(X, 0, bnext);
      }
#pragma unroll
      for (int jj = 0; jj < GH; ++jj) {
        const int ks = 2 * (gi * GH + jj);
        if (ks < nks) {
          const bool kon = 2 * ks + q < P1;  // this lane's coefficient 4 (ks / 2) + q exists
          double2 bb[NT];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            bb[nt] = (kon && so[nt] >= 0) ? to_d2(bcur[jj][nt]) : make_double2(0.0, 0.0);
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            if (r >= nrt) continue;
            const double are = As[(4 * ks + q) * RS + 16 * r + i];  // A row i of tile r
            const double aim = As[(4 * ks + 4 + q) * RS + 16 * r + i];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) C[r][nt] = mfma16(are, bb[nt].x, C[r][nt]);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) C[r][nt] = mfma16(aim, bb[nt].y, C[r][nt]);
          }
        }
      }
#pragma unroll
      for (int jj = 0; jj < GH; ++jj)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bcur[jj][nt] = bnext[jj][nt];
    }
  }
  // lane (column j = lane & 15, group g = lane >> 4) holds rows (centers) 16 r + g + 4 v
  const int g = q, j = i;
  const int32_t nbc = bctr1[b] - bctr0[b];
  const int32_t nnear = n_near_chunks[b];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ci = 16 * r + g + 4 * v;
      if (ci >= n_ctr) continue;
      const int32_t cv = cfirst + ci;
      const int32_t t0 = c2t_start[cv];
      if (c2t_start[cv + 1] <= t0) continue;
      const int32_t tslot = c2t_slot[t0];
      const int64_t row0 = (int64_t)part_base[b] + (cv - bctr0[b]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int sl = d0 + 16 * nt + j;
        if (sl >= nslots) continue;
        double val = C[r][nt][v];
        for (int32_t ch = 0; ch < nnear; ++ch)
          val += nval[(int64_t)sl * nv_st + row0 + (int64_t)ch * nbc];
        tv[(int64_t)sl * tv_st + tslot] = -kInv2Pi * val;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Direct (unaccelerated) QBX: every center of one order bucket (clist, n) takes every source,
// staged through LDS tiles.
template <int KIND, int PQ>
__global__ void __launch_bounds__(256) k_direct(
    int32_t nc, const int32_t *__restrict__ clist, const double2 *__restrict__ cxy,
    const double *__restrict__ cr, int32_t ns,
    const double2 *__restrict__ sxy, const double *__restrict__ sq,
    const double2 *__restrict__ sdip, const int32_t *__restrict__ c2t_start,
    const int32_t *__restrict__ c2t_slot, const double2 *__restrict__ txy,
    double *__restrict__ tv, int64_t src_st, int64_t tv_st, const double2 *__restrict__ tnrm) {
  __shared__ double2 ts[256];
  {
    const int64_t jd = blockIdx.y;
    sq += jd * src_st;
    sdip += jd * src_st;
    tv += jd * tv_st;
  }
  __shared__ double tq[256];
  __shared__ double2 td[256];
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < nc;
  const int32_t c = active ? clist[i] : 0;
  const double2 cc = active ? cxy[c] : make_double2(0.0, 0.0);
  const double r = active ? cr[c] : 1.0;
  const double2 *lt = g_log_tab;
  NearAcc<KIND, PQ> acc;
  acc.zero();
  for (int32_t base = 0; base < ns; base += 256) {
    const int32_t n = min(256, ns - base);
    __syncthreads();
    if ((int32_t)threadIdx.x < n) {
      ts[threadIdx.x] = sxy[base + threadIdx.x];
      if (KIND & 1) tq[threadIdx.x] = sq[base + threadIdx.x];
      if (KIND & 2) td[threadIdx.x] = sdip[base + threadIdx.x];
    }
    __syncthreads();
    if (!active) continue;
    for (int32_t j = 0; j < n; ++j) {
      const double2 z = make_double2(ts[j].x - cc.x, ts[j].y - cc.y);
      acc.add(z, (KIND & 1) ? tq[j] : 0.0, (KIND & 2) ? td[j] : make_double2(0.0, 0.0), lt);
    }
  }
  if (!active) return;
  double2 alpha[PQ + 1];
#pragma unroll
  for (int m = 0; m <= PQ; ++m) alpha[m] = make_double2(0.0, 0.0);
  acc.finish(alpha, r);
  eval_targets<PQ>(c, cc, r, alpha, c2t_start, c2t_slot, txy, tv, tnrm);
}

// ------------------------------------------------------------------------------------------
// The device natural logarithm (log_tab) or reciprocal (rcp_nr) of the kernels above, elementwise,
// so that their accuracy can be tested on their own.
__global__ void k_math(int fn, int64_t n, const double *__restrict__ x, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = fn == 1 ? log_tab(x[i], g_log_tab) : rcp_nr(x[i]);
}

// ------------------------------------------------------------------------------------------
// Average the target slots into the caller's output row: value row y of tv goes to row y of out,
// or for y >= n_first to row y - n_first of out2 (S and D rows of one evaluation in one launch).
__global__ void k_finalize(int32_t nt, const int32_t *__restrict__ tctr, const double *__restrict__ tv,
                           double *__restrict__ out, int64_t tv_st, int64_t ld_out,
                           double *__restrict__ out2, int32_t n_first) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int32_t y = (int32_t)blockIdx.y;
  tv += (int64_t)y * tv_st;
  out = y < n_first ? out + (int64_t)y * ld_out : out2 + (int64_t)(y - n_first) * ld_out;
  double s = 0.0;
  int n = 0;
  if (tctr[2 * t] >= 0) { s += tv[2 * t]; n++; }
  if (tctr[2 * t + 1] >= 0) { s += tv[2 * t + 1]; n++; }
  out[t] = n == 2 ? 0.5 * s : s;
}

// Records a HIP event pair around one stage when the context profiles (see gq_set_profiling).
class StageTimer {
 public:
  StageTimer(gq_ctx *ctx, int stage, hipStream_t s) : ctx_(ctx), s_(s) {
    if (!ctx->profiling) return;
    slot_ = (ctx->cur_kind - 1) * GQ_N_STAGES + stage;
    a_ = take(ctx);
    if (a_) (void)hipEventRecord(a_, s_);
  }
  StageTimer(gq_ctx *ctx, int stage) : StageTimer(ctx, stage, ctx->stream) {}
  ~StageTimer() {
    if (!ctx_->profiling || !a_) return;
    hipEvent_t b = take(ctx_);
    if (!b) return;
    (void)hipEventRecord(b, s_);
    ctx_->prof.push_back({slot_, a_, b});
  }

 private:
  static hipEvent_t take(gq_ctx *ctx) {
    if (!ctx->event_pool.empty()) {
      hipEvent_t e = ctx->event_pool.back();
      ctx->event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
  }
  gq_ctx *ctx_;
  hipStream_t s_;
  int slot_ = 0;
  hipEvent_t a_ = nullptr;
};

// Workspace slots from which M2L and the Stage 7 gather run as GEMMs over the slots (a full
// column tile of 8 slots per wavefront); fewer slots keep the kernels that batch 8 pairs as the
// columns of one slot.
constexpr int kSlotGemmMin = 8;
// dynamic LDS of the grouped M2L: the o^-k rows of the List 2 offsets in use
constexpr size_t kM2gLdsMax = 64 * 1024;
// Densities of a GQ_S_AND_D batch from which the direct interactions run on the matrix cores.
constexpr int kNearMfmaMin = 8;

// The direct moments and P2L of a GQ_S_AND_D batch on the matrix cores (in the expansion
// precision), from kNearMfmaMin densities.
// FP32 expansions up to 32 coefficients (two row tiles per wavefront, no spills).
template <int KIND, typename E>
bool use_p2x_mfma(int nd, int P1) {
  return KIND == 4 && nd >= kNearMfmaMin && (sizeof(E) == sizeof(double2) || P1 <= 32);
}
template <int MODE, typename E>
auto p2x_kernel(int P1) {
  if constexpr (sizeof(E) == sizeof(double2)) return P1 <= 32 ? k_p2x_mfma<MODE, 2, E> : k_p2x_mfma<MODE, 4, E>;
  else return k_p2x_mfma<MODE, 2, E>;
}

// Per-density strides of the batched buffers (elements).
struct Strides {
  int64_t src, box, row, tv, nv;
};

Strides strides(const gq_ctx *ctx) {
  const int64_t P1 = ctx->params.p_fmm + 1;
  return {ctx->ns, ctx->tree.n_boxes() * P1, ctx->n_near_rows * (ctx->params.p_qbx + 1),
          2 * ctx->nt, std::max<int64_t>(ctx->n_near_rows, 1)};
}

template <int KIND>
hipError_t launch_gather(gq_ctx *ctx, const double *d1, int64_t ld1, const double *d2,
                         int64_t ld2, int nd) {
  StageTimer st_(ctx, GQ_STAGE_GATHER);
  const int32_t ns = (int32_t)ctx->ns;
  hipLaunchKernelGGL(k_gather<KIND>, dim3((ns + 255) / 256, nd), dim3(256), 0, ctx->stream, ns,
                     ctx->d.sperm, ctx->d.sw, ctx->d.snrm, d1, ld1, d2, ld2, ctx->d.sq,
                     ctx->d.sdip);
  return hipGetLastError();
}

// Translation tables in the expansion precision.
template <typename E> struct ExpTables;
template <> struct ExpTables<double2> {
  const double *m2l_bt;
  const double2 *opow, *m2g_opow;
  explicit ExpTables(const DevBuffers &d) : m2l_bt(d.m2l_bt), opow(d.opow), m2g_opow(d.m2g_opow) {}
};
template <> struct ExpTables<float2> {
  const float *m2l_bt;
  const float2 *opow, *m2g_opow;
  explicit ExpTables(const DevBuffers &d)
      : m2l_bt(d.m2l_bt_f), opow(d.opow_f), m2g_opow(d.m2g_opow_f) {}
};

// Unused LDS requested by the one-density direct pass when it runs on the side stream beside the
// tree passes: 10 KB per work-group caps it at four waves per SIMD (seven by its registers
// alone), which leaves wave slots to the moments, M2L and the Stage 7 gather on the critical
// path. Per step of the 16-star workload: 0.410-0.413 ms against 0.443 uncapped, 0.413 at three
// waves per SIMD and 0.419 at five.
constexpr size_t kNearSideLds = 5120;

// Whether the direct pass of nd densities of a kind sums at the centers' targets (dense values
// instead of coefficient rows): every center serves at most one target, the expansions are not
// differentiated at the targets (GQ_SP), and either one density (k_near_sd_t) or S and D of a
// batch (k_near_val_mfma).
inline bool near_values(const gq_ctx *ctx, int nd, int kind) {
  return nd >= 1 && ctx->one_target_per_center && ctx->d.n_near_chunks != nullptr &&
         !ctx->eval_sp && (kind == 4 || nd == 1);
}

// Whether the List 3 far part is summed at the centers' targets too (k_m2qbxl_packed, VAL): the
// direct pass is, and every List 3 far chunk is a packed unit (no k_m2qbxl items). The center
// stage then reads one value per row, direct and far alike.
inline bool m2q_values(const gq_ctx *ctx, int nd, int kind) {
  return near_values(ctx, nd, kind) && ctx->n_far_items == 0;
}

// The three per-order stages of one order bucket.
template <int KIND, int PQ, typename E>
void launch_near_bucket(gq_ctx *ctx, const OrderBucket &bk, int nd, hipStream_t s,
                        const Strides &S, double2 *anear) {
  auto &d = ctx->d;
  const int32_t n = (int32_t)(bk.near1 - bk.near0);
  if (n > 0 && near_values(ctx, nd, KIND)) {  // one density, summed at the targets
    hipLaunchKernelGGL((k_near_sd_t<KIND, PQ>), dim3(n, 1), dim3(64),
                       ctx->params.overlap ? kNearSideLds : 0, s, n, d.near_items + 2 * bk.near0,
                       d.near_src, d.cxy, d.sxy, d.sq, d.sdip, d.c2t_start, d.c2t_slot, d.txy,
                       d.nval, S.nv);
    return;
  }
  // Densities per work item: two by default. Four hold 4 (PQ + 1) complex accumulators per lane,
  // which above order 6 leaves one or two waves per SIMD and runs slower than two.
  const int dg = nd < 2 ? 1 : ctx->params.near_dens_group > 0 ? ctx->params.near_dens_group : 2;
  if (n > 0 && dg == 4)
    hipLaunchKernelGGL((k_near_md<KIND, PQ, 4>), dim3(n, (nd + 3) / 4), dim3(64), 0, s, n,
                       d.near_items + 2 * bk.near0, d.near_src, d.cxy, d.cr, d.sxy, d.sq, d.sdip,
                       anear, ctx->params.p_qbx + 1, S.src, S.row, nd);
  else if (n > 0 && dg == 2)
    hipLaunchKernelGGL((k_near_md<KIND, PQ, 2>), dim3(n, (nd + 1) / 2), dim3(64), 0, s, n,
                       d.near_items + 2 * bk.near0, d.near_src, d.cxy, d.cr, d.sxy, d.sq, d.sdip,
                       anear, ctx->params.p_qbx + 1, S.src, S.row, nd);
  else if (n > 0)
    hipLaunchKernelGGL((k_near<KIND, PQ>), dim3(n, nd), dim3(64), 0, s, n, d.near_items + 2 * bk.near0,
                       d.near_src, d.cxy, d.cr, d.sxy, d.sq, d.sdip, anear,
                       ctx->params.p_qbx + 1, S.src, S.row);
}



template <int PQ, int NT>
void launch_near_val_mfma(gq_ctx *ctx, const OrderBucket &bk, int nd, hipStream_t s,
                          const Strides &S) {
  auto &d = ctx->d;
  const int32_t nv = (int32_t)(bk.nvf1 - bk.nvf0);
  hipLaunchKernelGGL((k_near_val_mfma<PQ, NT>), dim3((uint32_t)nv, (nd + 16 * NT - 1) / (16 * NT)),
                     dim3(256), 0, s, d.near_vitems + 2 * bk.nvf0, d.near_src, d.cxy, d.sxy,
                     d.snrm, d.sq, d.c2t_start, d.c2t_slot, d.txy, d.nval, S.src, S.nv, nd,
                     (int64_t)nd);
}

// S and D of the same densities (nd of them): one fused pass for a single density, else the
// per-kind launches (their density groups already share the pair geometry across densities).
template <int PQ, typename E>
void launch_near_bucket_sd(gq_ctx *ctx, const OrderBucket &bk, int nd, hipStream_t s,
                           const Strides &S) {
  auto &d = ctx->d;
  const int32_t n = (int32_t)(bk.near1 - bk.near0);
  if (n <= 0) return;
  if (near_values(ctx, nd, 4)) {
    if (nd == 1)
      hipLaunchKernelGGL((k_near_sd_t<4, PQ>), dim3(n, 1), dim3(64),
                         ctx->params.overlap ? kNearSideLds : 0, s, n,
                         d.near_items + 2 * bk.near0, d.near_src, d.cxy, d.sxy, d.sq, d.sdip,
                         d.c2t_start, d.c2t_slot, d.txy, d.nval, S.nv);
    else if (bk.nvf1 > bk.nvf0 && nd <= 16)
      launch_near_val_mfma<PQ, 1>(ctx, bk, nd, s, S);
    else if (bk.nvf1 > bk.nvf0 && nd <= 32)
      launch_near_val_mfma<PQ, 2>(ctx, bk, nd, s, S);
    else if (bk.nvf1 > bk.nvf0)
      launch_near_val_mfma<PQ, 4>(ctx, bk, nd, s, S);
    return;
  }
  if (nd == 1) {
    hipLaunchKernelGGL((k_near_sd<PQ>), dim3(n, 1), dim3(64), 0, s, n, d.near_items + 2 * bk.near0,
                       d.near_src, d.cxy, d.cr, d.sxy, d.sq, d.sdip, d.anear,
                       ctx->params.p_qbx + 1, S.src, S.row, (int64_t)1);
    return;
  }
  const int32_t nm = (int32_t)(bk.nmf1 - bk.nmf0);
  if (nd >= kNearMfmaMin && nm > 0) {
    // one GEMM per center over the sources and a block of densities on the matrix cores
    constexpr int NT = PQ <= 12 ? 4 : 2;
    hipLaunchKernelGGL((k_near_mfma<PQ, NT>), dim3((uint32_t)nm, (nd + 16 * NT - 1) / (16 * NT)),
                       dim3(256), 0, s, nm, d.near_mitems + 2 * bk.nmf0, d.near_src, d.cxy, d.cr,
                       d.sxy, d.snrm, d.sq, d.anear, ctx->params.p_qbx + 1, S.src, S.row, nd,
                       (int64_t)nd);
    return;
  }
  launch_near_bucket<1, PQ, E>(ctx, bk, nd, s, S, d.anear);
  launch_near_bucket<2, PQ, E>(ctx, bk, nd, s, S, d.anear + (int64_t)nd * S.row);
}

// vals: the packed List 3 far units as values at the centers' targets (m2q_values)
template <int PQ, typename E>
void launch_m2qbxl_bucket(gq_ctx *ctx, const OrderBucket &bk, int nd, hipStream_t s,
                          const Strides &S, const E *M, bool vals) {
  auto &d = ctx->d;
  const int32_t nw = (int32_t)(bk.m2q1 - bk.m2q0);
  if (nw > 0) {
    const size_t lds = 64 * sizeof(int4) + (vals ? 64 * sizeof(double2) : 0) +
                       std::max(sizeof(E) * (size_t)ctx->m2q_stage_rows * (ctx->params.p_fmm + 1),
                                sizeof(double2) * kM2qBlock * 64);
    hipLaunchKernelGGL((vals ? k_m2qbxl_packed<PQ, E, true> : k_m2qbxl_packed<PQ, E, false>),
                       dim3(nw, nd), dim3(64), lds, s, d.m2q_wave + 2 * bk.m2q0, d.m2q_slot,
                       d.m2q_geo, d.m2q_stage, d.m2q_unit, M, ctx->params.p_fmm + 1, d.anear,
                       ctx->params.p_qbx + 1, S.box, S.row, d.m2q_uz, d.nval, S.nv);
  }
  const int32_t n = (int32_t)(bk.far1 - bk.far0);
  const size_t lds = sizeof(E) * (size_t)ctx->far_chunk * (ctx->params.p_fmm + 1);
  if (n > 0)
    hipLaunchKernelGGL((k_m2qbxl<PQ, E>), dim3(n, nd), dim3(64), lds, s, n,
                       d.far_items + 2 * bk.far0, d.wf_idx, d.cxy, d.cr, d.bc, d.blevel,
                       d.level_side, M, ctx->params.p_fmm + 1, d.anear, ctx->params.p_qbx + 1,
                       S.box, S.row);
}

// n_val_chunks: per box, how many of its leading rows are values at the centers' targets
// (nullptr: none)
template <int KIND, int PQ, typename E>
void launch_center_bucket(gq_ctx *ctx, const OrderBucket &bk, int nd, hipStream_t s,
                          const Strides &S, const E *L, const int32_t *n_val_chunks) {
  auto &d = ctx->d;
  const int32_t n = (int32_t)(bk.ctr1 - bk.ctr0);
  if (n > 0)
    hipLaunchKernelGGL((k_qbx_center<KIND, PQ, E>), dim3((n + 63) / 64, nd), dim3(64),
                       sizeof(E) * kCenterStage * (ctx->params.p_fmm + 1), s, n,
                       d.ctr_list + bk.ctr0, ctx->params.p_qbx + 1, ctx->params.p_qbx + 1, d.cxy,
                       d.cr, d.cbox, d.bc, d.blevel, d.level_side, L, ctx->params.p_fmm + 1,
                       d.l2q_binom, d.bctr0, d.bctr1, d.part_base, d.n_chunks,
                       n_val_chunks, n_val_chunks ? d.nval : nullptr,
                       d.anear, d.c2t_start, d.c2t_slot, d.txy, d.tv, S.box, S.row, S.tv,
                       ctx->eval_sp ? ctx->tnrm_dev : nullptr, S.nv);
}

// The center stage summed at the targets (k_ctr_val), which also takes the List 3 far
// multipoles: with the direct values of a S and D evaluation of kNearMfmaMin or more densities
// (the weights are formed once for all slots; for fewer slots the coefficient kernels are faster).
inline bool center_at_targets(const gq_ctx *ctx, int nd, bool sd) {
  return sd && nd >= kNearMfmaMin && near_values(ctx, nd, 4) && ctx->d.cval_items != nullptr;
}

// Centers per k_ctr_val item: two row tiles of 16 (the box's expansions read once for up to 32
// of its centers).
constexpr int kCtrValRT = 2;

template <int PQ, int NT, typename E>
void launch_ctr_val(gq_ctx *ctx, const OrderBucket &bk, int slots, hipStream_t s, const Strides &S,
                    const E *M, const E *L) {
  auto &d = ctx->d;
  const int32_t n = (int32_t)(bk.cv1 - bk.cv0);
  if (n <= 0) return;
  const int P1 = ctx->params.p_fmm + 1;
  const int ke = 8 * ((P1 + 3) / 4);
  const size_t lds =
      sizeof(double) * ((size_t)ke * (16 * kCtrValRT + 1) + (size_t)P1 * (PQ + 1));
  hipLaunchKernelGGL((k_ctr_val<PQ, NT, kCtrValRT, E>),
                     dim3((uint32_t)n, (slots + 16 * NT - 1) / (16 * NT)),
                     dim3(64), lds, s, d.cval_items + 2 * bk.cv0, d.wf_idx, d.cxy, d.bc, d.blevel,
                     d.level_side, M, L, P1, d.m2q_binom, ctx->params.p_qbx + 1,
                     d.bctr0, d.bctr1, d.part_base, d.n_near_chunks, d.nval, d.c2t_start,
                     d.c2t_slot, d.txy, d.tv, S.box, S.nv, S.tv, slots);
}

template <int PQ, typename E>
void launch_ctr_val_bucket(gq_ctx *ctx, const OrderBucket &bk, int slots, hipStream_t s,
                           const Strides &S, const E *M, const E *L) {
  if (slots <= 16) launch_ctr_val<PQ, 1, E>(ctx, bk, slots, s, S, M, L);
  else if (slots <= 32) launch_ctr_val<PQ, 2, E>(ctx, bk, slots, s, S, M, L);
  else launch_ctr_val<PQ, 4, E>(ctx, bk, slots, s, S, M, L);
}

template <int KIND, typename E>
hipError_t launch_fmm_t(gq_ctx *ctx, int nd) {
  // KIND 4: S and D of nd densities; the charge and dipole strengths of density j sit in source
  // slot j, and every expansion, row and target array holds S in slot j and D in slot nd + j.
  // Stages that only move expansions run once over all 2 nd slots.
  constexpr bool SD = KIND == 4;
  const int slots = SD ? 2 * nd : nd;
  constexpr int CK = SD ? 1 : KIND;  // the center stage does not depend on the kind
  auto &d = ctx->d;
  auto &t = ctx->tree;
  const ExpTables<E> X(d);
  E *M = reinterpret_cast<E *>(d.M);
  E *L = reinterpret_cast<E *>(d.L);
  E *Lf = reinterpret_cast<E *>(d.Lf);
  const int P1 = ctx->params.p_fmm + 1;
  const hipStream_t st = ctx->stream;
  const Strides S = strides(ctx);
  // The direct-interaction kernel needs only the source strengths: it runs on the side stream
  // while the upward pass, M2L, List 3 far and the downward pass proceed on the caller's stream
  // (without overlap both "streams" are the caller's stream and the events order nothing new).
  const hipStream_t side = ctx->params.overlap ? ctx->side : st;
  hipError_t e = hipEventRecord(ctx->ev_fork, st);
  if (e != hipSuccess) return e;
  e = hipStreamWaitEvent(side, ctx->ev_fork, 0);
  if (e != hipSuccess) return e;
  {
    StageTimer st_(ctx, GQ_STAGE_NEAR, side);
    for (const OrderBucket &bk : ctx->buckets) {
      switch (bk.pq) {
#define GQ_CASE(P)                                                 \
  case P:                                                          \
    if constexpr (SD) launch_near_bucket_sd<P, E>(ctx, bk, nd, side, S); \
    else launch_near_bucket<KIND, P, E>(ctx, bk, nd, side, S, d.anear); \
    break;
        GQ_PQ_LIST(GQ_CASE)
#undef GQ_CASE
      }
    }
  }
  constexpr int PK = SD ? 4 : KIND;
  constexpr int NK = SD ? 2 : 1;
  const int64_t part_st = ctx->n_p2m_parts * 2 * P1;
  if (ctx->n_p2m_items > 0) {
    StageTimer st_(ctx, GQ_STAGE_P2M);
    if (use_p2x_mfma<KIND, E>(nd, P1)) {
      auto kern = p2x_kernel<0, E>(P1);
      hipLaunchKernelGGL(kern, dim3((uint32_t)ctx->n_p2m_items, (nd + 63) / 64), dim3(256), 0, st,
                         (int32_t)ctx->n_p2m_items, d.p2m_item, nullptr, d.bc, d.blevel, d.level_inv_side, d.level_log_side,
                         d.sxy, d.snrm, d.sq, P1, M, d.Mp, S.src,
                         S.box, part_st, nd, (int64_t)nd * S.box);
    } else {
      auto kern = P1 <= 8 ? k_p2m_all<PK, 1, E> : P1 <= 16 ? k_p2m_all<PK, 2, E>
                : P1 <= 32 ? k_p2m_all<PK, 4, E> : k_p2m_all<PK, 8, E>;
      hipLaunchKernelGGL(kern, dim3((uint32_t)ctx->n_p2m_items, nd), dim3(64), 0, st, d.p2m_item,
                         d.bc, d.blevel, d.level_inv_side, d.sxy, d.sq, d.sdip, P1, M, d.Mp, S.src,
                         S.box, part_st, (int64_t)nd * S.box);
    }
  }
  if (ctx->n_p2m_red > 0) {
    StageTimer st_(ctx, GQ_STAGE_M2M);
    const bool few = nd < kNearMfmaMin;
    hipLaunchKernelGGL((few ? k_m_reduce<NK, 4, E> : k_m_reduce<NK, 1, E>),
                       dim3((uint32_t)ctx->n_p2m_red, nd), dim3(few ? 256 : 64), 0, st,
                       d.p2m_red, d.Mp, P1, M, part_st, S.box, (int64_t)nd * S.box);
  }
  e = hipEventRecord(ctx->ev_up, st);
  if (e != hipSuccess) return e;
  // List 3 far multipoles -> centers on the side stream, once the upward pass is complete
  e = hipStreamWaitEvent(side, ctx->ev_up, 0);
  if (e != hipSuccess) return e;
  const bool ctr_vals = center_at_targets(ctx, nd, SD);
  const bool qvals = m2q_values(ctx, nd, KIND);
  if ((ctx->n_far_items > 0 || ctx->n_m2q_waves > 0) && !ctr_vals) {
    StageTimer st_(ctx, GQ_STAGE_M2QBXL, side);
    for (const OrderBucket &bk : ctx->buckets) {
      switch (bk.pq) {
#define GQ_CASE(P) \
  case P: launch_m2qbxl_bucket<P, E>(ctx, bk, slots, side, S, M, qvals); break;
        GQ_PQ_LIST(GQ_CASE)
#undef GQ_CASE
      }
    }
  }
  e = hipEventRecord(ctx->ev_join, side);
  if (e != hipSuccess) return e;
  const int32_t ntb = (int32_t)ctx->n_tboxes;
  if (ntb > 0) {
    StageTimer st_(ctx, GQ_STAGE_M2L_P2L);
    // the o^-k table, then 4 wavefronts x (8 slots x 16 RT orders) staged multipole rows
    const size_t m2g_lds = (((size_t)ctx->m2g_n_off * P1 + 1) & ~(size_t)1) * sizeof(E) +
                           (size_t)4 * (P1 <= 16 ? 4 : 8) * 32 * sizeof(E);
    if (slots >= kSlotGemmMin && P1 <= 32 && ctx->n_m2g_items > 0 && m2g_lds <= kM2gLdsMax) {
      // sibling groups: a GEMM per (record, member) over the slots (8 per wavefront)
      const int nw = std::min(4, (slots + 7) / 8);
      auto kern = P1 <= 16 ? k_m2l_grp<1, E> : k_m2l_grp<2, E>;
      hipLaunchKernelGGL(kern, dim3((uint32_t)ctx->n_m2g_items, (slots + 8 * nw - 1) / (8 * nw)),
                         dim3(64 * nw), m2g_lds, st, d.m2g_item, d.m2g_rec, d.m2g_plog, d.m2g_grp,
                         M, X.m2l_bt, X.m2g_opow, ctx->m2g_n_off, P1, L, S.box, slots);
    } else if (slots >= kSlotGemmMin) {
      // a GEMM per List 2 pair over the slots (8 per wavefront)
      const int nw = std::min(4, (slots + 7) / 8);
      auto kern = P1 <= 16 ? k_m2l_slots<1, E> : P1 <= 32 ? k_m2l_slots<2, E>
                : P1 <= 48 ? k_m2l_slots<3, E> : k_m2l_slots<4, E>;
      hipLaunchKernelGGL(kern, dim3((uint32_t)ctx->n_m2l_items, (slots + 8 * nw - 1) / (8 * nw)),
                         dim3(64 * nw), 0, st, (int32_t)ctx->n_m2l_items, d.m2l_item, d.m2l_pr, d.m2l_plog, M, X.m2l_bt,
                         X.opow, P1, L, S.box, slots);
    } else {
      auto kern = P1 <= 16 ? k_m2l_mb<1, E> : P1 <= 32 ? k_m2l_mb<2, E>
                : P1 <= 48 ? k_m2l_mb<3, E> : k_m2l_mb<4, E>;
      hipLaunchKernelGGL(kern, dim3((uint32_t)ctx->n_m2l_items, slots), dim3(64), 0, st,
                         d.m2l_item, d.m2l_pr, d.m2l_plog, M, X.m2l_bt, X.opow, P1, L, S.box);
    }
    if (ctx->n_p2l_boxes > 0) {
      if (use_p2x_mfma<KIND, E>(nd, P1)) {
        auto kp = p2x_kernel<1, E>(P1);
        hipLaunchKernelGGL(kp, dim3((uint32_t)ctx->n_p2l_boxes, (nd + 63) / 64), dim3(256), 0,
                           st, (int32_t)ctx->n_p2l_boxes, d.p2l_item, d.p2l_src, d.bc, d.blevel, d.level_inv_side,
                           d.level_log_side, d.sxy, d.snrm, d.sq, P1, L, nullptr, S.src, S.box,
                           (int64_t)0, nd,
                           (int64_t)nd * S.box);
      } else {
        auto kp = P1 <= 8 ? k_p2l<PK, 1, E> : P1 <= 16 ? k_p2l<PK, 2, E>
                : P1 <= 32 ? k_p2l<PK, 4, E> : k_p2l<PK, 8, E>;
        hipLaunchKernelGGL(kp, dim3((uint32_t)ctx->n_p2l_boxes, nd), dim3(64), 0, st, d.p2l_item,
                           d.p2l_src, d.bc, d.blevel, d.level_inv_side, d.level_log_side, d.sxy,
                           d.sq, d.sdip, P1, L, S.src, S.box, (int64_t)nd * S.box);
      }
    }
  }
  if (ctx->n_l2g_sinks > 0) {
    StageTimer st_(ctx, GQ_STAGE_L2L);
    if (slots >= kSlotGemmMin) {
      const int nw = std::min(4, (slots + 7) / 8);
      auto kern = P1 <= 16 ? k_l2l_slots<1, E> : P1 <= 32 ? k_l2l_slots<2, E>
                : P1 <= 48 ? k_l2l_slots<3, E> : k_l2l_slots<4, E>;
      hipLaunchKernelGGL(kern, dim3((uint32_t)ctx->n_l2g_items, (slots + 8 * nw - 1) / (8 * nw)),
                         dim3(64 * nw), 0, st, (int32_t)ctx->n_l2g_items, d.l2g_item, d.l2g_pr, d.l2g_tw, d.l2g_binom_t, P1,
                         L, Lf, S.box, slots);
    } else {
      auto kern = P1 <= 16 ? k_l2l_gather<1, E> : P1 <= 32 ? k_l2l_gather<2, E>
                : P1 <= 48 ? k_l2l_gather<3, E> : k_l2l_gather<4, E>;
      hipLaunchKernelGGL(kern, dim3((uint32_t)ctx->n_l2g_items, slots), dim3(64), 0, st,
                         d.l2g_item, d.l2g_pr, d.l2g_tw, d.l2g_binom_t, P1, L, Lf, S.box);
    }
  }
  e = hipStreamWaitEvent(st, ctx->ev_join, 0);
  if (e != hipSuccess) return e;
  if (ctr_vals) {
    StageTimer st_(ctx, GQ_STAGE_QBX_CENTER);
    for (const OrderBucket &bk : ctx->buckets) {
      switch (bk.pq) {
#define GQ_CASE(P) \
  case P: launch_ctr_val_bucket<P, E>(ctx, bk, slots, st, S, M, Lf); break;
        GQ_PQ_LIST(GQ_CASE)
#undef GQ_CASE
      }
    }
  } else {
    StageTimer st_(ctx, GQ_STAGE_QBX_CENTER);
    const int32_t *nvc = qvals ? d.n_chunks : near_values(ctx, nd, KIND) ? d.n_near_chunks : nullptr;
    for (const OrderBucket &bk : ctx->buckets) {
      switch (bk.pq) {
#define GQ_CASE(P) \
  case P: launch_center_bucket<CK, P, E>(ctx, bk, slots, st, S, Lf, nvc); break;
        GQ_PQ_LIST(GQ_CASE)
#undef GQ_CASE
      }
    }
  }
  return hipGetLastError();
}

template <int KIND>
hipError_t launch_fmm(gq_ctx *ctx, int nd) {
  return ctx->params.precision == GQ_MIXED_FP32 ? launch_fmm_t<KIND, float2>(ctx, nd)
                                                : launch_fmm_t<KIND, double2>(ctx, nd);
}

template <int KIND, int PQ>
void launch_direct(gq_ctx *ctx, const OrderBucket &bk, int nd, const Strides &S) {
  auto &d = ctx->d;
  const int32_t n = (int32_t)(bk.ctr1 - bk.ctr0);
  if (n > 0)
    hipLaunchKernelGGL((k_direct<KIND, PQ>), dim3((n + 255) / 256, nd), dim3(256), 0, ctx->stream,
                       n, d.ctr_list + bk.ctr0, d.cxy, d.cr, (int32_t)ctx->ns, d.sxy, d.sq, d.sdip,
                       d.c2t_start, d.c2t_slot, d.txy, d.tv, S.src, S.tv,
                       ctx->eval_sp ? ctx->tnrm_dev : nullptr);
}

// Direct QBX at each center's box order (the same effective orders as the FMM path).
template <int KIND>
hipError_t dispatch_direct(gq_ctx *ctx, int nd) {
  const Strides S = strides(ctx);
  StageTimer st_(ctx, GQ_STAGE_DIRECT);
  for (const OrderBucket &bk : ctx->buckets) {
    switch (bk.pq) {
#define GQ_CASE(P) \
  case P: launch_direct<KIND, P>(ctx, bk, nd, S); break;
      GQ_PQ_LIST(GQ_CASE)
#undef GQ_CASE
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace

const std::vector<int> &compiled_pq() {
  static const std::vector<int> v = {
#define GQ_CASE(P) P,
      GQ_PQ_LIST(GQ_CASE)
#undef GQ_CASE
  };
  return v;
}

bool pq_supported(int pq) {
  switch (pq) {
#define GQ_CASE(P) case P:
    GQ_PQ_LIST(GQ_CASE)
#undef GQ_CASE
    return true;
  }
  return false;
}

hipError_t upload_log_table() {
  double2 tab[kLogTab];
  for (int j = 0; j < kLogTab; ++j) {
    const long double mj = 1.0L + ((long double)j + 0.5L) / kLogTab;
    const double c = (double)(1.0L / mj);
    tab[j] = make_double2(c, (double)(-std::log((long double)c)));
  }
  return hipMemcpyToSymbol(HIP_SYMBOL(g_log_tab), tab, sizeof(tab), 0, hipMemcpyHostToDevice);
}

hipError_t run_math(int fn, int64_t n, const double *x, double *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_math, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, fn, n, x, out);
  return hipGetLastError();
}

hipError_t run_eval(gq_ctx *ctx, int kind, const double *d1, int64_t ld1, const double *d2,
                    int64_t ld2, double *out, int64_t ld_out, int nd, bool direct, double *out2) {
  hipError_t e;
  // GQ_SP: the expansions of S, differentiated along the target normals where they are evaluated
  struct SpFlag {
    gq_ctx *c;
    ~SpFlag() { c->eval_sp = false; }
  } sp_{ctx};
  ctx->eval_sp = kind == 5;
  if (kind == 5) kind = 1;
  ctx->cur_kind = kind == 4 ? 1 : kind;
  if (kind == 4) {  // S and D of the same densities through one expansion pipeline
    if (direct || !out2) return hipErrorInvalidValue;
    e = launch_gather<4>(ctx, d1, ld1, nullptr, 0, nd);
    if (e != hipSuccess) return e;
    e = launch_fmm<4>(ctx, nd);
    if (e != hipSuccess) return e;
    const int32_t nt = (int32_t)ctx->nt;
    StageTimer st_(ctx, GQ_STAGE_FINALIZE);
    hipLaunchKernelGGL(k_finalize, dim3((nt + 255) / 256, 2 * nd), dim3(256), 0, ctx->stream, nt,
                       ctx->d.tctr, ctx->d.tv, out, 2 * ctx->nt, ld_out, out2, nd);
    return hipGetLastError();
  }
  switch (kind) {
    case 1: e = launch_gather<1>(ctx, d1, ld1, d2, ld2, nd); break;
    case 2: e = launch_gather<2>(ctx, d1, ld1, d2, ld2, nd); break;
    case 3: e = launch_gather<3>(ctx, d1, ld1, d2, ld2, nd); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (direct) {
    switch (kind) {
      case 1: e = dispatch_direct<1>(ctx, nd); break;
      case 2: e = dispatch_direct<2>(ctx, nd); break;
      case 3: e = dispatch_direct<3>(ctx, nd); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (kind) {
      case 1: e = launch_fmm<1>(ctx, nd); break;
      case 2: e = launch_fmm<2>(ctx, nd); break;
      case 3: e = launch_fmm<3>(ctx, nd); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  const int32_t nt = (int32_t)ctx->nt;
  StageTimer st_(ctx, GQ_STAGE_FINALIZE);
  hipLaunchKernelGGL(k_finalize, dim3((nt + 255) / 256, nd), dim3(256), 0, ctx->stream, nt,
                     ctx->d.tctr, ctx->d.tv, out, 2 * ctx->nt, ld_out, nullptr, nd);
  return hipGetLastError();
}

}  // namespace gq
