/*
 * Oracle for 2-D Laplace layer potentials evaluated by QBX -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of what the accelerated method
 * approximates: unaccelerated ("direct") global QBX with brute-force expansion formation.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * this library; the GPU library never calls it and shares no code with it.
 *
 * Definitions followed (Wala & Kloeckner, "A Fast Algorithm with Error Bounds for Quadrature
 * by Expansion"):
 *   - single/double layer potentials: Sec. 1, eqs. (slp-definition), (dlp-definition)
 *       S mu(x) = -1/(2 pi) int mu(y) log|y - x| ds(y)
 *       D mu(x) = -1/(2 pi) int mu(y) n(y) . grad_y log|y - x| ds(y)
 *   - identification R^2 = C and Re log z = log|z|: Sec. 2.1
 *   - QBX formula S_QBX(p, N): Sec. 2.1, eq. (qbx): the p-th order Taylor expansion of the
 *     quadrature-discretised potential about a center c, evaluated at the target x.
 *   - multipole / local expansions of a unit source: Sec. 3.1, eqs. (multipole), (local).
 *
 * Readings (stated once here, also listed in the design notes):
 *   - Only Re of any complex logarithm is physical; the oracle keeps log|.| and never forms the
 *     imaginary part (it would only enter Im of the 0-th coefficient, which is discarded).
 *   - The double-layer kernel in complex form: n . grad_y log|y - x| = Re( n / (y - x) ), n the
 *     unit normal as a complex number; its Taylor coefficients about c are n / (y - c)^(m+1).
 *   - kind 3 is the Green's-formula combination S(sigma) - D(tau) with two densities.
 *
 * Sums over sources use Neumaier-compensated FP64 accumulation so that the oracle's rounding
 * error stays far below the 1e-10 parity tolerance.
 *
 * Array conventions: points and normals are (n, 2) row-major interleaved (x, y); complex
 * coefficients are (.., p+1) interleaved (re, im); target-center association is (n_tgt, 2)
 * int32 with -1 meaning "no center" (a target with no center is a conventional point target
 * and gets the plain quadrature sum).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_S 1
#define ORACLE_D 2
#define ORACLE_S_MINUS_D 3

typedef double complex cplx;

/* Neumaier compensated sum. */
typedef struct { double s, c; } ksum;
static inline void ks_add(ksum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static inline double ks_val(const ksum *a) { return a->s + a->c; }

/* Per-source charge q (single layer) and dipole strength delta (double layer) for a kind. */
static int source_strengths(int kind, int64_t i, const double *w, const double *d1,
                            const double *d2, double *q, double *delta) {
  switch (kind) {
    case ORACLE_S: *q = w[i] * d1[i]; *delta = 0.0; return 0;
    case ORACLE_D: *q = 0.0; *delta = w[i] * d1[i]; return 0;
    case ORACLE_S_MINUS_D: *q = w[i] * d1[i]; *delta = -w[i] * d2[i]; return 0;
    default: return -1;
  }
}

static inline cplx pt(const double *xy, int64_t i) { return xy[2 * i] + I * xy[2 * i + 1]; }

/*
 * QBX local coefficients about center c, eq. (qbx): alpha_m = sum_i w_i mu_i (1/m!) d^m/dc^m
 * log(y_i - c). For a charge: alpha_0 = q log|y - c|, alpha_m = -q / (m (y - c)^m).
 * For a dipole of strength delta along normal n: alpha_m = delta n / (y - c)^(m+1).
 * These are also the coefficients of eq. (local) about c with z0 = y - c.
 */
static void qbx_coeffs_one(int kind, int64_t n_src, const double *src_xy, const double *src_nrm,
                           const double *src_w, const double *d1, const double *d2, cplx c,
                           int p, cplx *alpha) {
  ksum *acc = (ksum *)calloc((size_t)2 * (p + 1), sizeof(ksum));
  for (int64_t i = 0; i < n_src; ++i) {
    double q, delta;
    source_strengths(kind, i, src_w, d1, d2, &q, &delta);
    cplx z = pt(src_xy, i) - c;          /* y_i - c */
    cplx inv = 1.0 / z;
    cplx nrm = pt(src_nrm, i);
    if (q != 0.0) {
      ks_add(&acc[0], q * log(cabs(z)));
      cplx pw = 1.0;
      for (int m = 1; m <= p; ++m) {
        pw *= inv;                       /* (y - c)^-m */
        cplx t = -q * pw / (double)m;
        ks_add(&acc[2 * m], creal(t));
        ks_add(&acc[2 * m + 1], cimag(t));
      }
    }
    if (delta != 0.0) {
      cplx pw = inv;                     /* (y - c)^-(m+1) at m = 0 */
      for (int m = 0; m <= p; ++m) {
        cplx t = delta * nrm * pw;
        ks_add(&acc[2 * m], creal(t));
        ks_add(&acc[2 * m + 1], cimag(t));
        pw *= inv;
      }
    }
  }
  for (int m = 0; m <= p; ++m) alpha[m] = ks_val(&acc[2 * m]) + I * ks_val(&acc[2 * m + 1]);
  free(acc);
}

/* -1/(2 pi) Re sum_m alpha_m (x - c)^m : the QBX local expansion evaluated at x. */
static double eval_local_at(int p, const cplx *alpha, cplx c, cplx x) {
  ksum s = {0, 0};
  cplx pw = 1.0, dz = x - c;
  for (int m = 0; m <= p; ++m) {
    ks_add(&s, creal(alpha[m] * pw));
    pw *= dz;
  }
  return -ks_val(&s) / (2.0 * M_PI);
}

/* Plain quadrature (point) potential at x: -1/(2 pi) sum_i [q_i log|y_i - x| + delta_i Re(n_i/(y_i - x))]. */
static double point_potential_at(int kind, int64_t n_src, const double *src_xy,
                                 const double *src_nrm, const double *src_w, const double *d1,
                                 const double *d2, cplx x) {
  ksum s = {0, 0};
  for (int64_t i = 0; i < n_src; ++i) {
    double q, delta;
    source_strengths(kind, i, src_w, d1, d2, &q, &delta);
    cplx z = pt(src_xy, i) - x;
    if (q != 0.0) ks_add(&s, q * log(cabs(z)));
    if (delta != 0.0) ks_add(&s, delta * creal(pt(src_nrm, i) / z));
  }
  return -ks_val(&s) / (2.0 * M_PI);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* QBX coefficients alpha_m (unscaled, m = 0..p) for every center. coef: n_ctr x (p+1) x 2. */
int oracle_qbx_coeffs(int kind, int64_t n_src, const double *src_xy, const double *src_nrm,
                      const double *src_w, const double *dens1, const double *dens2,
                      int64_t n_ctr, const double *ctr_xy, int p, double *coef) {
  if (kind < ORACLE_S || kind > ORACLE_S_MINUS_D || p < 0 || n_src < 0 || n_ctr < 0) return -1;
  if (kind == ORACLE_S_MINUS_D && !dens2) return -1;
  int fail = 0;
#pragma omp parallel
  {
    cplx *alpha = (cplx *)malloc(sizeof(cplx) * (size_t)(p + 1));
    if (!alpha) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 4)
    for (int64_t j = 0; j < n_ctr; ++j) {
      if (!alpha) continue;
      qbx_coeffs_one(kind, n_src, src_xy, src_nrm, src_w, dens1, dens2, pt(ctr_xy, j), p, alpha);
      for (int m = 0; m <= p; ++m) {
        coef[(j * (p + 1) + m) * 2] = creal(alpha[m]);
        coef[(j * (p + 1) + m) * 2 + 1] = cimag(alpha[m]);
      }
    }
    free(alpha);
  }
  return fail ? -2 : 0;
}

/*
 * Direct QBX evaluation at targets. Each target averages the expansions of its (one or two)
 * associated centers; a target with no center gets the plain quadrature sum.
 */
int oracle_qbx_eval(int kind, int64_t n_src, const double *src_xy, const double *src_nrm,
                    const double *src_w, const double *dens1, const double *dens2,
                    int64_t n_ctr, const double *ctr_xy, int p, int64_t n_tgt,
                    const double *tgt_xy, const int32_t *tgt_ctr, double *out) {
  if (kind < ORACLE_S || kind > ORACLE_S_MINUS_D || p < 0 || n_src < 0 || n_tgt < 0) return -1;
  if (kind == ORACLE_S_MINUS_D && !dens2) return -1;
  for (int64_t t = 0; t < n_tgt; ++t)
    for (int s = 0; s < 2; ++s)
      if (tgt_ctr[2 * t + s] >= n_ctr) return -1;
  int fail = 0;
#pragma omp parallel
  {
    cplx *alpha = (cplx *)malloc(sizeof(cplx) * (size_t)(p + 1));
    if (!alpha) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < n_tgt; ++t) {
      if (!alpha) continue;
      cplx x = pt(tgt_xy, t);
      double sum = 0.0;
      int used = 0;
      for (int s = 0; s < 2; ++s) {
        int32_t j = tgt_ctr[2 * t + s];
        if (j < 0) continue;
        cplx c = pt(ctr_xy, j);
        qbx_coeffs_one(kind, n_src, src_xy, src_nrm, src_w, dens1, dens2, c, p, alpha);
        sum += eval_local_at(p, alpha, c, x);
        used++;
      }
      out[t] = used ? sum / used
                    : point_potential_at(kind, n_src, src_xy, src_nrm, src_w, dens1, dens2, x);
    }
    free(alpha);
  }
  return fail ? -2 : 0;
}

/*
 * S' (the normal derivative of the single layer potential at a target, n(x) . grad_x S mu(x),
 * the operator of Sec. 1, eq. (ext-neumann-ie)) by direct QBX. The potential near the target is
 * u(x) = -1/(2 pi) Re F(x), F(x) = sum_m alpha_m (x - c)^m the expansion of eq. (qbx) about an
 * associated center; F is analytic, so with nu = n_x + i n_y,
 *   n . grad u = -1/(2 pi) Re( nu F'(x) ),  F'(x) = sum_{m>=1} m alpha_m (x - c)^(m-1).
 * Targets average their centers' values; a target with no center takes the plain quadrature sum
 * -1/(2 pi) sum_i q_i Re( nu / (x - y_i) ) (the gradient of log|x - y| is 1/(x - y) conjugated).
 */
static double eval_local_deriv_at(int p, const cplx *alpha, cplx c, cplx x, cplx nu) {
  ksum s = {0, 0};
  cplx pw = 1.0, dz = x - c;
  for (int m = 1; m <= p; ++m) {
    ks_add(&s, creal(nu * (double)m * alpha[m] * pw));
    pw *= dz;
  }
  return -ks_val(&s) / (2.0 * M_PI);
}

int oracle_qbx_normal_derivative(int64_t n_src, const double *src_xy, const double *src_nrm,
                                 const double *src_w, const double *dens, int64_t n_ctr,
                                 const double *ctr_xy, int p, int64_t n_tgt,
                                 const double *tgt_xy, const double *tgt_nrm,
                                 const int32_t *tgt_ctr, double *out) {
  if (p < 0 || n_src < 0 || n_tgt < 0) return -1;
  for (int64_t t = 0; t < n_tgt; ++t)
    for (int s = 0; s < 2; ++s)
      if (tgt_ctr[2 * t + s] >= n_ctr) return -1;
  int fail = 0;
#pragma omp parallel
  {
    cplx *alpha = (cplx *)malloc(sizeof(cplx) * (size_t)(p + 1));
    if (!alpha) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < n_tgt; ++t) {
      if (!alpha) continue;
      cplx x = pt(tgt_xy, t), nu = pt(tgt_nrm, t);
      double sum = 0.0;
      int used = 0;
      for (int s = 0; s < 2; ++s) {
        int32_t j = tgt_ctr[2 * t + s];
        if (j < 0) continue;
        cplx c = pt(ctr_xy, j);
        qbx_coeffs_one(ORACLE_S, n_src, src_xy, src_nrm, src_w, dens, NULL, c, p, alpha);
        sum += eval_local_deriv_at(p, alpha, c, x, nu);
        used++;
      }
      if (used) {
        out[t] = sum / used;
      } else {
        ksum a = {0, 0};
        for (int64_t i = 0; i < n_src; ++i)
          ks_add(&a, src_w[i] * dens[i] * creal(nu / (x - pt(src_xy, i))));
        out[t] = -ks_val(&a) / (2.0 * M_PI);
      }
    }
    free(alpha);
  }
  return fail ? -2 : 0;
}

/* Plain quadrature potential at arbitrary points (no QBX). */
int oracle_point_potential(int kind, int64_t n_src, const double *src_xy, const double *src_nrm,
                           const double *src_w, const double *dens1, const double *dens2,
                           int64_t n_tgt, const double *tgt_xy, double *out) {
  if (kind < ORACLE_S || kind > ORACLE_S_MINUS_D || n_src < 0 || n_tgt < 0) return -1;
  if (kind == ORACLE_S_MINUS_D && !dens2) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < n_tgt; ++t)
    out[t] = point_potential_at(kind, n_src, src_xy, src_nrm, src_w, dens1, dens2, pt(tgt_xy, t));
  return 0;
}

/*
 * Multipole expansion about center (cx, cy), eq. (multipole) summed over sources:
 * phi(z) = a_0 log(z - c) + sum_k a_k / (z - c)^k with, for a charge q at y,
 * a_0 = q, a_k = -q (y - c)^k / k, and for a dipole delta n at y, a_k = -delta n (y - c)^(k-1).
 */
int oracle_multipole(int kind, int64_t n_src, const double *src_xy, const double *src_nrm,
                     const double *src_w, const double *dens1, const double *dens2, double cx,
                     double cy, int p, double *coef) {
  if (kind < ORACLE_S || kind > ORACLE_S_MINUS_D || p < 0) return -1;
  if (kind == ORACLE_S_MINUS_D && !dens2) return -1;
  ksum *acc = (ksum *)calloc((size_t)2 * (p + 1), sizeof(ksum));
  if (!acc) return -2;
  cplx c = cx + I * cy;
  for (int64_t i = 0; i < n_src; ++i) {
    double q, delta;
    source_strengths(kind, i, src_w, dens1, dens2, &q, &delta);
    cplx y = pt(src_xy, i) - c, nrm = pt(src_nrm, i);
    ks_add(&acc[0], q);
    cplx pw = 1.0;                       /* (y - c)^(k-1) */
    for (int k = 1; k <= p; ++k) {
      cplx t = -delta * nrm * pw;
      pw *= y;                           /* (y - c)^k */
      t += -q * pw / (double)k;
      ks_add(&acc[2 * k], creal(t));
      ks_add(&acc[2 * k + 1], cimag(t));
    }
  }
  for (int k = 0; k <= p; ++k) {
    coef[2 * k] = ks_val(&acc[2 * k]);
    coef[2 * k + 1] = ks_val(&acc[2 * k + 1]);
  }
  free(acc);
  return 0;
}

/* Local (Taylor) expansion about (cx, cy), eq. (local), summed over sources (Re of b_0 only). */
int oracle_local(int kind, int64_t n_src, const double *src_xy, const double *src_nrm,
                 const double *src_w, const double *dens1, const double *dens2, double cx,
                 double cy, int p, double *coef) {
  if (kind < ORACLE_S || kind > ORACLE_S_MINUS_D || p < 0) return -1;
  if (kind == ORACLE_S_MINUS_D && !dens2) return -1;
  cplx *alpha = (cplx *)malloc(sizeof(cplx) * (size_t)(p + 1));
  if (!alpha) return -2;
  qbx_coeffs_one(kind, n_src, src_xy, src_nrm, src_w, dens1, dens2, cx + I * cy, p, alpha);
  for (int k = 0; k <= p; ++k) {
    coef[2 * k] = creal(alpha[k]);
    coef[2 * k + 1] = cimag(alpha[k]);
  }
  free(alpha);
  return 0;
}

/* -1/(2 pi) Re[a_0 log(z - c) + sum_k a_k (z - c)^-k] at each point. */
int oracle_eval_multipole(int p, const double *coef, double cx, double cy, int64_t n,
                          const double *xy, double *out) {
  cplx c = cx + I * cy;
  for (int64_t t = 0; t < n; ++t) {
    cplx z = pt(xy, t) - c, inv = 1.0 / z, pw = 1.0;
    ksum s = {0, 0};
    ks_add(&s, coef[0] * log(cabs(z)));
    for (int k = 1; k <= p; ++k) {
      pw *= inv;
      ks_add(&s, creal((coef[2 * k] + I * coef[2 * k + 1]) * pw));
    }
    out[t] = -ks_val(&s) / (2.0 * M_PI);
  }
  return 0;
}

/* -1/(2 pi) Re sum_k b_k (z - c)^k at each point. */
int oracle_eval_local(int p, const double *coef, double cx, double cy, int64_t n,
                      const double *xy, double *out) {
  cplx c = cx + I * cy;
  cplx *b = (cplx *)malloc(sizeof(cplx) * (size_t)(p + 1));
  if (!b) return -2;
  for (int k = 0; k <= p; ++k) b[k] = coef[2 * k] + I * coef[2 * k + 1];
  for (int64_t t = 0; t < n; ++t) out[t] = eval_local_at(p, b, c, pt(xy, t));
  free(b);
  return 0;
}
