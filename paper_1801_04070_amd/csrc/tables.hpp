// Fixed translation tables for scaled expansions (host side).
//
// Every box expansion is stored with coefficients scaled by powers of the box side s:
//   multipole  M_b(z) = a_0 log(z - c_b) + sum_k a_k (z - c_b)^-k,   stored as  a_k / s^k
//   local      L_b(z) = sum_k b_k (z - c_b)^k,                       stored as  b_k s^k
// With this scaling the translations of Sec. 3.1 become level independent:
//   multipoles are formed directly from each box's subtree sources (the M2M of eq. (m2m) keeps
//   the first p + 1 moments exact in 2-D, so no table is needed);
//   L2L (eq. l2l) from an ancestor across any level gap: a fixed binomial matrix between
//   diagonal factors of the shift (applied on the device);
//   M2L (eq. m2l, with the sign of the a_0 term corrected, see below) between same-level boxes at
//   integer offset o = (c_local - c_multipole)/s factors as diag(o^-m) B diag(o^-k) with a fixed
//   real matrix B; the log term a_0 log|s o| is added to the 0-th coefficient.
// Reading of eq. (m2l): expanding log(y + w) = log y + sum_m (-1)^(m+1) w^m / (m y^m) gives the
// a_0 contribution (-1)^m (-a_0 / (m y^m)) to beta_m; the paper's printed "+a_0/(m y^m)" has the
// opposite sign. The a_k terms and beta_0 are as printed.
#pragma once

#include <vector>

namespace gq {

// Real matrices are stored transposed ([k][m]) so that lanes indexed by m read consecutive words.
struct Tables {
  int p = 0;                      // FMM order; arrays use P1 = p + 1 coefficients
  std::vector<double> m2l_bt;     // [P1 (k)][P1 (m)] real B, transposed
  std::vector<double> m2l_b;      // [P1][P1] real B
  std::vector<double> opow;       // [121][P1] complex: o^-k for o = (i - 5) + (j - 5) i, index i*11+j
  std::vector<double> ologabs;    // [121] log|o|
  int nbinom = 0;                 // rows of the Pascal triangle
  std::vector<double> binom;      // [nbinom][nbinom] Pascal triangle C(n, k)
};

// Tables for FMM order p; the Pascal triangle covers C(n, k) for n < p + max_pq + 2 as well.
void build_tables(Tables &t, int p, int max_pq);

}  // namespace gq
