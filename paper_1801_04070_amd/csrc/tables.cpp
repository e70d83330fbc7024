// Fixed translation tables for scaled expansions (see tables.hpp for the scaling and the reading
// of eq. (m2l)). Computed once per FMM order in long double and rounded to FP64.
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <complex>

namespace gq {

using cld = std::complex<long double>;

void build_tables(Tables &t, int p, int max_pq) {
  t = Tables();
  t.p = p;
  const int P1 = p + 1;
  const int NB = std::max(2 * p + 2, p + max_pq + 2);
  t.nbinom = NB;
  t.binom.assign((size_t)NB * NB, 0.0);
  std::vector<long double> pas((size_t)NB * NB, 0.0L);
  for (int n = 0; n < NB; ++n) {
    pas[(size_t)n * NB] = 1.0L;
    for (int k = 1; k <= n; ++k)
      pas[(size_t)n * NB + k] = pas[(size_t)(n - 1) * NB + k - 1] + (k <= n - 1 ? pas[(size_t)(n - 1) * NB + k] : 0.0L);
  }
  for (size_t i = 0; i < pas.size(); ++i) t.binom[i] = (double)pas[i];
  auto C = [&](int n, int k) -> long double {
    if (k < 0 || n < 0 || k > n) return 0.0L;
    return pas[(size_t)n * NB + k];
  };
  auto cpow = [](cld z, int n) {
    cld r(1.0L, 0.0L);
    for (int i = 0; i < n; ++i) r *= z;
    return r;
  };

  // M2L factor B, eq. (m2l) with the corrected sign of the a_0 term
  t.m2l_b.assign((size_t)P1 * P1, 0.0);
  for (int m = 0; m <= p; ++m)
    for (int k = 0; k <= p; ++k) {
      long double v;
      if (m == 0) v = (k == 0) ? 0.0L : 1.0L;
      else if (k == 0) v = ((m % 2) ? 1.0L : -1.0L) / (long double)m;
      else v = ((m % 2) ? -1.0L : 1.0L) * C(m + k - 1, k - 1);
      t.m2l_b[(size_t)m * P1 + k] = (double)v;
    }
  t.m2l_bt.assign((size_t)P1 * P1, 0.0);
  for (int m = 0; m <= p; ++m)
    for (int k = 0; k <= p; ++k) t.m2l_bt[(size_t)k * P1 + m] = t.m2l_b[(size_t)m * P1 + k];

  t.opow.assign((size_t)121 * P1 * 2, 0.0);
  t.ologabs.assign(121, 0.0);
  for (int i = 0; i < 11; ++i)
    for (int j = 0; j < 11; ++j) {
      const int oi = i * 11 + j;
      const long double ox = i - 5, oy = j - 5;
      if (std::max(std::fabs(ox), std::fabs(oy)) < 3) continue;  // never a List-2 offset
      const cld inv = 1.0L / cld(ox, oy);
      cld pw(1.0L);
      for (int k = 0; k <= p; ++k) {
        t.opow[((size_t)oi * P1 + k) * 2] = (double)pw.real();
        t.opow[((size_t)oi * P1 + k) * 2 + 1] = (double)pw.imag();
        pw *= inv;
      }
      t.ologabs[oi] = (double)(0.5L * std::log(ox * ox + oy * oy));
    }
}

}  // namespace gq
