// operators.cpp -- multipole-to-local operators, built once per plan in FP64.
//
// The bilinear form B_{m_i,m}(v_{m_i}, v) of Section 2.2.1 between a source box
// and a target box of its interaction list depends only on their offset once the
// box vectors are expressed in box-size-scaled coordinates; it is built here in
// double precision (Discussion (3)) before any evaluation (Discussion (2)).
//
// 2D (G = log r).  Source coefficients A_m about the source centre, target
// coefficients B_l about the target centre, both scaled by the box side s, and
// u = (z_source - z_target)/s a Gaussian integer with max(|Re u|, |Im u|) in {2, 3}.
// Greengard's multipole-to-local lemma in these variables gives
//   B_0 += A_0 (log(-u) + log s) + sum_{m>=1} (-1)^m u^-m A_m
//   B_l += -A_0 / (l u^l) + sum_{m>=1} (-1)^m C(l+m-1, m-1) u^-(l+m) A_m
// The log s term depends on the level and is applied by the kernel.
#include <cmath>
#include <complex>
#include <vector>

#include "fmm_internal.h"

namespace sffmm {

using cd = std::complex<double>;

static double binomial(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double c = 1.0;
  for (int i = 1; i <= k; ++i) c *= double(n - k + i) / double(i);
  return c;
}

void build_m2l2d_operators(int p, double* out) {
  const int P = p + 1;
  for (int dy = -3; dy <= 3; ++dy)
    for (int dx = -3; dx <= 3; ++dx) {
      const int slot = (dx + 3) + 7 * (dy + 3);
      double* T = out + (size_t)slot * P * P * 2;
      for (int i = 0; i < P * P * 2; ++i) T[i] = 0.0;
      if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;  // adjacent: never in a list
      const cd u(dx, dy);
      std::vector<cd> uinv(2 * P + 1);
      uinv[0] = 1.0;
      const cd ui = 1.0 / u;
      for (int k = 1; k <= 2 * p; ++k) uinv[k] = uinv[k - 1] * ui;
      auto put = [&](int l, int m, cd v) {
        T[(l * P + m) * 2] = v.real();
        T[(l * P + m) * 2 + 1] = v.imag();
      };
      put(0, 0, std::log(-u));
      for (int m = 1; m <= p; ++m) put(0, m, (m & 1 ? -1.0 : 1.0) * uinv[m]);
      for (int l = 1; l <= p; ++l) {
        put(l, 0, -uinv[l] / double(l));
        for (int m = 1; m <= p; ++m)
          put(l, m, (m & 1 ? -1.0 : 1.0) * binomial(l + m - 1, m - 1) * uinv[l + m]);
      }
    }
}

}  // namespace sffmm
