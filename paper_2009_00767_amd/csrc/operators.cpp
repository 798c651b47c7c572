// operators.cpp -- multipole-to-local operators, built once per plan in FP64.
//
// The bilinear form B_{m_i,m}(v_{m_i}, v) of Section 2.2.1 between a source box
// and a target box of its interaction list depends only on their offset once the
// box vectors are expressed in box-size-scaled coordinates; it is built here in
// double precision (Discussion (3)) before any evaluation (Discussion (2)) and
// rounded once to the working precision.
//
// 2D (G = log r).  Source coefficients A_m about the source centre, target
// coefficients B_l about the target centre, both scaled by the box side s, and
// u = (z_source - z_target)/s a Gaussian integer with max(|Re u|, |Im u|) in {2, 3}.
// Greengard's multipole-to-local lemma in these variables gives
//   B_0 += A_0 (log(-u) + log s) + sum_{m>=1} (-1)^m u^-m A_m
//   B_l += -A_0 / (l u^l) + sum_{m>=1} (-1)^m C(l+m-1, m-1) u^-(l+m) A_m
// The log s term depends on the level and is applied by the kernel.
//
// Coefficient layout of a box (both moments and locals): real and imaginary
// parts of coefficients 1..p at 2(m-1) and 2(m-1)+1, then coefficient 0 at 2p
// and 2p+1, padded to a multiple of 4 values.
//
// Operator pack per offset slot (dx + 3) + 7 (dy + 3), in the order
//   Wb[Npad][Kpad]  real form of T[l][m], l, m >= 1: entry [j][k] multiplies
//                   input value k into output value j (j, k in the layout above)
//   c0[Npad]        contribution of Re A_0 to output j (A_0 is real)
//   r0[Kpad]        contribution of input k to Re B_0
//   t00, pad[3]     contribution of Re A_0 to Re B_0 (Re log(-u))
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

M2lLayout m2l2d_layout(int pb) {
  const int p = pb;
  M2lLayout L{};
  L.p = pb;
  L.kpad = (2 * p + 3) / 4 * 4;
  L.npad = (2 * p + 15) / 16 * 16;
  L.stride = L.npad * L.kpad + L.npad + L.kpad + 4;
  L.cs = (2 * p + 2 + 3) / 4 * 4;
  return L;
}

void build_m2l2d_operators(int p, const M2lLayout& L, double* out) {
  for (int dy = -3; dy <= 3; ++dy)
    for (int dx = -3; dx <= 3; ++dx) {
      const int slot = (dx + 3) + 7 * (dy + 3);
      double* W = out + (size_t)slot * L.stride;
      double* c0 = W + L.npad * L.kpad;
      double* r0 = c0 + L.npad;
      double* t00 = r0 + L.kpad;
      for (int i = 0; i < L.stride; ++i) W[i] = 0.0;
      if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;  // adjacent: never in a list
      const cd u(dx, dy);
      std::vector<cd> uinv(2 * p + 1);
      uinv[0] = 1.0;
      const cd ui = 1.0 / u;
      for (int k = 1; k <= 2 * p; ++k) uinv[k] = uinv[k - 1] * ui;
      // T[l][m] for l, m >= 1: real 2x2 blocks [[Tr, -Ti], [Ti, Tr]]
      for (int l = 1; l <= p; ++l)
        for (int m = 1; m <= p; ++m) {
          const cd t = (m & 1 ? -1.0 : 1.0) * binomial(l + m - 1, m - 1) * uinv[l + m];
          const int jr = 2 * (l - 1), kr = 2 * (m - 1);
          W[(jr)*L.kpad + kr] = t.real();
          W[(jr)*L.kpad + kr + 1] = -t.imag();
          W[(jr + 1) * L.kpad + kr] = t.imag();
          W[(jr + 1) * L.kpad + kr + 1] = t.real();
        }
      // T[l][0] = -1/(l u^l), l >= 1, times the real A_0
      for (int l = 1; l <= p; ++l) {
        const cd t = -uinv[l] / double(l);
        c0[2 * (l - 1)] = t.real();
        c0[2 * (l - 1) + 1] = t.imag();
      }
      // Re B_0 from A_m, m >= 1: Re(T[0][m] A_m) = Tr Ar - Ti Ai
      for (int m = 1; m <= p; ++m) {
        const cd t = (m & 1 ? -1.0 : 1.0) * uinv[m];
        r0[2 * (m - 1)] = t.real();
        r0[2 * (m - 1) + 1] = -t.imag();
      }
      t00[0] = std::log(-u).real();
    }
}

}  // namespace sffmm
