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
#include <cstring>
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
  L.kbf = 32 * bf16_chunks(p);
  L.nbf = (1 + 2 * p + 15) / 16 * 16;
  const int ks = L.kpad / 4, nb = L.npad / 16;
  L.lstride = 64 * (nb * (ks + 1) + ks) + 4;
  L.l16 = (L.nbf / 16) * (L.kbf / 32) * 64 * 8;
  return L;
}

// Lane-major pack for the 16x16x4 MFMA steps (lane l: i = l % 16, g = l / 16),
// per slot:
//   B[nb][s][l], s < KS : Wb[16 nb + i][4 s + g]   (step s contracts K = 4s..4s+3)
//   B[nb][KS][l]        : c0[16 nb + i] for g = 0, else 0 (the A_0 step)
//   R[s][l], s < KS     : r0[4 s + g]                (this lane's Re B_0 weights)
//   t00, pad[3]
// so that every operator load of the kernel is one coalesced dword per lane.
void build_m2l2d_lane_pack(const M2lLayout& L, const double* pack, double* out) {
  const int ks = L.kpad / 4, nbk = L.npad / 16;
  for (int slot = 0; slot < 49; ++slot) {
    const double* W = pack + (size_t)slot * L.stride;
    const double* c0 = W + L.npad * L.kpad;
    const double* r0 = c0 + L.npad;
    double* o = out + (size_t)slot * L.lstride;
    for (int nb = 0; nb < nbk; ++nb)
      for (int st = 0; st <= ks; ++st)
        for (int l = 0; l < 64; ++l) {
          const int i = l & 15, g = l >> 4;
          o[((size_t)nb * (ks + 1) + st) * 64 + l] =
              st < ks ? W[(size_t)(16 * nb + i) * L.kpad + 4 * st + g]
                      : (g == 0 ? c0[16 * nb + i] : 0.0);
        }
    double* R = o + (size_t)nbk * (ks + 1) * 64;
    for (int st = 0; st < ks; ++st)
      for (int l = 0; l < 64; ++l) R[(size_t)st * 64 + l] = r0[4 * st + (l >> 4)];
    double* t = R + (size_t)ks * 64;
    t[0] = r0[L.kpad];
    t[1] = t[2] = t[3] = 0.0;
  }
}

// Round-to-nearest-even FP32 -> BF16 (finite inputs), as a bit pattern.
static uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

static double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Lane-major BF16 pack for the 16x16x32 MFMA steps of the BF16 mode, per slot
// [nb][c][l][e] (lane l = 16 g + i): the K x N product matrix entry
// B[32 c + 8 g + e][16 nb + i].  N order: column 0 is Re B_0, column 1 + j
// output value j.  K order (the kernel stages its inputs in the same order):
//   0..5            the A_0 terms as cross products of three-part splits (input
//                   parts hi, hi, mid, hi, mid, lo against operator parts hi,
//                   mid, hi, lo, mid, hi)
//   6 + k           input value k (k < 2 pb), operator entry rounded once
//   6 + 2pb + v     the low part of input value v (v < 2 ms) against the high
//                   part of the operator entry
//   6 + 2pb + 2ms + v   the high part of input value v against the low part of
//                   the operator entry
// (ms = bf16_split(pb)): the leading coefficients, the largest terms after A_0,
// run as two-term splits on both sides.
void build_m2l2d_bf16(const M2lLayout& L, const double* pack, uint16_t* out) {
  const int nbk = L.nbf / 16, kc = L.kbf / 32, p2 = 2 * L.p, ms2 = 2 * bf16_split(L.p);
  static const int opart[6] = {0, 1, 0, 2, 1, 0};  // operator part per A_0 slot
  auto split3 = [](double v, uint16_t* h) {
    double r = v;
    for (int t = 0; t < 3; ++t) {
      h[t] = bf16_bits((float)r);
      r -= bf16_value(h[t]);
    }
  };
  for (int slot = 0; slot < 49; ++slot) {
    const double* W = pack + (size_t)slot * L.stride;
    const double* c0 = W + L.npad * L.kpad;
    const double* r0 = c0 + L.npad;
    const double t00 = r0[L.kpad];
    uint16_t* o = out + (size_t)slot * L.l16;
    for (int nb = 0; nb < nbk; ++nb)
      for (int c = 0; c < kc; ++c)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e) {
            const int i = l & 15, g = l >> 4, kq = 32 * c + 8 * g + e, col = 16 * nb + i;
            uint16_t v = 0;
            if (col <= p2) {
              // operator entry of input value k for this column
              auto entry = [&](int k) { return col == 0 ? r0[k] : W[(size_t)(col - 1) * L.kpad + k]; };
              uint16_t parts[3];
              if (kq < 6) {
                split3(col == 0 ? t00 : c0[col - 1], parts);
                v = parts[opart[kq]];
              } else if (kq < 6 + p2) {
                v = bf16_bits((float)entry(kq - 6));
              } else if (kq < 6 + p2 + ms2) {
                v = bf16_bits((float)entry(kq - 6 - p2));
              } else if (kq < 6 + p2 + 2 * ms2) {
                split3(entry(kq - 6 - p2 - ms2), parts);
                v = parts[1];
              }
            }
            o[(((size_t)nb * kc + c) * 64 + l) * 8 + e] = v;
          }
  }
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

// ---------------------------------------------------------------------------
// 3D (G = 1/r).  Solid harmonics with the Condon-Shortley phase,
//   R_n^m = r^n P_n^m(cos t) e^{i m f} / (n+m)!,  I_n^m = (n-m)! P_n^m e^{i m f} / r^{n+1},
// box-side-scaled moments M_n^m = sum q conj R_n^m((r - r_b)/s) and locals with
// potential (1/s) sum L_j^k R_j^k((r - r_t)/s).  With u = (r_b - r_t)/s:
//   L_j^k = (-1)^k sum_{n,m} (-1)^n M_n^m I_{j+n}^{m-k}(u),
// and M_n^-m = (-1)^m conj M_n^m, L_j^-k = (-1)^k conj L_j^k, so only m, k >= 0
// are stored: per degree n the real part of m = 0, then re/im of m = 1..n.
//
// Real layout of a box ((PB+1)^2 values, PB = order bucket): degree n >= 1 at
// n^2 - 1 (m = 0), n^2 - 1 + 2m - 1 (re, m >= 1), n^2 - 1 + 2m (im); the
// degree-0 value at (PB+1)^2 - 1; padded to a multiple of 4.
// Operator pack per offset slot (dx+3) + 7 (dy+3) + 49 (dz+3), as in 2D:
//   Wb[Npad][Kpad] (degrees >= 1 -> degrees >= 1), c0[Npad] (M_0^0 -> output j),
//   r0[Kpad] (input k -> L_0^0), t00 (M_0^0 -> L_0^0), pad.
// ---------------------------------------------------------------------------

static int ri3(int n, int m, int im) { return n * n - 1 + (m == 0 ? 0 : 2 * m - 1 + im); }

M2lLayout m2l3d_layout(int pb) {
  M2lLayout L{};
  L.p = pb;
  const int nr = (pb + 1) * (pb + 1);
  L.kpad = (nr - 1 + 3) / 4 * 4;
  L.npad = (nr - 1 + 15) / 16 * 16;
  L.stride = L.npad * L.kpad + L.npad + L.kpad + 4;
  L.cs = (nr + 3) / 4 * 4;
  L.lstride = 64 * ((L.npad / 16) * (L.kpad / 4 + 1) + L.kpad / 4) + 4;
  L.nr = nr;
  return L;
}

// ---------------------------------------------------------------------------
// 3D with the paper's fixed point charges (Appendix, STEP1-STEP3): 4 points per
// axis at (-2, -1, 1, 2) / 5 of the box side from the centre, point i + 4 j +
// 16 l at offsets (a_i, a_j, a_l).  The bilinear form of two boxes is the pair
// sum of their point charges, so the operator of offset o (in box sides) is
//   W_o[t][s] = 1 / |o + y_s - y_t|   (unit box side; level k scales it by 1/s_k),
// every entry of the 64 x 64 block; the degree-0 routes of the harmonic format
// (c0, r0, t00) stay zero.
// ---------------------------------------------------------------------------
M2lLayout points3d_layout() {
  M2lLayout L{};
  L.p = 4;  // points per axis
  L.nr = 65;
  L.kpad = 64;
  L.npad = 64;
  L.stride = L.npad * L.kpad + L.npad + L.kpad + 4;
  L.cs = 68;
  L.lstride = 64 * ((L.npad / 16) * (L.kpad / 4 + 1) + L.kpad / 4) + 4;
  return L;
}

void build_points3d_operators(const M2lLayout& L, int node_set, double* out) {
  double a[4];  // node offsets in units of the box side
  for (int i = 0; i < 4; ++i) a[i] = point_node(node_set, i) / 5.0;
  for (int dz = -3; dz <= 3; ++dz)
    for (int dy = -3; dy <= 3; ++dy)
      for (int dx = -3; dx <= 3; ++dx) {
        const int slot = (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);
        double* W = out + (size_t)slot * L.stride;
        for (int i = 0; i < L.stride; ++i) W[i] = 0.0;
        if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
        for (int t = 0; t < 64; ++t)
          for (int s = 0; s < 64; ++s) {
            const double rx = dx + a[s & 3] - a[t & 3];
            const double ry = dy + a[(s >> 2) & 3] - a[(t >> 2) & 3];
            const double rz = dz + a[s >> 4] - a[t >> 4];
            W[(size_t)t * L.kpad + s] = 1.0 / std::sqrt(rx * rx + ry * ry + rz * rz);
          }
      }
}

// Lane-major 3D pack for the matrix-core kernel (lane l: i = l % 16, g = l / 16;
// lane group g supplies the KS = kpad / 4 consecutive input values g KS .. g KS +
// KS - 1 of its source row), per slot:
//   B[nb][s][l], s < KS : Wb[16 nb + i][g KS + s]
//   B[nb][KS][l]        : c0[16 nb + i] for g = 0, else 0 (the degree-0 input step)
//   R[s][l], s < KS     : r0[g KS + s]
//   t00, pad[3]
void build_m2l3d_lane_pack(const M2lLayout& L, const double* pack, double* out) {
  const int ks = L.kpad / 4, nbk = L.npad / 16;
  for (int slot = 0; slot < 343; ++slot) {
    const double* W = pack + (size_t)slot * L.stride;
    const double* c0 = W + (size_t)L.npad * L.kpad;
    const double* r0 = c0 + L.npad;
    double* o = out + (size_t)slot * L.lstride;
    for (int nb = 0; nb < nbk; ++nb)
      for (int st = 0; st <= ks; ++st)
        for (int l = 0; l < 64; ++l) {
          const int i = l & 15, g = l >> 4;
          o[((size_t)nb * (ks + 1) + st) * 64 + l] =
              st < ks ? W[(size_t)(16 * nb + i) * L.kpad + g * ks + st]
                      : (g == 0 ? c0[16 * nb + i] : 0.0);
        }
    double* R = o + (size_t)nbk * (ks + 1) * 64;
    for (int st = 0; st < ks; ++st)
      for (int l = 0; l < 64; ++l) R[(size_t)st * 64 + l] = r0[(l >> 4) * ks + st];
    double* t = R + (size_t)ks * 64;
    t[0] = r0[L.kpad];
    t[1] = t[2] = t[3] = 0.0;
  }
}

// Irregular harmonics I_n^m(u), n <= P, m >= 0, by the recurrences
//   I_0^0 = 1/r,  I_m^m = -(2m-1)(x + i y)/r^2 I_{m-1}^{m-1},
//   r^2 I_n^m = (2n-1) z I_{n-1}^m - (n+m-1)(n-m-1) I_{n-2}^m.
static void irregular(int P, double x, double y, double z, std::vector<cd>& I) {
  I.assign((size_t)(P + 1) * (P + 1), 0.0);
  auto at = [&](int n, int m) -> cd& { return I[(size_t)n * (P + 1) + m]; };
  const double r2 = x * x + y * y + z * z;
  const cd xy(x, y);
  at(0, 0) = 1.0 / std::sqrt(r2);
  for (int m = 1; m <= P; ++m) at(m, m) = -(2.0 * m - 1.0) * xy / r2 * at(m - 1, m - 1);
  for (int m = 0; m <= P; ++m)
    for (int n = m + 1; n <= P; ++n) {
      const cd prev2 = n - 2 >= m ? at(n - 2, m) : cd(0.0);
      at(n, m) = ((2.0 * n - 1.0) * z * at(n - 1, m) - double(n + m - 1) * double(n - m - 1) * prev2) / r2;
    }
}

void build_m2l3d_operators(int p, const M2lLayout& L, double* out) {
  const int pb = L.p;
  const int i00 = (pb + 1) * (pb + 1) - 1;
  std::vector<cd> I;
  for (int dz = -3; dz <= 3; ++dz)
    for (int dy = -3; dy <= 3; ++dy)
      for (int dx = -3; dx <= 3; ++dx) {
        const int slot = (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);
        double* W = out + (size_t)slot * L.stride;
        for (int i = 0; i < L.stride; ++i) W[i] = 0.0;
        if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
        irregular(2 * p, dx, dy, dz, I);
        auto Inm = [&](int n, int m) -> cd {  // any sign of m
          if (std::abs(m) > n) return 0.0;
          const cd v = I[(size_t)n * (2 * p + 1) + std::abs(m)];
          return m >= 0 ? v : ((-m) & 1 ? -std::conj(v) : std::conj(v));
        };
        double* c0 = W + L.npad * L.kpad;
        double* r0 = c0 + L.npad;
        double* t00 = r0 + L.kpad;
        // entry(out_index, in_index, value) routed to Wb / c0 / r0 / t00
        auto put = [&](int oi, int ii, double v) {
          if (oi == i00 && ii == i00)
            t00[0] += v;
          else if (oi == i00)
            r0[ii] += v;
          else if (ii == i00)
            c0[oi] += v;
          else
            W[(size_t)oi * L.kpad + ii] += v;
        };
        for (int j = 0; j <= p; ++j)
          for (int k = 0; k <= j; ++k)
            for (int n = 0; n <= p; ++n)
              for (int m = 0; m <= n; ++m) {
                const double sg = ((k + n) & 1) ? -1.0 : 1.0;
                const int oRe = j == 0 ? i00 : ri3(j, k, 0);
                const int oIm = k == 0 ? -1 : ri3(j, k, 1);
                const int iRe = n == 0 ? i00 : ri3(n, m, 0);
                if (m == 0) {  // M_n^0 = a real
                  const cd c = sg * Inm(j + n, -k);
                  put(oRe, iRe, c.real());
                  if (oIm >= 0) put(oIm, iRe, c.imag());
                } else {  // M = a + i b and its mirror (-1)^m (a - i b)
                  const int iIm = ri3(n, m, 1);
                  const double pm = (m & 1) ? -1.0 : 1.0;
                  const cd A = Inm(j + n, m - k), B = Inm(j + n, -m - k);
                  const cd C = sg * (A + pm * B), D = sg * (A - pm * B);
                  put(oRe, iRe, C.real());
                  put(oRe, iIm, -D.imag());
                  if (oIm >= 0) {
                    put(oIm, iRe, C.imag());
                    put(oIm, iIm, D.real());
                  }
                }
              }
      }
}

}  // namespace sffmm
