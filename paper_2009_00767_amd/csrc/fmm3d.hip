// fmm3d.hip -- particle passes of the shift-free FMM for the 3D 1/r kernel.
//
// Two realisations of the box vectors: solid harmonics (below) and the paper's
// own fixed point charges (Appendix STEP1-STEP2, points_accumulate and
// eval_points3); the passes around them are shared.
//
// Box vectors are solid-harmonic moments of degree <= p about each box centre,
// scaled by the box side s_k (the particle map does not depend on the level,
// the Note closing Section 2.2.2), with the Condon-Shortley phase:
//   R_n^m(w) = |w|^n P_n^m(cos t) e^{i m f} / (n+m)!,   w = (r - r_b) / s_k,
//   M_n^m    = sum q conj R_n^m(w)                       (m >= 0 stored),
// and the local polynomial of a box is phi(r) = (1/s_k) sum_{j,k} L_j^k R_j^k(w).
// R_n^m is generated on the fly by the Cartesian recurrences
//   R_m^m = -(x + i y) / (2m) R_{m-1}^{m-1},
//   (n - m)(n + m) R_n^m = (2n - 1) z R_{n-1}^m - |w|^2 R_{n-2}^m,
// one order m at a time, and consumed immediately (few live registers).
// Real layout of a box: degree n >= 1 at n^2 - 1 (m = 0), n^2 - 1 + 2m - 1
// (re) and n^2 - 1 + 2m (im); degree 0 last ((PB+1)^2 - 1).
#include "device_common.h"

namespace sffmm {

template <int PB>
__host__ __device__ constexpr int ri3(int n, int m) {
  return n == 0 ? (PB + 1) * (PB + 1) - 1 : n * n - 1 + (m == 0 ? 0 : 2 * m - 1);
}

// Calls f(n, m, Rr, Ri) for every n <= p (<= PB), 0 <= m <= n.
template <typename T, int PB, typename F>
__device__ __forceinline__ void for_each_regular(T wx, T wy, T wz, int p, F&& f) {
  const T r2 = wx * wx + wy * wy + wz * wz;
  T dr = (T)1, di = (T)0;  // R_m^m
#pragma unroll
  for (int m = 0; m <= PB; ++m) {
    if (m <= p) {
      if (m > 0) {
        const T s = (T)(-1.0 / (2.0 * m));
        const T nr = (wx * dr - wy * di) * s;
        di = (wx * di + wy * dr) * s;
        dr = nr;
      }
      T r1r = dr, r1i = di, r0r = (T)0, r0i = (T)0;  // R_{n-1}, R_{n-2}
      f(m, m, r1r, r1i);
#pragma unroll
      for (int n = m + 1; n <= PB; ++n) {
        if (n <= p) {
          const T c1 = (T)((2.0 * n - 1.0) / ((double)(n - m) * (double)(n + m)));
          const T c2 = (T)(1.0 / ((double)(n - m) * (double)(n + m)));
          const T nr = c1 * wz * r1r - c2 * r2 * r0r;
          const T ni = c1 * wz * r1i - c2 * r2 * r0i;
          r0r = r1r;
          r0i = r1i;
          r1r = nr;
          r1i = ni;
          f(n, m, nr, ni);
        }
      }
    }
  }
}

#define SFFMM_PB3_DISPATCH(fn, p, ...)   \
  do {                                   \
    switch (order_bucket3(p)) {          \
      case 4: fn<4>(__VA_ARGS__); break; \
      case 8: fn<8>(__VA_ARGS__); break; \
      default: fn<12>(__VA_ARGS__); break; \
    }                                    \
  } while (0)

// ---------------------------------------------------------------------------
// P2M (work plan in device_common.h): register accumulation, group butterfly
// reduction, slice partials added in order by k_p2m3d_slices.
// ---------------------------------------------------------------------------
size_t p2m3d_partial_entries(int klo, int khi, int64_t maxn, int cs) {
  return p2m_partial_rows(3, klo, khi, maxn) * (size_t)cs + 1;
}

template <typename T, int PB, bool LL, int BASIS>
__global__ __launch_bounds__(256) void k_p2m3d(FmmArgs a, P2mPlan pl) {
  constexpr bool PTS = BASIS != 0;
  constexpr int NR = PTS ? 64 : (PB + 1) * (PB + 1);
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if ((t & ~(int64_t)63) >= pl.thr_off[pl.khi + 1]) return;  // whole wave beyond the end
  const LevelTable& lt = a.lt;
  int k = pl.klo;
  while (k < pl.khi && t >= pl.thr_off[k + 1]) ++k;
  const int G = pl.G[k], S = pl.S[k];
  const int64_t local = t - pl.thr_off[k];
  const int64_t nb = (int64_t)1 << (3 * k);
  const int64_t b = local / (G * S);
  const bool valid = b < nb;
  const int rem = (int)(local - b * G * S);
  const int j = rem / G, r = rem - (rem / G) * G;
  const int sh = lt.L - k;
  const int p = a.p;
  T acc[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) acc[i] = (T)0;
  if (valid) {
    const int64_t s0 = a.leaf_start[b << (3 * sh)], s1 = a.leaf_start[(b + 1) << (3 * sh)];
    const int64_t len = s1 - s0;
    const int64_t lo = s0 + len * j / S, hi = s0 + len * (j + 1) / S;
    const T is = (T)lt.inv_s[k], sL = (T)lt.s[lt.L];
    T cx = 0, cy = 0, cz = 0;
    if (!LL) {
      const uint32_t ub = (uint32_t)b;
      cx = (T)(lt.origin[0] + lt.s[k] * ((double)compact3(ub) + 0.5));
      cy = (T)(lt.origin[1] + lt.s[k] * ((double)compact3(ub >> 1) + 0.5));
      cz = (T)(lt.origin[2] + lt.s[k] * ((double)compact3(ub >> 2) + 0.5));
    }
    for (int64_t i = lo + r; i < hi; i += G) {
      T q, wx, wy, wz;
      if (LL) {
        const float4 pt = a.pts[i];
        const uint32_t key = a.keys[i];
        q = (T)pt.w;
        wx = ((T)pt.x + leaf_to_box<T>(compact3(key), sh) * sL) * is;
        wy = ((T)pt.y + leaf_to_box<T>(compact3(key >> 1), sh) * sL) * is;
        wz = ((T)pt.z + leaf_to_box<T>(compact3(key >> 2), sh) * sL) * is;
      } else {
        q = (T)a.qs[i];
        wx = ((T)a.xs[i] - cx) * is;
        wy = ((T)a.ys[i] - cy) * is;
        wz = ((T)a.zs[i] - cz) * is;
      }
      if constexpr (PTS) {
        points_accumulate<BASIS, T>(acc, q, wx, wy, wz);
      } else {
        for_each_regular<T, PB>(wx, wy, wz, p, [&](int n, int m, T rr, T rim) {
          const int idx = ri3<PB>(n, m);
          acc[idx] += q * rr;
          if (m > 0) acc[idx + 1] -= q * rim;  // conj
        });
      }
    }
  }
  for (int d = 1; d < G; d <<= 1) {
#pragma unroll
    for (int i = 0; i < NR; ++i) acc[i] += __shfl_xor(acc[i], d, 64);
  }
  if (!valid || r != 0) return;
  const int cs = a.cs;
  T* out;
  if (S == 1)
    out = (sizeof(T) == 8 ? (T*)a.mom64 : (T*)a.mom32) + (lt.off[k] + b) * cs;
  else
    out = (sizeof(T) == 8 ? (T*)a.part64 : (T*)a.part32) + (pl.part_off[k] + b * S + j) * cs;
#pragma unroll
  for (int i = 0; i < NR; ++i) out[i] = acc[i];
}

template <typename T>
__global__ void k_p2m3d_slices(FmmArgs a, P2mPlan pl, int k, int nc) {
  const int64_t nb = (int64_t)1 << (3 * k);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nb * nc) return;
  const int64_t b = g / nc;
  const int c = (int)(g - b * nc);
  const int S = pl.S[k];
  const T* part = sizeof(T) == 8 ? (const T*)a.part64 : (const T*)a.part32;
  T* mom = sizeof(T) == 8 ? (T*)a.mom64 : (T*)a.mom32;
  const T* src = part + (pl.part_off[k] + b * S) * a.cs + c;
  T acc = 0;
  for (int j = 0; j < S; ++j) acc += src[(int64_t)j * a.cs];
  mom[(a.lt.off[k] + b) * a.cs + c] = acc;
}

template <int PB, int BASIS = 0>
static void p2m3d_dispatch(const FmmArgs& a, bool ll, bool f64, hipStream_t st) {
  const P2mPlan pl = make_p2m_plan(3, a.klo, a.khi, a.n);
  const int64_t thr = pl.thr_off[a.khi + 1];
  const dim3 grid((unsigned)((thr + 255) / 256));
  if (f64) {
    if (ll)
      hipLaunchKernelGGL((k_p2m3d<double, PB, true, BASIS>), grid, dim3(256), 0, st, a, pl);
    else
      hipLaunchKernelGGL((k_p2m3d<double, PB, false, BASIS>), grid, dim3(256), 0, st, a, pl);
  } else {
    hipLaunchKernelGGL((k_p2m3d<float, PB, true, BASIS>), grid, dim3(256), 0, st, a, pl);
  }
  constexpr int NR = BASIS ? 64 : (PB + 1) * (PB + 1);
  for (int k = a.klo; k <= a.khi; ++k)
    if (pl.S[k] > 1) {
      const int64_t cnt = ((int64_t)1 << (3 * k)) * NR;
      if (f64)
        hipLaunchKernelGGL(k_p2m3d_slices<double>, dim3((cnt + 255) / 256), dim3(256), 0, st, a,
                           pl, k, NR);
      else
        hipLaunchKernelGGL(k_p2m3d_slices<float>, dim3((cnt + 255) / 256), dim3(256), 0, st, a,
                           pl, k, NR);
    }
}

void launch_p2m3d(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st) {
  if (a.khi < a.klo || a.n <= 0) return;
  if (a.basis == 1) {
    p2m3d_dispatch<4, 1>(a, leaf_local, fp64, st);
    return;
  }
  if (a.basis == 2) {
    p2m3d_dispatch<4, 2>(a, leaf_local, fp64, st);
    return;
  }
  SFFMM_PB3_DISPATCH(p2m3d_dispatch, a.p, a, leaf_local, fp64, st);
}

// ---------------------------------------------------------------------------
// L2P.  With F(w) = sum_{j,k} L_j^k R_j^k(w) (real), d/dz R_j^k = R_{j-1}^k and
// (d/dx + i d/dy) R_j^k = R_{j-1}^{k+1}, every R_n^m (m >= 0) contributes
//   F  += c_m Re(L_n^m R_n^m)                     (c_0 = 1, c_m = 2)
//   Fz += c_m Re(L_{n+1}^m R_n^m)
//   G  += L_{n+1}^{m-1} R_n^m (m >= 1) - conj(L_{n+1}^{m+1} R_n^m)
// with G = dF/dx + i dF/dy; phi = F / s, field = -(Re G, Im G, Fz) / s^2.
// ---------------------------------------------------------------------------
template <typename T, int CS>
__device__ __forceinline__ void load_row3(const T* B, T (&r)[CS]) {
  if (sizeof(T) == 4) {
    const float4* v = reinterpret_cast<const float4*>(B);
#pragma unroll
    for (int i = 0; i < CS / 4; ++i) {
      const float4 t = v[i];
      r[4 * i] = t.x;
      r[4 * i + 1] = t.y;
      r[4 * i + 2] = t.z;
      r[4 * i + 3] = t.w;
    }
  } else {
    const double2* v = reinterpret_cast<const double2*>(B);
#pragma unroll
    for (int i = 0; i < CS / 2; ++i) {
      const double2 t = v[i];
      r[2 * i] = t.x;
      r[2 * i + 1] = t.y;
    }
  }
}

template <typename T, int PB>
__device__ __forceinline__ void eval_local3(const T* B, int p, T wx, T wy, T wz, T& F, T& Fz,
                                            T& Gr, T& Gi) {
  constexpr int CS = ((PB + 1) * (PB + 1) + 3) / 4 * 4;
  T L[CS];
  load_row3<T, CS>(B, L);
  auto lre = [&](int n, int m) -> T { return L[ri3<PB>(n, m)]; };
  auto lim = [&](int n, int m) -> T { return m == 0 ? (T)0 : L[ri3<PB>(n, m) + 1]; };
  F = Fz = Gr = Gi = (T)0;
  for_each_regular<T, PB>(wx, wy, wz, p, [&](int n, int m, T rr, T ri) {
    const T c = m == 0 ? (T)1 : (T)2;
    F += c * (lre(n, m) * rr - lim(n, m) * ri);
    if (n + 1 <= p) {
      Fz += c * (lre(n + 1, m) * rr - lim(n + 1, m) * ri);
      if (m >= 1) {
        const T a = lre(n + 1, m - 1), b = lim(n + 1, m - 1);
        Gr += a * rr - b * ri;
        Gi += a * ri + b * rr;
      }
      const T a = lre(n + 1, m + 1), b = lim(n + 1, m + 1);
      Gr -= a * rr - b * ri;
      Gi += a * ri + b * rr;
    }
  });
}

// Fixed point-charge basis: the potential of a unit probe at w is
// (1/s) sum f_i f_j f_l L_{ijl} (the probe mapped by STEP2), contracted one axis
// at a time; its gradient uses d/dw = 5 d/du, returned in the harmonic form's
// outputs (F, Fz, Gr, Gi) = (phi, dphi/dz, dphi/dx, dphi/dy) * s (times s^2 for
// the derivatives).
template <int NS, typename T>
__device__ __forceinline__ void eval_points3(const T* B, T wx, T wy, T wz, T& F, T& Fz, T& Gr,
                                             T& Gi) {
  T L[64];
  load_row3<T, 64>(B, L);
  T fx[4], dfx[4], fy[4], dfy[4], fz[4], dfz[4];
  lag4d<NS>(wx, fx, dfx);
  lag4d<NS>(wy, fy, dfy);
  lag4d<NS>(wz, fz, dfz);
  F = Fz = Gr = Gi = (T)0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    T h = 0, hx = 0, hy = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      T g = 0, gd = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        g += fx[i] * L[i + 4 * j + 16 * l];
        gd += dfx[i] * L[i + 4 * j + 16 * l];
      }
      h += fy[j] * g;
      hx += fy[j] * gd;
      hy += dfy[j] * g;
    }
    F += fz[l] * h;
    Gr += fz[l] * hx;
    Gi += fz[l] * hy;
    Fz += dfz[l] * h;
  }
  Gr *= (T)5;
  Gi *= (T)5;
  Fz *= (T)5;
}

template <int PB, bool LL, int BASIS>
__global__ __launch_bounds__(256) void k_l2p3d(FmmArgs a) {
  constexpr bool PTS = BASIS != 0;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const LevelTable& lt = a.lt;
  const uint32_t key = a.keys[j];
  const uint32_t lx = compact3(key), ly = compact3(key >> 1), lz = compact3(key >> 2);
  const int p = a.p, cs = a.cs;
  float4 pt = make_float4(0.f, 0.f, 0.f, 0.f);
  double x = 0, y = 0, z = 0;
  if (LL)
    pt = a.pts[j];
  else {
    x = a.xs[j];
    y = a.ys[j];
    z = a.zs[j];
  }
  double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
  for (int k = lt.kmin; k <= lt.L; ++k) {
    const int sh = lt.L - k;
    const uint32_t box = key >> (3 * sh);
    if (k < lt.split) {
      double wx, wy, wz;
      if (LL) {
        const double sL = lt.s[lt.L], is = lt.inv_s[k];
        wx = ((double)pt.x + leaf_to_box<double>(lx, sh) * sL) * is;
        wy = ((double)pt.y + leaf_to_box<double>(ly, sh) * sL) * is;
        wz = ((double)pt.z + leaf_to_box<double>(lz, sh) * sL) * is;
      } else {
        wx = (x - (lt.origin[0] + lt.s[k] * ((double)(lx >> sh) + 0.5))) * lt.inv_s[k];
        wy = (y - (lt.origin[1] + lt.s[k] * ((double)(ly >> sh) + 0.5))) * lt.inv_s[k];
        wz = (z - (lt.origin[2] + lt.s[k] * ((double)(lz >> sh) + 0.5))) * lt.inv_s[k];
      }
      double F, Fz, Gr, Gi;
      if constexpr (PTS)
        eval_points3<BASIS, double>(a.loc64 + (lt.off[k] + box) * cs, wx, wy, wz, F, Fz, Gr, Gi);
      else
        eval_local3<double, PB>(a.loc64 + (lt.off[k] + box) * cs, p, wx, wy, wz, F, Fz, Gr, Gi);
      const double is = lt.inv_s[k];
      phi += F * is;
      ex -= Gr * is * is;
      ey -= Gi * is * is;
      ez -= Fz * is * is;
    } else {
      const float sL = (float)lt.s[lt.L], is = (float)lt.inv_s[k];
      const float wx = (pt.x + leaf_to_box<float>(lx, sh) * sL) * is;
      const float wy = (pt.y + leaf_to_box<float>(ly, sh) * sL) * is;
      const float wz = (pt.z + leaf_to_box<float>(lz, sh) * sL) * is;
      float F, Fz, Gr, Gi;
      if constexpr (PTS)
        eval_points3<BASIS, float>(a.loc32 + (lt.off[k] + box) * cs, wx, wy, wz, F, Fz, Gr, Gi);
      else
        eval_local3<float, PB>(a.loc32 + (lt.off[k] + box) * cs, p, wx, wy, wz, F, Fz, Gr, Gi);
      const double id = lt.inv_s[k];
      phi += (double)F * id;
      ex -= (double)Gr * id * id;
      ey -= (double)Gi * id * id;
      ez -= (double)Fz * id * id;
    }
  }
  const int64_t o = a.perm[j];
  a.pot[o] = phi + a.near_pot[j];
  if (a.field) {
    a.field[3 * o] = ex + a.near_ex[j];
    a.field[3 * o + 1] = ey + a.near_ey[j];
    a.field[3 * o + 2] = ez + a.near_ez[j];
  }
}

template <int PB, int BASIS = 0>
static void l2p3d_dispatch(const FmmArgs& a, bool ll, hipStream_t st) {
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (ll)
    hipLaunchKernelGGL((k_l2p3d<PB, true, BASIS>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_l2p3d<PB, false, BASIS>), grid, dim3(256), 0, st, a);
}

void launch_l2p3d(const FmmArgs& a, bool leaf_local, hipStream_t st) {
  if (a.n <= 0) return;
  if (a.basis == 1) {
    l2p3d_dispatch<4, 1>(a, leaf_local, st);
    return;
  }
  if (a.basis == 2) {
    l2p3d_dispatch<4, 2>(a, leaf_local, st);
    return;
  }
  SFFMM_PB3_DISPATCH(l2p3d_dispatch, a.p, a, leaf_local, st);
}

// ---------------------------------------------------------------------------
// P2P: one thread per sorted target over the 27 leaves around it; pairs with
// r = 0 (the target itself, coincident points) contribute nothing.
// phi += q / r,  field += q (x_t - x_s) / r^3.
// ---------------------------------------------------------------------------
// 1 / sqrt(x) for normal x > 0: the hardware estimate refined by two
// Newton-Raphson steps for f(y) = 1/y^2 - x, y <- y + y (1 - x y^2) / 2; each
// step squares the relative error, which ends within a few units in the last
// place (instead of a correctly rounded square root and division).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// One source.  r^2 is formed on a floor, fma(dx, dx, fma(dy, dy, fma(dz, dz,
// 2^-400))), which keeps 1 / sqrt finite at r = 0, and the charge of a pair at
// r = 0 is taken as zero by a select (a branch per pair costs more); for real
// pairs the floor changes r^2 by 2^-400 / r^2.
constexpr double kP2p3Eps = 0x1p-400;
__device__ __forceinline__ void pair3_f64(double x, double y, double z, double sx, double sy,
                                          double sz, double sq, double& phi, double& ex,
                                          double& ey, double& ez) {
  const double dx = x - sx, dy = y - sy, dz = z - sz;
  const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, kP2p3Eps)));
  const double rinv = rsqrt_nr(r2);
  const double qr = (r2 > kP2p3Eps ? sq : 0.0) * rinv;
  phi += qr;
  const double w = qr * rinv * rinv;
  ex += w * dx;
  ey += w * dy;
  ez += w * dz;
}

// PARTS > 1 (few particles for the chip): PARTS waves per 64 targets (a
// workgroup of 64 PARTS threads), wave w walking the in-domain neighbour leaves
// w, w + PARTS, ... of the 27; the partial sums meet in LDS and are added in
// wave order.  PARTS = 1: 256 targets per workgroup.
template <int PARTS>
constexpr int p2p3_threads() {
  return PARTS == 1 ? 256 : 64 * PARTS;
}

template <int PARTS>
__device__ __forceinline__ void p2p3d_finish(FmmArgs& a, int64_t j, bool live, double phi,
                                             double ex, double ey, double ez) {
  if constexpr (PARTS > 1) {
    constexpr int TPB = 64;
    __shared__ double red[4][PARTS][TPB];
    const int part = threadIdx.x / TPB, tl = threadIdx.x % TPB;
    red[0][part][tl] = phi;
    red[1][part][tl] = ex;
    red[2][part][tl] = ey;
    red[3][part][tl] = ez;
    __syncthreads();
    if (part != 0 || !live) return;
#pragma unroll
    for (int w = 1; w < PARTS; ++w) {
      phi += red[0][w][tl];
      ex += red[1][w][tl];
      ey += red[2][w][tl];
      ez += red[3][w][tl];
    }
  }
  a.near_pot[j] = phi;
  a.near_ex[j] = ex;
  a.near_ey[j] = ey;
  a.near_ez[j] = ez;
}

// Sources [i0, i1) four at a time, their loads issued together (the sums keep
// the source order).
__device__ __forceinline__ void p2p3_range_f64(const FmmArgs& a, int32_t i0, int32_t i1, double x,
                                               double y, double z, double& phi, double& ex,
                                               double& ey, double& ez) {
  int32_t i = i0;
  for (; i + 4 <= i1; i += 4) {
    double sx[4], sy[4], sz[4], sq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sx[u] = a.xs[i + u];
      sy[u] = a.ys[i + u];
      sz[u] = a.zs[i + u];
      sq[u] = a.qs[i + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) pair3_f64(x, y, z, sx[u], sy[u], sz[u], sq[u], phi, ex, ey, ez);
  }
  for (; i < i1; ++i) pair3_f64(x, y, z, a.xs[i], a.ys[i], a.zs[i], a.qs[i], phi, ex, ey, ez);
}

// Orders the LDS accesses of one wave whose lanes read what other lanes wrote:
// no access moves across it (a wave's LDS instructions complete in order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// p2p3_range_f64 for a wave whose 64 lanes all walk the same range: 64 sources
// at a time come in with coalesced loads (a source per lane) into the wave's LDS
// stage (x, y in the first 64 slots, z, q in the next 64), and every lane reads
// them back from there (one address for the whole wave), instead of four 8-byte
// vector loads per source and pair.  The order of the sums is unchanged.
__device__ __forceinline__ void p2p3_range_f64_staged(const FmmArgs& a, int32_t i0, int32_t i1,
                                                      double x, double y, double z,
                                                      double2* stage, int lane, double& phi,
                                                      double& ex, double& ey, double& ez) {
  for (int32_t g0 = i0; g0 < i1; g0 += 64) {
    const int m = i1 - g0 < 64 ? i1 - g0 : 64;
    double2 u = make_double2(0.0, 0.0), v = make_double2(0.0, 0.0);
    if (lane < m) {
      u = make_double2(a.xs[g0 + lane], a.ys[g0 + lane]);
      v = make_double2(a.zs[g0 + lane], a.qs[g0 + lane]);
    }
    wave_lds_sync();  // the previous chunk's reads are done
    stage[lane] = u;
    stage[64 + lane] = v;
    wave_lds_sync();
    int s = 0;
    for (; s + 4 <= m; s += 4) {
      double2 su[4], sv[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        su[w] = stage[s + w];
        sv[w] = stage[64 + s + w];
      }
#pragma unroll
      for (int w = 0; w < 4; ++w)
        pair3_f64(x, y, z, su[w].x, su[w].y, sv[w].x, sv[w].y, phi, ex, ey, ez);
    }
    for (; s < m; ++s) {
      const double2 su = stage[s], sv = stage[64 + s];
      pair3_f64(x, y, z, su.x, su.y, sv.x, sv.y, phi, ex, ey, ez);
    }
  }
}

// A wave whose 64 targets lie in one leaf walks the sources through its LDS stage.
template <int PARTS>
__global__ __launch_bounds__(p2p3_threads<PARTS>()) void k_p2p3d_f64(FmmArgs a) {
  constexpr int TPB = PARTS == 1 ? 256 : 64;
  __shared__ double2 stage[p2p3_threads<PARTS>() / 64][128];
  const int part = threadIdx.x / TPB;
  const int64_t j = (int64_t)blockIdx.x * TPB + threadIdx.x % TPB;
  const bool live = j < a.n;
  if (PARTS == 1 && !live) return;
  const uint32_t key = live ? a.keys[j] : 0u;
  const uint32_t k0 = __builtin_amdgcn_readfirstlane(key);
  const bool uni = __ballot(live && key == k0) == ~0ull;  // every lane live, one leaf
  double2* wstage = stage[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63;
  double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
  if (live) {
    const int L = a.lt.L;
    const int lx = (int)compact3(key), ly = (int)compact3(key >> 1), lz = (int)compact3(key >> 2);
    const int nl = 1 << L;
    const double x = a.xs[j], y = a.ys[j], z = a.zs[j];
    int nbr = 0;
    for (int nz = lz - 1; nz <= lz + 1; ++nz) {
      if (nz < 0 || nz >= nl) continue;
      for (int ny = ly - 1; ny <= ly + 1; ++ny) {
        if (ny < 0 || ny >= nl) continue;
        for (int nx = lx - 1; nx <= lx + 1; ++nx) {
          if (nx < 0 || nx >= nl) continue;
          if (PARTS > 1 && nbr++ % PARTS != part) continue;
          const uint32_t nk = spread3(nx) | (spread3(ny) << 1) | (spread3(nz) << 2);
          const int32_t i0 = a.leaf_start[nk], i1 = a.leaf_start[nk + 1];
          if (uni)
            p2p3_range_f64_staged(a, i0, i1, x, y, z, wstage, lane, phi, ex, ey, ez);
          else
            p2p3_range_f64(a, i0, i1, x, y, z, phi, ex, ey, ez);
        }
      }
    }
  }
  p2p3d_finish<PARTS>(a, j, live, phi, ex, ey, ez);
}

// t: the target's leaf-local coordinates moved into the source leaf's frame
// (its offset added once per neighbouring leaf)
__device__ __forceinline__ void pair3_f32(float tx, float ty, float tz, const float4& s,
                                          float& fp, float& fx, float& fy, float& fz) {
  const float dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
  const float r2 = dx * dx + dy * dy + dz * dz;
  const float ri = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
  const float qr = s.w * ri;
  fp += qr;
  const float w = qr * ri * ri;
  fx += w * dx;
  fy += w * dy;
  fz += w * dz;
}

// Sources [i0, i1) in runs of at most 32, each run's FP32 sums flushed to FP64;
// four source loads issued together.
__device__ __forceinline__ void p2p3_range_f32(const float4* __restrict__ pts, int32_t i0,
                                               int32_t i1, float tx, float ty, float tz,
                                               double& phi, double& ex, double& ey, double& ez) {
  for (int32_t c0 = i0; c0 < i1; c0 += 32) {
    const int32_t c1 = c0 + 32 < i1 ? c0 + 32 : i1;
    float fp = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
    int32_t i = c0;
    for (; i + 4 <= c1; i += 4) {
      float4 sb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) sb[u] = pts[i + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) pair3_f32(tx, ty, tz, sb[u], fp, fx, fy, fz);
    }
    for (; i < c1; ++i) pair3_f32(tx, ty, tz, pts[i], fp, fx, fy, fz);
    phi += (double)fp;
    ex += (double)fx;
    ey += (double)fy;
    ez += (double)fz;
  }
}

// p2p3_range_f32 for a wave whose 64 lanes all walk the same range: 64 sources
// at a time come in with one coalesced load (a record per lane) into the
// wave's LDS stage, and every lane reads them back from there (one address for
// the whole wave), instead of a 16-byte vector load per source and pair.  The
// runs and the order of the sums are those of p2p3_range_f32.
__device__ __forceinline__ void p2p3_range_f32_staged(const float4* __restrict__ pts, int32_t i0,
                                                      int32_t i1, float tx, float ty, float tz,
                                                      float4* stage, int lane, double& phi,
                                                      double& ex, double& ey, double& ez) {
  for (int32_t g0 = i0; g0 < i1; g0 += 64) {
    const int m = i1 - g0 < 64 ? i1 - g0 : 64;
    const float4 v = lane < m ? pts[g0 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
    wave_lds_sync();  // the previous chunk's reads are done
    stage[lane] = v;
    wave_lds_sync();
    for (int r0 = 0; r0 < m; r0 += 32) {
      const int r1 = r0 + 32 < m ? r0 + 32 : m;
      float fp = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
      int s = r0;
      for (; s + 4 <= r1; s += 4) {
        float4 sb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) sb[u] = stage[s + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) pair3_f32(tx, ty, tz, sb[u], fp, fx, fy, fz);
      }
      for (; s < r1; ++s) pair3_f32(tx, ty, tz, stage[s], fp, fx, fy, fz);
      phi += (double)fp;
      ex += (double)fx;
      ey += (double)fy;
      ez += (double)fz;
    }
  }
}

// FP32 pair terms from leaf-local coordinates (leaf-centre offsets exact).  A
// wave whose 64 targets lie in one leaf walks the sources through its LDS stage.
template <int PARTS>
__global__ __launch_bounds__(p2p3_threads<PARTS>(), 8) void k_p2p3d_f32(FmmArgs a) {
  constexpr int TPB = PARTS == 1 ? 256 : 64;
  __shared__ float4 stage[p2p3_threads<PARTS>() / 64][64];
  const int part = threadIdx.x / TPB;
  const int64_t j = (int64_t)blockIdx.x * TPB + threadIdx.x % TPB;
  const bool live = j < a.n;
  if (PARTS == 1 && !live) return;
  const uint32_t key = live ? a.keys[j] : 0u;
  const uint32_t k0 = __builtin_amdgcn_readfirstlane(key);
  const bool uni = __ballot(live && key == k0) == ~0ull;  // every lane live, one leaf
  float4* wstage = stage[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63;
  double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
  if (live) {
    const int L = a.lt.L;
    const int lx = (int)compact3(key), ly = (int)compact3(key >> 1), lz = (int)compact3(key >> 2);
    const int nl = 1 << L;
    const float sL = (float)a.lt.s[L];
    const float4 t = a.pts[j];
    int nbr = 0;
    for (int nz = lz - 1; nz <= lz + 1; ++nz) {
      if (nz < 0 || nz >= nl) continue;
      const float oz = (float)(lz - nz) * sL;
      for (int ny = ly - 1; ny <= ly + 1; ++ny) {
        if (ny < 0 || ny >= nl) continue;
        const float oy = (float)(ly - ny) * sL;
        for (int nx = lx - 1; nx <= lx + 1; ++nx) {
          if (nx < 0 || nx >= nl) continue;
          if (PARTS > 1 && nbr++ % PARTS != part) continue;
          const float ox = (float)(lx - nx) * sL;
          const float tx = t.x + ox, ty = t.y + oy, tz = t.z + oz;
          const uint32_t nk = spread3(nx) | (spread3(ny) << 1) | (spread3(nz) << 2);
          const int32_t i0 = a.leaf_start[nk], i1 = a.leaf_start[nk + 1];
          if (uni)
            p2p3_range_f32_staged(a.pts, i0, i1, tx, ty, tz, wstage, lane, phi, ex, ey, ez);
          else
            p2p3_range_f32(a.pts, i0, i1, tx, ty, tz, phi, ex, ey, ez);
        }
      }
    }
  }
  p2p3d_finish<PARTS>(a, j, live, phi, ex, ey, ez);
}

template <int PARTS>
static void p2p3d_launch(const FmmArgs& a, bool leaf_local, hipStream_t st) {
  constexpr int tpb = PARTS == 1 ? 256 : 64;
  const dim3 grid((unsigned)((a.n + tpb - 1) / tpb)), block(p2p3_threads<PARTS>());
  if (leaf_local)
    hipLaunchKernelGGL(k_p2p3d_f32<PARTS>, grid, block, 0, st, a);
  else
    hipLaunchKernelGGL(k_p2p3d_f64<PARTS>, grid, block, 0, st, a);
}

// Several waves per 64 targets while the targets alone would leave the chip's
// SIMDs short of waves (below 16 waves of targets per SIMD): eight when a
// target meets many sources (27 times the mean leaf occupancy at least 8192),
// where shorter waves even out the launch's tail (the paper's 200k-particle
// level-3 run: 1.11 -> 1.01 ms, its 80k level-2 run 1.36 -> 1.12 ms), else four,
// which leaves the moments chain beside it more of the chip (the 80k level-3
// run: 0.38 ms with four, 0.40 with eight).
void launch_p2p3d(const FmmArgs& a, bool leaf_local, hipStream_t st) {
  if (a.n <= 0) return;
  const double leaves = (double)((int64_t)a.lt.nsys << (3 * a.lt.L));
  const double per_target = 27.0 * (double)a.n / leaves;
  if (a.n >= (int64_t)256 * 16 * 64)
    p2p3d_launch<1>(a, leaf_local, st);
  else if (per_target >= 8192.0)
    p2p3d_launch<8>(a, leaf_local, st);
  else
    p2p3d_launch<4>(a, leaf_local, st);
}

}  // namespace sffmm
