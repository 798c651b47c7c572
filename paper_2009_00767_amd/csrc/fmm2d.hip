// fmm2d.hip -- particle passes of the shift-free FMM for the 2D log kernel.
//
// Box vectors are complex Laurent coefficients of order p about each box
// centre, scaled by the box side s_k (the vector space V of Section 2.2.1; the
// map from a particle to its coefficients does not depend on the level, the
// Note closing Section 2.2.2):
//   A_0 = sum q,   A_m = -(1/m) sum q w^m,   w = (z - z_b) / s_k.
// Pass structure (no M2M, no L2L):
//   p2m : every level's box vectors straight from the Morton-sorted particles
//         (U-bar-1, U-bar-2 realised without a shift);
//   m2l : m2l2d.hip (D-bar-1);
//   l2p : every level's local polynomial evaluated at the particles and summed
//         over levels in FP64 (D-bar-2 and F(v) = L_{m^l}(v));
//   p2p : the near field (E-2 of Section 2.1), in sorted order; it only needs
//         the sort, so it runs on its own stream beside the far-field chain,
//         and l2p adds near + far and scatters back to input order.
// Two particle representations: FP64 absolute coordinates (FP64 mode) and FP32
// offsets from the leaf centre (FP32 modes).  Leaf-centre differences between
// boxes of any level are multiples of s_L / 2 and are formed exactly.
//
// Coefficient layout of a box: re/im of coefficients 1..PB at 2(m-1), 2(m-1)+1,
// coefficient 0 at 2 PB, 2 PB + 1 (PB = order bucket of the largest order).
// Each level k has its own order p_k <= PB (a.ord[k]): moments above p_k are
// written as zeros, locals above p_k are never read.
#include <algorithm>
#include <type_traits>

#include "device_common.h"

namespace sffmm {

#define SFFMM_PB_DISPATCH(fn, p, ...) \
  do {                                \
    switch (order_bucket(p)) {        \
      case 8: fn<8>(__VA_ARGS__); break;   \
      case 12: fn<12>(__VA_ARGS__); break; \
      case 16: fn<16>(__VA_ARGS__); break; \
      case 20: fn<20>(__VA_ARGS__); break; \
      case 24: fn<24>(__VA_ARGS__); break; \
      default: fn<30>(__VA_ARGS__); break; \
    }                                 \
  } while (0)

// ---------------------------------------------------------------------------
// P2M (work plan in device_common.h).  Lanes accumulate in registers, a group
// reduction by butterfly shuffles combines the G lanes of a box, and the
// slices of a box are added by a second kernel in a fixed order (one wave per
// coefficient): deterministic, no floating-point atomics.
// ---------------------------------------------------------------------------
size_t p2m2d_partial_entries(const LevelTable& lt, int klo, int khi, int64_t maxn, int cs) {
  return p2m_partial_rows(2, klo, khi, maxn, lt.nsys) * (size_t)cs + 1;
}

// Runs f(integral_constant<PK>) with PK the order bucket of p (at most PB), so
// that a level's work follows its own order and not the layout's: the loops
// over coefficients are unrolled to PK with no per-coefficient test.
// FULL: every level runs at the layout order PB.
template <int PB, bool FULL, class F>
__device__ __forceinline__ void with_order_bucket(int p, F&& f) {
  if (FULL) {
    f(std::integral_constant<int, PB>());
    return;
  }
  const int pk = order_bucket(p);
  if constexpr (PB > 8)
    if (pk == 8) {
      f(std::integral_constant<int, 8>());
      return;
    }
  if constexpr (PB > 12)
    if (pk == 12) {
      f(std::integral_constant<int, 12>());
      return;
    }
  if constexpr (PB > 16)
    if (pk == 16) {
      f(std::integral_constant<int, 16>());
      return;
    }
  if constexpr (PB > 20)
    if (pk == 20) {
      f(std::integral_constant<int, 20>());
      return;
    }
  if constexpr (PB > 24)
    if (pk == 24) {
      f(std::integral_constant<int, 24>());
      return;
    }
  f(std::integral_constant<int, PB>());
}

// Moments of one (box, slice, lane) work item up to order PK (>= p): powers
// of w above p are formed too and dropped at the store, where every moment
// above p is written as zero.
template <typename T, int PB, int PK, bool LL>
__device__ __forceinline__ void p2m_item(const FmmArgs& a, const P2mPlan& pl, int k, int p,
                                         bool valid, int64_t b, int j, int r, int G, int S) {
  const LevelTable& lt = a.lt;
  const int sh = lt.L - k;
  T re[PK + 1], im[PK + 1];
#pragma unroll
  for (int m = 0; m <= PK; ++m) re[m] = im[m] = (T)0;
  // adaptive depth: only the moments some interaction list reads, those of
  // boxes whose parent has an open box in its 3 x 3 (every box at kmin)
  if (valid && a.adapt_open && k > lt.kmin)
    valid = (a.adapt_open[adapt_open_off(k - 1) + (b >> 2)] & 2) != 0;
  if (valid) {
    const int64_t s0 = a.leaf_start[b << (2 * sh)], s1 = a.leaf_start[(b + 1) << (2 * sh)];
    const int64_t len = s1 - s0;
    const int64_t lo = s0 + len * j / S, hi = s0 + len * (j + 1) / S;
    const T is = (T)lt.inv_s[k];
    T cx = 0, cy = 0, sL = (T)lt.s[lt.L];
    if (!LL) {
      const uint32_t lb = local2((uint32_t)b, k);
      cx = (T)(lt.origin[0] + lt.s[k] * ((double)compact2(lb) + 0.5));
      cy = (T)(lt.origin[1] + lt.s[k] * ((double)compact2(lb >> 1) + 0.5));
    }
    // the next particle's inputs are loaded while this one is accumulated
    float4 npt = make_float4(0.f, 0.f, 0.f, 0.f);
    double nx = 0, ny = 0, nq = 0;
    if (lo + r < hi) {
      if (LL) {
        npt = a.pts[lo + r];
      } else {
        nx = a.xs[lo + r];
        ny = a.ys[lo + r];
        nq = a.qs[lo + r];
      }
    }
    for (int64_t i = lo + r; i < hi; i += G) {
      T q, wr, wi;
      const float4 pt = npt;
      const double px = nx, py = ny, pq = nq;
      if (i + G < hi) {
        if (LL) {
          npt = a.pts[i + G];
        } else {
          nx = a.xs[i + G];
          ny = a.ys[i + G];
          nq = a.qs[i + G];
        }
      }
      if (LL) {
        const uint32_t lb = __float_as_uint(pt.w);  // the leaf's column | row << 16
        const T ox = leaf_to_box<T>(lb & 0xFFFFu, sh) * sL;
        const T oy = leaf_to_box<T>(lb >> 16, sh) * sL;
        q = (T)pt.z;
        wr = ((T)pt.x + ox) * is;
        wi = ((T)pt.y + oy) * is;
      } else {
        q = (T)pq;
        wr = ((T)px - cx) * is;
        wi = ((T)py - cy) * is;
      }
      re[0] += q;
      T pr = q * wr, pi = q * wi;  // q w^m
#pragma unroll
      for (int m = 1; m <= PK; ++m) {
        re[m] += pr;
        im[m] += pi;
        const T nr = pr * wr - pi * wi;
        pi = pr * wi + pi * wr;
        pr = nr;
      }
    }
  }
  for (int d = 1; d < G; d <<= 1) {
#pragma unroll
    for (int m = 0; m <= PK; ++m) {
      re[m] += __shfl_xor(re[m], d, 64);
      im[m] += __shfl_xor(im[m], d, 64);
    }
  }
  if (!valid || r != 0) return;
  const int cs = a.cs;
  T* out;
  if (S == 1)
    out = (sizeof(T) == 8 ? (T*)a.mom64 : (T*)a.mom32) + (lt.off[k] + b) * cs;
  else
    out = (sizeof(T) == 8 ? (T*)a.part64 : (T*)a.part32) + (pl.part_off[k] + b * S + j) * cs;
#pragma unroll
  for (int m = 1; m <= PB; ++m) {
    T vr = (T)0, vi = (T)0;
    if (m <= PK) {
      const T f = (T)(-1.0 / (double)m);
      vr = m <= p ? re[m] * f : (T)0;
      vi = m <= p ? im[m] * f : (T)0;
    }
    out[2 * (m - 1)] = vr;
    out[2 * (m - 1) + 1] = vi;
  }
  out[2 * PB] = re[0];
  out[2 * PB + 1] = (T)0;
}

template <typename T, int PB, bool LL, bool FULL>
__global__ __launch_bounds__(256) void k_p2m2d(FmmArgs a, P2mPlan pl) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if ((t & ~(int64_t)63) >= pl.thr_off[pl.khi + 1]) return;  // whole wave beyond the end
  const LevelTable& lt = a.lt;
  int k = pl.klo;
  while (k < pl.khi && t >= pl.thr_off[k + 1]) ++k;
  const int G = pl.G[k], S = pl.S[k];
  const int64_t local = t - pl.thr_off[k];
  const int64_t nb = (int64_t)lt.nsys << (2 * k);
  const int64_t b = local / (G * S);
  const bool valid = b < nb;
  const int rem = (int)(local - b * G * S);
  const int j = rem / G, r = rem - (rem / G) * G;
  const int p = FULL ? PB : a.ord[k];  // this level's order (waves never straddle levels)
  with_order_bucket<PB, FULL>(p, [&](auto pk) {
    p2m_item<T, PB, decltype(pk)::value, LL>(a, pl, k, p, valid, b, j, r, G, S);
  });
}

// Slice partials of every level of a launch added up in one launch: one wave
// per (level, box, coefficient), lane l taking slices l, l + 64, ... in order,
// then a fixed butterfly across the wave (deterministic).  jb.off[i] is the
// first wave of the i-th level with slices, jb.lev[i] that level.
struct SliceJob {
  int n;
  int lev[kMaxLevels2D + 1];
  int64_t off[kMaxLevels2D + 2];
};

template <typename T>
__global__ __launch_bounds__(256) void k_p2m_slices(FmmArgs a, P2mPlan pl, SliceJob jb) {
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wv >= jb.off[jb.n]) return;  // whole waves
  int i = 0;
  while (i + 1 < jb.n && wv >= jb.off[i + 1]) ++i;
  const int k = jb.lev[i];
  const int nc = 2 * order_bucket(a.p) + 2;
  const int64_t item = wv - jb.off[i];
  const int64_t b = item / nc;
  const int c = (int)(item - b * nc);
  const int S = pl.S[k];
  const T* part = sizeof(T) == 8 ? (const T*)a.part64 : (const T*)a.part32;
  T* mom = sizeof(T) == 8 ? (T*)a.mom64 : (T*)a.mom32;
  const T* src = part + (pl.part_off[k] + b * S) * a.cs + c;
  T acc = 0;
  for (int j = lane; j < S; j += 64) acc += src[(int64_t)j * a.cs];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if (lane == 0) mom[(a.lt.off[k] + b) * a.cs + c] = acc;
}

template <int PB>
static void p2m_dispatch(const FmmArgs& a, bool ll, bool f64, hipStream_t st) {
  const P2mPlan pl = make_p2m_plan(2, a.klo, a.khi, a.n, a.lt.nsys);
  const int64_t thr = pl.thr_off[a.khi + 1];
  const dim3 grid((unsigned)((thr + 255) / 256));
  const bool full = a.ord_full != 0;
  if (f64) {
    if (ll && full)
      hipLaunchKernelGGL((k_p2m2d<double, PB, true, true>), grid, dim3(256), 0, st, a, pl);
    else if (ll)
      hipLaunchKernelGGL((k_p2m2d<double, PB, true, false>), grid, dim3(256), 0, st, a, pl);
    else if (full)
      hipLaunchKernelGGL((k_p2m2d<double, PB, false, true>), grid, dim3(256), 0, st, a, pl);
    else
      hipLaunchKernelGGL((k_p2m2d<double, PB, false, false>), grid, dim3(256), 0, st, a, pl);
  } else {
    if (full)
      hipLaunchKernelGGL((k_p2m2d<float, PB, true, true>), grid, dim3(256), 0, st, a, pl);
    else
      hipLaunchKernelGGL((k_p2m2d<float, PB, true, false>), grid, dim3(256), 0, st, a, pl);
  }
  SliceJob jb{};
  int64_t waves = 0;
  for (int k = a.klo; k <= a.khi; ++k)
    if (pl.S[k] > 1) {
      jb.lev[jb.n] = k;
      jb.off[jb.n] = waves;
      ++jb.n;
      waves += ((int64_t)a.lt.nsys << (2 * k)) * (2 * PB + 2);
    }
  jb.off[jb.n] = waves;
  if (jb.n > 0) {
    const dim3 sgrid((unsigned)((waves * 64 + 255) / 256));
    if (f64)
      hipLaunchKernelGGL(k_p2m_slices<double>, sgrid, dim3(256), 0, st, a, pl, jb);
    else
      hipLaunchKernelGGL(k_p2m_slices<float>, sgrid, dim3(256), 0, st, a, pl, jb);
  }
}

void launch_p2m2d(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st) {
  if (a.khi < a.klo || a.n <= 0) return;
  SFFMM_PB_DISPATCH(p2m_dispatch, a.p, a, leaf_local, fp64, st);
}

// ---------------------------------------------------------------------------
// L2P: one thread per sorted particle, every level; each level's polynomial
// and its derivative by Horner's rule (FP64 for levels < split, FP32 above),
// potential and field accumulated over levels in FP64.
// ---------------------------------------------------------------------------
// Loads a box's coefficient row (CS values, 16-byte aligned) with vector loads.
template <int CS>
__device__ __forceinline__ void load_row(const float* B, float (&r)[CS]) {
  const float4* v = reinterpret_cast<const float4*>(B);
#pragma unroll
  for (int i = 0; i < CS / 4; ++i) {
    const float4 t = v[i];
    r[4 * i] = t.x;
    r[4 * i + 1] = t.y;
    r[4 * i + 2] = t.z;
    r[4 * i + 3] = t.w;
  }
}
template <int CS>
__device__ __forceinline__ void load_row(const double* B, double (&r)[CS]) {
  const double2* v = reinterpret_cast<const double2*>(B);
#pragma unroll
  for (int i = 0; i < CS / 2; ++i) {
    const double2 t = v[i];
    r[2 * i] = t.x;
    r[2 * i + 1] = t.y;
  }
}

// Horner's rule for g(w) = sum_l B_l w^l and g'(w) over the coefficients
// 0..p of one box (row layout above): g' <- g' w + g, then g <- g w + B_l,
// each complex step as two fused multiply-adds per real part.  The loop runs
// to PK, the order bucket of p (locals above a level's order are not
// formed): the coefficients above p, only possible past the next lower
// bucket, enter as zeros, which leaves g and g' unchanged.  FULL: p == PK == PB.
__host__ __device__ constexpr int lower_bucket(int pk) {
  return pk <= 8 ? 0 : pk <= 12 ? 8 : pk <= 16 ? 12 : pk <= 20 ? 16 : pk <= 24 ? 20 : 24;
}

template <typename T, int PB, int PK, bool FULL>
__device__ __forceinline__ void horner_row(const T (&r)[(2 * PB + 2 + 3) / 4 * 4], int p, T wr,
                                           T wi, T& gr, T& gi, T& dr, T& di) {
  gr = gi = dr = di = (T)0;
#pragma unroll
  for (int l = PK; l >= 0; --l) {
    T br = l ? r[2 * (l - 1)] : r[2 * PB];
    T bi = l ? r[2 * (l - 1) + 1] : r[2 * PB + 1];
    if (!FULL && l > lower_bucket(PK)) {
      br = l <= p ? br : (T)0;
      bi = l <= p ? bi : (T)0;
    }
    const T ndr = fma(dr, wr, fma(-di, wi, gr));
    const T ndi = fma(dr, wi, fma(di, wr, gi));
    const T ngr = fma(gr, wr, fma(-gi, wi, br));
    const T ngi = fma(gr, wi, fma(gi, wr, bi));
    dr = ndr;
    di = ndi;
    gr = ngr;
    gi = ngi;
  }
}

template <typename T, int PB, int PK, bool FULL>
__device__ __forceinline__ void horner(const T* B, int p, T wr, T wi, T& gr, T& gi, T& dr,
                                       T& di) {
  constexpr int CS = (2 * PB + 2 + 3) / 4 * 4;
  T r[CS];
  load_row<CS>(B, r);  // (the chunks no coefficient <= PK lies in are never loaded)
  horner_row<T, PB, PK, FULL>(r, p, wr, wi, gr, gi, dr, di);
}

// g and g' of one level at the particle for the coarse levels, whose boxes hold
// many consecutive sorted particles: the distinct boxes of the wave are taken
// one at a time (usually one); each box's coefficient row is read from a
// wave-uniform address, which the compiler turns into scalar loads (the row
// arrives in scalar registers: no vector memory traffic, no lane reads), and
// is evaluated by the lanes in that box.  Lanes with live == false only take
// part in the wave's box selection.
template <typename T, int PB, int PK, bool FULL>
__device__ __forceinline__ void eval_level_shared(const T* base, uint32_t box, int cs, int p, T wr,
                                                  T wi, bool live, T& gr, T& gi, T& dr, T& di) {
  constexpr int CS = (2 * PB + 2 + 3) / 4 * 4;
  gr = gi = dr = di = (T)0;
  bool done = !live;
  for (;;) {
    const uint64_t todo = __ballot(!done);
    if (todo == 0) break;
    const uint32_t b0 = __builtin_amdgcn_readlane(box, __ffsll((unsigned long long)todo) - 1);
    T r[CS];
    load_row<CS>(base + (int64_t)b0 * cs, r);  // a wave-uniform address
    if (!done && box == b0) {
      horner_row<T, PB, PK, FULL>(r, p, wr, wi, gr, gi, dr, di);
      done = true;
    }
  }
}

// Offset of the particle from the centre of its level-k box in units of s_k.
template <typename T, bool LL>
__device__ __forceinline__ void box_offset(const LevelTable& lt, int k, uint32_t lx, uint32_t ly,
                                           float xl, float yl, double x, double y, T& wr, T& wi) {
  const int sh = lt.L - k;
  if (LL) {
    if (sizeof(T) == 8) {
      wr = (T)(((double)xl + leaf_to_box<double>(lx, sh) * lt.s[lt.L]) * lt.inv_s[k]);
      wi = (T)(((double)yl + leaf_to_box<double>(ly, sh) * lt.s[lt.L]) * lt.inv_s[k]);
    } else {
      const float sL = (float)lt.s[lt.L], is = (float)lt.inv_s[k];
      wr = (T)((xl + leaf_to_box<float>(lx, sh) * sL) * is);
      wi = (T)((yl + leaf_to_box<float>(ly, sh) * sL) * is);
    }
  } else {
    const double cx = lt.origin[0] + lt.s[k] * ((double)(lx >> sh) + 0.5);
    const double cy = lt.origin[1] + lt.s[k] * ((double)(ly >> sh) + 0.5);
    wr = (T)((x - cx) * lt.inv_s[k]);
    wi = (T)((y - cy) * lt.inv_s[k]);
  }
}

// Adds one level's far field: phi += Re g, E += (-Re g', Im g') / s_k.
template <typename T>
__device__ __forceinline__ void add_level(double is, T gr, T dr, T di, double& phi, double& ex,
                                          double& ey) {
  phi += (double)gr;
  if (sizeof(T) == 8) {
    ex -= (double)dr * is;
    ey += (double)di * is;
  } else {
    ex -= (double)(dr * (float)is);
    ey += (double)(di * (float)is);
  }
}

// ADA (adaptive depth): each particle adds the levels kmin..depth[j] only, every
// level through the wave's shared rows.
template <int PB, bool LL, bool FULL, bool ADA>
__global__ __launch_bounds__(256) void k_l2p2d(FmmArgs a) {
  constexpr int CS = (2 * PB + 2 + 3) / 4 * 4;
  // lanes past the end evaluate the last particle again and write nothing
  const int64_t jt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = jt < a.n;
  const int64_t j = live ? jt : a.n - 1;
  const LevelTable& lt = a.lt;
  const int L = lt.L;
  const uint32_t key = a.keys[j];
  const uint32_t lx = compact2(local2(key, L)), ly = compact2(local2(key, L) >> 1);
  const int cs = a.cs;
  float xl = 0, yl = 0;
  double x = 0, y = 0;
  if (LL) {
    const float4 pt = a.pts[j];
    xl = pt.x;
    yl = pt.y;
  } else {
    x = a.xs[j];
    y = a.ys[j];
  }
  double phi = 0.0, ex = 0.0, ey = 0.0;
  const int k32 = lt.split > lt.kmin ? lt.split : lt.kmin;  // first FP32 level
  if constexpr (ADA) {
    const int dj = a.depth[j];
    for (int k = lt.kmin; k <= L; ++k) {
      const uint32_t box = key >> (2 * (L - k));
      const int p = a.ord[k];
      const bool lk = live && k <= dj;  // lanes past their leaf level add zeros
      if (k < lt.split) {
        double wr, wi, gr, gi, dr, di;
        box_offset<double, LL>(lt, k, lx, ly, xl, yl, x, y, wr, wi);
        with_order_bucket<PB, FULL>(p, [&](auto pk) {
          eval_level_shared<double, PB, decltype(pk)::value, FULL>(
              a.loc64 + lt.off[k] * cs, box, cs, p, wr, wi, lk, gr, gi, dr, di);
        });
        add_level<double>(lt.inv_s[k], gr, dr, di, phi, ex, ey);
      } else {
        float wr, wi, gr, gi, dr, di;
        box_offset<float, LL>(lt, k, lx, ly, xl, yl, x, y, wr, wi);
        with_order_bucket<PB, FULL>(p, [&](auto pk) {
          eval_level_shared<float, PB, decltype(pk)::value, FULL>(
              a.loc32 + lt.off[k] * cs, box, cs, p, wr, wi, lk, gr, gi, dr, di);
        });
        add_level<float>(lt.inv_s[k], gr, dr, di, phi, ex, ey);
      }
    }
  } else if (LL && L >= k32 && L > lt.kmin) {
    // FP32 modes: the coarser levels go through the shared rows, then the
    // finest level's row (each lane its own leaf) is loaded and used (held
    // across the coarse levels it cost 34 registers and two waves per SIMD)
    for (int k = lt.kmin; k < L; ++k) {
      const uint32_t box = key >> (2 * (L - k));
      const int p = a.ord[k];
      if (k < lt.split) {
        double wr, wi, gr, gi, dr, di;
        box_offset<double, LL>(lt, k, lx, ly, xl, yl, x, y, wr, wi);
        with_order_bucket<PB, FULL>(p, [&](auto pk) {
          eval_level_shared<double, PB, decltype(pk)::value, FULL>(
              a.loc64 + lt.off[k] * cs, box, cs, p, wr, wi, live, gr, gi, dr, di);
        });
        add_level<double>(lt.inv_s[k], gr, dr, di, phi, ex, ey);
      } else {
        float wr, wi, gr, gi, dr, di;
        box_offset<float, LL>(lt, k, lx, ly, xl, yl, x, y, wr, wi);
        with_order_bucket<PB, FULL>(p, [&](auto pk) {
          eval_level_shared<float, PB, decltype(pk)::value, FULL>(
              a.loc32 + lt.off[k] * cs, box, cs, p, wr, wi, live, gr, gi, dr, di);
        });
        add_level<float>(lt.inv_s[k], gr, dr, di, phi, ex, ey);
      }
    }
    float rL[CS];
    load_row<CS>(a.loc32 + (lt.off[L] + key) * cs, rL);
    float wr, wi, gr, gi, dr, di;
    box_offset<float, LL>(lt, L, lx, ly, xl, yl, x, y, wr, wi);
    const int pL = a.ord[L];
    with_order_bucket<PB, FULL>(pL, [&](auto pk) {
      horner_row<float, PB, decltype(pk)::value, FULL>(rL, pL, wr, wi, gr, gi, dr, di);
    });
    add_level<float>(lt.inv_s[L], gr, dr, di, phi, ex, ey);
  } else {
    for (int k = lt.kmin; k <= L; ++k) {
      const uint32_t box = key >> (2 * (L - k));
      const int p = a.ord[k];
      if (k < lt.split) {
        double wr, wi, gr, gi, dr, di;
        box_offset<double, LL>(lt, k, lx, ly, xl, yl, x, y, wr, wi);
        with_order_bucket<PB, FULL>(p, [&](auto pk) {
          constexpr int PK = decltype(pk)::value;
          if (k < L || LL)  // (FP32 modes reach here only when level 2 is the finest)
            eval_level_shared<double, PB, PK, FULL>(a.loc64 + lt.off[k] * cs, box, cs, p, wr, wi,
                                                    live, gr, gi, dr, di);
          else
            horner<double, PB, PK, FULL>(a.loc64 + (lt.off[k] + box) * cs, p, wr, wi, gr, gi, dr,
                                         di);
        });
        add_level<double>(lt.inv_s[k], gr, dr, di, phi, ex, ey);
      } else {
        float wr, wi, gr, gi, dr, di;
        box_offset<float, LL>(lt, k, lx, ly, xl, yl, x, y, wr, wi);
        with_order_bucket<PB, FULL>(p, [&](auto pk) {
          horner<float, PB, decltype(pk)::value, FULL>(a.loc32 + (lt.off[k] + box) * cs, p, wr,
                                                       wi, gr, gi, dr, di);
        });
        add_level<float>(lt.inv_s[k], gr, dr, di, phi, ex, ey);
      }
    }
  }
  // near + far in FP64, scattered back to input order
  if (!live) return;
  double* pot = a.pot;
  double* field = a.field;
  if (a.io) {
    pot = a.io->pot;
    field = a.io->field;
  }
  const int64_t o = a.perm[j];
  pot[o] = phi + a.near_pot[j];
  if (field) {
    const double fx = ex + a.near_ex[j], fy = ey + a.near_ey[j];
    if ((reinterpret_cast<uintptr_t>(field) & 15) == 0) {  // one 16-byte store
      reinterpret_cast<double2*>(field)[o] = make_double2(fx, fy);
    } else {
      field[2 * o] = fx;
      field[2 * o + 1] = fy;
    }
  }
}

template <int PB, bool ADA>
static void l2p_dispatch_a(const FmmArgs& a, bool ll, hipStream_t st) {
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (ll) {
    if (a.ord_full)
      hipLaunchKernelGGL((k_l2p2d<PB, true, true, ADA>), grid, dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_l2p2d<PB, true, false, ADA>), grid, dim3(256), 0, st, a);
  } else {
    if (a.ord_full)
      hipLaunchKernelGGL((k_l2p2d<PB, false, true, ADA>), grid, dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_l2p2d<PB, false, false, ADA>), grid, dim3(256), 0, st, a);
  }
}

template <int PB>
static void l2p_dispatch(const FmmArgs& a, bool ll, hipStream_t st) {
  if (a.depth)
    l2p_dispatch_a<PB, true>(a, ll, st);
  else
    l2p_dispatch_a<PB, false>(a, ll, st);
}

void launch_l2p2d(const FmmArgs& a, bool leaf_local, hipStream_t st) {
  if (a.n <= 0) return;
  SFFMM_PB_DISPATCH(l2p_dispatch, a.p, a, leaf_local, st);
}

// ---------------------------------------------------------------------------
// P2P: one thread per sorted target; sources from the target's leaf and its
// adjacent leaves; the near field is written in sorted order (L2P adds the far
// field and scatters back to input order).  Consecutive targets share leaves, so
// a wave's source loads are broadcasts of a few addresses.  Pairs with r = 0
// (the target itself, coincident points) contribute nothing.
// ---------------------------------------------------------------------------
// one source: pairs with r = 0 (the target itself, coincident points) add nothing
__device__ __forceinline__ void pair2_f64(double x, double y, double sx, double sy, double q,
                                          double& phi, double& ex, double& ey) {
  const double dx = x - sx, dy = y - sy;
  const double r2 = dx * dx + dy * dy;
  if (r2 == 0.0) return;
  phi += q * 0.5 * log(r2);
  const double w = q / r2;
  ex -= w * dx;
  ey -= w * dy;
}

// lsh = 2 (L - d) when the launch works at level d = lt.L of an adaptive tree
// of depth L: leaf keys and leaf offsets are those of level d, and only the
// targets whose leaf lies at level d are taken.
__global__ __launch_bounds__(256) void k_p2p2d_f64(FmmArgs a, int lsh) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const LevelTable& lt = a.lt;
  if (a.depth && a.depth[j] != lt.L) return;
  const uint32_t key = a.keys[j] >> lsh;
  const uint32_t sysbits = key & ~local2(0xFFFFFFFFu, lt.L);
  const int lx = (int)compact2(local2(key, lt.L)), ly = (int)compact2(local2(key, lt.L) >> 1);
  const int nl = 1 << lt.L;
  const double x = a.xs[j], y = a.ys[j];
  double phi = 0.0, ex = 0.0, ey = 0.0;
  for (int ny = ly - 1; ny <= ly + 1; ++ny) {
    if (ny < 0 || ny >= nl) continue;
    for (int nx = lx - 1; nx <= lx + 1; ++nx) {
      if (nx < 0 || nx >= nl) continue;
      const uint32_t nk = sysbits | spread2(nx) | (spread2(ny) << 1);
      const int32_t i0 = a.leaf_start[(int64_t)nk << lsh], i1 = a.leaf_start[(int64_t)(nk + 1) << lsh];
      // sources four at a time, their loads issued together (the sums keep
      // the source order)
      int32_t i = i0;
      for (; i + 4 <= i1; i += 4) {
        double sx[4], sy[4], sq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          sx[u] = a.xs[i + u];
          sy[u] = a.ys[i + u];
          sq[u] = a.qs[i + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) pair2_f64(x, y, sx[u], sy[u], sq[u], phi, ex, ey);
      }
      for (; i < i1; ++i) pair2_f64(x, y, a.xs[i], a.ys[i], a.qs[i], phi, ex, ey);
    }
  }
  a.near_pot[j] = phi;
  a.near_ex[j] = ex;
  a.near_ey[j] = ey;
}

// FP32 pair terms from leaf-local coordinates (leaf-centre offsets are
// multiples of s_L, exact in FP32); log2 and reciprocal on the hardware
// transcendental unit; running sums flushed to FP64 every 32 sources.
// Every r^2 carries a floor kP2pEps = 2^-96 as the addend of its first fused
// multiply-add: no instruction of its own, and log2 and the reciprocal stay
// finite without a compare and select per pair (12 -> 10 VALU instructions per
// pair in the direct kernel).  The floor moves r^2 of a pair at r = 1e-12 by
// 1.3e-5 of itself, below the FP32 resolution of leaf-local coordinates for
// any pair that close.  The target's own record meets itself with
// dx = dy = 0, so r^2 = 2^-96 exactly: its field terms are q 2^96 * 0 = 0 (finite
// for |q| < 2^32) and its potential term is the exact product q * log2(2^-96),
// which the target takes back once, in FP64, after its sums.  A distinct
// source at the target's own FP32 position counts as a pair at r = 2^-48.
constexpr float kP2pEps = 0x1p-96f;

// Near field of FP32 modes in two launches.  The tile kernel stages, per
// workgroup, the leaf-local records of a 4 x 4-leaf tile's 6 x 6-leaf halo in
// LDS, halo rows contiguous, so that each target's three neighbour rows are
// three contiguous LDS spans; a source's halo column travels in the record's
// spare fourth component and gives its leaf-centre offset exactly, the
// product (column difference) x s_L being exact.  Five waves take the tile's
// targets in chunks of 64 (a tile holds 16 leaves' worth).  Tiles whose
// halo exceeds the stage are flagged and their targets are left to the direct
// kernel, which reads sources from global memory leaf by leaf (dense clusters,
// where leaves are large: there a wave mostly lies in one leaf and reads its
// sources with scalar loads).
constexpr int kP2pHalo = 6;  // 4 x 4 tile + one leaf on each side
constexpr int kP2pHaloLeaves = kP2pHalo * kP2pHalo;
constexpr int kP2pThreads = 320;
constexpr int kP2pPad = 8;  // zero records after the stage: a span's last batch may read past it
constexpr int kTileBatch = 4;  // LDS records loaded together per target (batches of 8 spilled)

// Tile form: the x offset from the source's halo column (exact); the y offset is
// added to the target once per neighbour row (ty = t.y + oy, one rounding of
// the size of the one it replaces).
__device__ __forceinline__ void pair_f32_h(const float4& t, const float4& s, float txh, float sL,
                                           float ty, float& fp, float& fx, float& fy) {
  const float dx = (t.x - s.x) + (txh - s.w) * sL, dy = ty - s.y;
  const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, kP2pEps));
  const float w = s.z * __builtin_amdgcn_rcpf(r2);
  fp += s.z * __builtin_amdgcn_logf(r2);
  fx -= w * dx;
  fy -= w * dy;
}

// Workgroup order of the near-field kernels: chunks of kXcdChunk consecutive
// workgroups (consecutive sorted targets or tiles) go to one XCD, the chunks dealt over
// the 8 XCDs in the order the hardware deals workgroups, so that the waves that
// share a neighbourhood mostly read its sources through one XCD's L2.  The
// grid is a multiple of 8 kXcdChunk workgroups (direct_grid) and the map is a
// permutation of it.
constexpr int kXcdChunk = 8;
__device__ __forceinline__ int64_t xcd_chunk_remap(int64_t bid) {
  const int64_t x = bid & 7, i = bid >> 3;
  return ((i / kXcdChunk) * 8 + x) * kXcdChunk + (i % kXcdChunk);
}
static dim3 direct_grid(int64_t n) {
  const int64_t per = 8 * kXcdChunk;
  return dim3((unsigned)(((n + 255) / 256 + per - 1) / per * per));
}

// Eight waves per SIMD (64 registers): a few spills at the row level cost less
// than the lower occupancy without them (measured beside the moments chain).
__global__ __launch_bounds__(kP2pThreads, 8) void k_p2p2d_f32_tile(FmmArgs a, int cap) {
  extern __shared__ float4 src[];  // cap + kP2pPad records
  __shared__ int32_t hstart[kP2pHaloLeaves];
  __shared__ int32_t hoff[kP2pHaloLeaves + 1];
  const LevelTable& lt = a.lt;
  const int L = lt.L, nl = 1 << L, tid = threadIdx.x;
  const int64_t tl = xcd_chunk_remap(blockIdx.x);
  if (tl >= ((int64_t)lt.nsys << (2 * (lt.L - 2)))) return;  // grid padding (workgroup-uniform)
  const uint32_t tile = (uint32_t)tl;
  const uint32_t k0 = tile << 4;  // first leaf key of the tile (system bits included)
  const uint32_t sysbits = k0 & ~local2(0xFFFFFFFFu, L);
  const uint32_t tm = local2(k0, L);
  const int bx0 = (int)compact2(tm), by0 = (int)compact2(tm >> 1);
  int cnt = 0;
  if (tid < kP2pHaloLeaves) {
    const int x = bx0 - 1 + tid % kP2pHalo, y = by0 - 1 + tid / kP2pHalo;
    int32_t s0 = 0;
    if (x >= 0 && x < nl && y >= 0 && y < nl) {
      const uint32_t k = sysbits | spread2((uint32_t)x) | (spread2((uint32_t)y) << 1);
      s0 = a.leaf_start[k];
      cnt = a.leaf_start[k + 1] - s0;
    }
    hstart[tid] = s0;
  }
  if (tid < 64) {  // offsets of the halo leaves: an inclusive scan across wave 0
    int v = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int u = __shfl_up(v, d, 64);
      if (tid >= d) v += u;
    }
    if (tid < kP2pHaloLeaves) hoff[tid + 1] = v;
    if (tid == 0) hoff[0] = 0;
  }
  __syncthreads();
  const int total = hoff[kP2pHaloLeaves];
  if (tid == 0) a.p2p_over[tile] = total > cap ? 1 : 0;
  if (total > cap) return;  // workgroup-uniform
  for (int e = tid; e < total; e += kP2pThreads) {
    int lo = 0, hi = kP2pHaloLeaves - 1;  // the last halo leaf starting at or before e
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (hoff[mid] <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    float4 v = a.pts[hstart[lo] + (e - hoff[lo])];
    v.w = (float)(lo % kP2pHalo);
    src[e] = v;
  }
  if (tid < kP2pPad) src[total + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
  __syncthreads();
  const int32_t t0 = a.leaf_start[k0], t1 = a.leaf_start[k0 + 16];
  const float sL = (float)lt.s[L];
  // Targets in chunks of 64, one chunk per wave.  A full chunk gives each lane
  // one target.  A last, partial chunk of m targets gives each target P = 64 / W
  // lanes (W the power of two >= m): the lanes of a target take every P-th batch
  // of 8 sources and their sums meet in a butterfly, so the wave is not held
  // for a whole target loop by a few lanes.
  const int wave = tid >> 6, lane = tid & 63;
  for (int32_t base = t0 + wave * 64; base < t1; base += kP2pThreads) {
    const int m = t1 - base < 64 ? t1 - base : 64;
    int lw = 0;  // log2 W
    while ((1 << lw) < m) ++lw;
    const int W = 1 << lw, P = 64 >> lw;
    const int ti = lane & (W - 1), part = lane >> lw;
    const bool live = ti < m;
    const int32_t j = base + (live ? ti : 0);
    const uint32_t key = local2(a.keys[j], L);
    const int tx = (int)compact2(key) - bx0, ty = (int)compact2(key >> 1) - by0;
    const float4 t = a.pts[j];
    const float txh = (float)(tx + 1);  // halo column of the target's leaf
    double phi = 0.0, ex = 0.0, ey = 0.0;
#pragma unroll 1
    for (int dy = 0; dy < 3 && live; ++dy) {
      const int h = (ty + dy) * kP2pHalo + tx;  // halo leaves h, h + 1, h + 2
      const int c0 = hoff[h], c1 = hoff[h + 3];
      const float ty = t.y + (float)(1 - dy) * sL;
      if (P == 1) {  // wave-uniform
        for (int c = c0; c < c1; c += 32) {
          const int ce = c + 32 < c1 ? c + 32 : c1;
          float fp = 0.f, fx = 0.f, fy = 0.f;
          int i = c;
          for (; i + kTileBatch <= ce; i += kTileBatch) {
            float4 sb[kTileBatch];
#pragma unroll
            for (int u = 0; u < kTileBatch; ++u) sb[u] = src[i + u];
#pragma unroll
            for (int u = 0; u < kTileBatch; ++u) pair_f32_h(t, sb[u], txh, sL, ty, fp, fx, fy);
          }
          if (i < ce) {  // the last few sources: a full batch with the charges past the span
                         // zeroed (the stage has kP2pPad zero records after its end)
            float4 sb[kTileBatch];
#pragma unroll
            for (int u = 0; u < kTileBatch; ++u) {
              sb[u] = src[i + u];
              if (i + u >= ce) sb[u].z = 0.f;
            }
#pragma unroll
            for (int u = 0; u < kTileBatch; ++u) pair_f32_h(t, sb[u], txh, sL, ty, fp, fx, fy);
          }
          phi += (double)fp;
          ex += (double)fx;
          ey += (double)fy;
        }
      } else {
        // this lane's batches start at c0 + kTileBatch part and step
        // kTileBatch P; 32 / kTileBatch of them per FP32 running sum; charges
        // past the span zeroed
        constexpr int kPerSum = 32 / kTileBatch;
        for (int g = c0 + kTileBatch * part; g < c1; g += 32 * P) {
          float fp = 0.f, fx = 0.f, fy = 0.f;
#pragma unroll 1
          for (int u4 = 0, cb = g; u4 < kPerSum && cb < c1; ++u4, cb += kTileBatch * P) {
            float4 sb[kTileBatch];
#pragma unroll
            for (int u = 0; u < kTileBatch; ++u) {
              sb[u] = src[cb + u];
              if (cb + u >= c1) sb[u].z = 0.f;
            }
#pragma unroll
            for (int u = 0; u < kTileBatch; ++u) pair_f32_h(t, sb[u], txh, sL, ty, fp, fx, fy);
          }
          phi += (double)fp;
          ex += (double)fx;
          ey += (double)fy;
        }
      }
    }
    for (int d = W; d < 64; d <<= 1) {  // the P lanes of a target (none when P = 1)
      phi += __shfl_xor(phi, d, 64);
      ex += __shfl_xor(ex, d, 64);
      ey += __shfl_xor(ey, d, 64);
    }
    if (live && part == 0) {
      phi -= (double)t.z * (double)__builtin_amdgcn_logf(kP2pEps);  // the target's own term
      a.near_pot[j] = phi * 0.34657359027997264;  // (ln 2) / 2: log r = log2(r^2) ln2 / 2
      a.near_ex[j] = ex;
      a.near_ey[j] = ey;
    }
  }
}

// One neighbour leaf's sources [i0, i1) against the target t, running sums in
// FP32 flushed to FP64 every 32 sources.  When the range is wave-uniform the
// loads become scalar loads (the sources arrive in scalar registers, no vector
// memory traffic per pair).
// The leaf-centre offset (ox, oy) is added to the target once per leaf: one
// rounding of the size of the one it replaces in (t - s) + o.
__device__ __forceinline__ void pair_f32_o(float tx, float ty, const float4& s, float& fp,
                                           float& fx, float& fy) {
  const float dx = tx - s.x, dy = ty - s.y;
  const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, kP2pEps));
  const float w = s.z * __builtin_amdgcn_rcpf(r2);
  fp += s.z * __builtin_amdgcn_logf(r2);
  fx -= w * dx;
  fy -= w * dy;
}

__device__ __forceinline__ void p2p_leaf_f32(const float4* __restrict__ pts, int32_t i0,
                                             int32_t i1, const float4& t, float ox, float oy,
                                             double& phi, double& ex, double& ey) {
  const float tx = t.x + ox, ty = t.y + oy;
  for (int32_t c0 = i0; c0 < i1; c0 += 32) {
    const int32_t c1 = c0 + 32 < i1 ? c0 + 32 : i1;
    float fp = 0.f, fx = 0.f, fy = 0.f;
    int32_t i = c0;
    // batches of 8 independent source loads
    for (; i + 8 <= c1; i += 8) {
      float4 sb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) sb[u] = pts[i + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) pair_f32_o(tx, ty, sb[u], fp, fx, fy);
    }
    for (; i < c1; ++i) pair_f32_o(tx, ty, pts[i], fp, fx, fy);
    phi += (double)fp;
    ex += (double)fx;
    ey += (double)fy;
  }
}

// lsh as in k_p2p2d_f64 (adaptive depth: pts rebased to the level-d box centres).
__global__ __launch_bounds__(256) void k_p2p2d_f32(FmmArgs a, int tiled,
                                                  const float4* __restrict__ pts,
                                                  const int32_t* __restrict__ leaf_start, int lsh) {
  const int64_t j = xcd_chunk_remap(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const LevelTable& lt = a.lt;
  if (a.depth && a.depth[j] != lt.L) return;
  const uint32_t key = a.keys[j] >> lsh;
  if (tiled && !a.p2p_over[key >> 4]) return;  // done by the tile kernel
  const int nl = 1 << lt.L;
  const float sL = (float)lt.s[lt.L];
  const float4 t = pts[j];
  double phi = 0.0, ex = 0.0, ey = 0.0;
  const uint32_t lmask = local2(0xFFFFFFFFu, lt.L);
  const int lx = (int)compact2(key & lmask), ly = (int)compact2((key & lmask) >> 1);
  // The wave's distinct leaves (its targets are consecutive in sorted order, so
  // dense leaves give one or two): when there are at most four, of one system,
  // whose neighbourhoods fit in a 4 x 4-leaf box, and the sources of that box
  // are at most 1.2 x those of the largest single neighbourhood (a wave in one
  // leaf always), the wave walks the box with uniform leaf ranges and sources
  // (scalar loads), each lane taking the leaves next to its own; its leaves
  // come in the order of its own 3 x 3 walk, so the sums are the same as with
  // the per-lane walk below, which reads sources with vector loads.
  uint64_t todo = __ballot(true);
  int nd = 0, bx0 = 0, bx1 = -1, by0 = 0, by1 = -1;
  int dx0 = 0, dy0 = 0, dx1 = 0, dy1 = 0, dx2 = 0, dy2 = 0, dx3 = 0, dy3 = 0;
  uint32_t sys0 = 0;
  bool shared = true;
  while (todo != 0 && shared) {
    const uint32_t kk = __builtin_amdgcn_readlane(key, __ffsll((unsigned long long)todo) - 1);
    todo &= ~__ballot(key == kk);
    const int kx = (int)compact2(kk & lmask), ky = (int)compact2((kk & lmask) >> 1);
    const uint32_t ks = kk & ~lmask;
    if (nd == 0) {
      sys0 = ks;
      bx0 = kx - 1;
      bx1 = kx + 1;
      by0 = ky - 1;
      by1 = ky + 1;
    } else {
      bx0 = min(bx0, kx - 1);
      bx1 = max(bx1, kx + 1);
      by0 = min(by0, ky - 1);
      by1 = max(by1, ky + 1);
    }
    if (nd == 0) {
      dx0 = kx;
      dy0 = ky;
    } else if (nd == 1) {
      dx1 = kx;
      dy1 = ky;
    } else if (nd == 2) {
      dx2 = kx;
      dy2 = ky;
    } else {
      dx3 = kx;
      dy3 = ky;
    }
    ++nd;
    shared = nd <= 4 && ks == sys0 && (bx1 - bx0 + 1) * (by1 - by0 + 1) <= 16;
  }
  if (shared && nd > 1) {
    int usum = 0, o0 = 0, o1 = 0, o2 = 0, o3 = 0;
    for (int ny = max(by0, 0); ny <= min(by1, nl - 1); ++ny)
      for (int nx = max(bx0, 0); nx <= min(bx1, nl - 1); ++nx) {
        const uint32_t nk = sys0 | spread2(nx) | (spread2(ny) << 1);
        const int c = leaf_start[(int64_t)(nk + 1) << lsh] - leaf_start[(int64_t)nk << lsh];
        usum += c;
        if (abs(nx - dx0) <= 1 && abs(ny - dy0) <= 1) o0 += c;
        if (abs(nx - dx1) <= 1 && abs(ny - dy1) <= 1) o1 += c;
        if (nd > 2 && abs(nx - dx2) <= 1 && abs(ny - dy2) <= 1) o2 += c;
        if (nd > 3 && abs(nx - dx3) <= 1 && abs(ny - dy3) <= 1) o3 += c;
      }
    shared = 5 * usum <= 6 * max(max(o0, o1), max(o2, o3));
  }
  if (shared) {
    for (int ny = max(by0, 0); ny <= min(by1, nl - 1); ++ny) {
      const float oy = (float)(ly - ny) * sL;
      for (int nx = max(bx0, 0); nx <= min(bx1, nl - 1); ++nx) {
        const uint32_t nk = sys0 | spread2(nx) | (spread2(ny) << 1);
        const int32_t i0 = leaf_start[(int64_t)nk << lsh], i1 = leaf_start[(int64_t)(nk + 1) << lsh];
        if (abs(nx - lx) <= 1 && abs(ny - ly) <= 1)
          p2p_leaf_f32(pts, i0, i1, t, (float)(lx - nx) * sL, oy, phi, ex, ey);
      }
    }
  } else {
    const uint32_t sysbits = key & ~lmask;
    for (int ny = ly - 1; ny <= ly + 1; ++ny) {
      if (ny < 0 || ny >= nl) continue;
      const float oy = (float)(ly - ny) * sL;
      for (int nx = lx - 1; nx <= lx + 1; ++nx) {
        if (nx < 0 || nx >= nl) continue;
        const uint32_t nk = sysbits | spread2(nx) | (spread2(ny) << 1);
        p2p_leaf_f32(pts, leaf_start[(int64_t)nk << lsh], leaf_start[(int64_t)(nk + 1) << lsh], t,
                     (float)(lx - nx) * sL, oy, phi, ex, ey);
      }
    }
  }
  phi -= (double)t.z * (double)__builtin_amdgcn_logf(kP2pEps);  // the target's own term
  a.near_pot[j] = phi * 0.34657359027997264;  // (ln 2) / 2: log r = log2(r^2) ln2 / 2
  a.near_ex[j] = ex;
  a.near_ey[j] = ey;
}

// LDS records staged per tile: 1.5 x the mean halo occupancy, in [512, 2048].
int p2p2d_tile_cap(const LevelTable& lt, int64_t n) {
  const double leaves = (double)((int64_t)lt.nsys << (2 * lt.L));
  const double want = 1.5 * kP2pHaloLeaves * (double)n / leaves;
  const int cap = ((int)std::min(want, 2048.0) + 127) / 128 * 128;
  return std::max(512, std::min(2048, cap));
}

// ---------------------------------------------------------------------------
// Adaptive depth (one system).  A particle's leaf level is the first level
// k >= kmin at which the 3 x 3 boxes around its level-k box hold at most
// adapt_near particles (L if none): the bound of its near field.  Those counts
// only fall with k, so all particles of a level-k box agree on whether their
// depth reaches k.
// ---------------------------------------------------------------------------
// Flags of level k, coarse to fine.  Bit 0 (open): k < L, the parent is open
// (or k = kmin) and the 3 x 3 boxes around the box hold more than adapt_near
// particles (a closed parent leaves no more than that around its children).
// Bit 1 (k_adapt_near, once bit 0 of the level is complete): some box of the
// 3 x 3 around it is open, i.e. its children are in the interaction list of an
// open box's children and their moments are read.
__global__ __launch_bounds__(256) void k_adapt_open(FmmArgs a, int k, uint8_t* open) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= ((int64_t)1 << (2 * k))) return;
  uint8_t o = 0;
  if (k == a.lt.kmin || (open[adapt_open_off(k - 1) + (b >> 2)] & 1))
    o = around_count2(a.leaf_start, a.lt.L, k, (int)compact2((uint32_t)b),
                      (int)compact2((uint32_t)b >> 1)) > a.adapt_near;
  open[adapt_open_off(k) + b] = o;
}

__global__ __launch_bounds__(256) void k_adapt_near(int k, uint8_t* open) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = 1 << k;
  if (b >= (int64_t)nb * nb) return;
  const int bx = (int)compact2((uint32_t)b), by = (int)compact2((uint32_t)b >> 1);
  uint8_t* f = open + adapt_open_off(k);
  uint8_t any = 0;
  for (int y = by - 1; y <= by + 1; ++y)
    for (int x = bx - 1; x <= bx + 1; ++x)
      if (x >= 0 && y >= 0 && x < nb && y < nb) any |= f[spread2(x) | (spread2(y) << 1)] & 1;
  f[b] |= (uint8_t)(any << 1);
}

// A particle's depth: the first level at which its box is closed.
__global__ __launch_bounds__(256) void k_adapt_depth(FmmArgs a, const uint8_t* open,
                                                     uint8_t* depth) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const int L = a.lt.L;
  const uint32_t key = local2(a.keys[j], L);
  int d = a.lt.kmin;
  while (d < L && (open[adapt_open_off(d) + (key >> (2 * (L - d)))] & 1)) ++d;
  depth[j] = (uint8_t)d;
}

void launch_adapt_depth(const FmmArgs& a, uint8_t* open, uint8_t* depth, hipStream_t st) {
  for (int k = a.lt.kmin; k < a.lt.L; ++k) {
    const int64_t nb = (int64_t)1 << (2 * k);
    const dim3 grid((unsigned)((nb + 255) / 256));
    hipLaunchKernelGGL(k_adapt_open, grid, dim3(256), 0, st, a, k, open);
    hipLaunchKernelGGL(k_adapt_near, grid, dim3(256), 0, st, k, open);
  }
  if (a.n > 0)
    hipLaunchKernelGGL(k_adapt_depth, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a,
                       (const uint8_t*)open, depth);
}

// Adaptive FP32 near field of the targets whose depth d lies below L (each meets
// at most adapt_near sources).  Sources keep their leaf-local records; each
// one's offset from the target's leaf, (target leaf - source leaf) x s_L, is
// formed from the leaf column and row the record carries (exact), as in the
// tile kernel.  A wave whose targets share one level-d box reads the ranges
// and records from wave-uniform addresses (scalar loads); any other wave takes
// each lane's own box.
__device__ __forceinline__ void shallow_sum(const FmmArgs& a, int L, int d, int bx, int by,
                                            int ltx, int lty, const float4& t, float sL,
                                            double& phi, double& ex, double& ey) {
  const int dl = L - d, nb = 1 << d;
  for (int ny = by - 1; ny <= by + 1; ++ny) {
    if (ny < 0 || ny >= nb) continue;
    for (int nx = bx - 1; nx <= bx + 1; ++nx) {
      if (nx < 0 || nx >= nb) continue;
      const int64_t nk = (int64_t)(spread2(nx) | (spread2(ny) << 1));
      const int32_t i1 = a.leaf_start[(nk + 1) << (2 * dl)];
      for (int32_t c0 = a.leaf_start[nk << (2 * dl)]; c0 < i1; c0 += 32) {
        const int32_t c1 = c0 + 32 < i1 ? c0 + 32 : i1;
        float fp = 0.f, fx = 0.f, fy = 0.f;
        for (int32_t i = c0; i < c1; ++i) {
          const float4 sv = a.pts[i];
          const uint32_t lb = __float_as_uint(sv.w);  // the source leaf's column | row << 16
          const float dx = (t.x - sv.x) + (float)(ltx - (int)(lb & 0xFFFFu)) * sL;
          const float dy = (t.y - sv.y) + (float)(lty - (int)(lb >> 16)) * sL;
          const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, kP2pEps));
          const float w = sv.z * __builtin_amdgcn_rcpf(r2);
          fp += sv.z * __builtin_amdgcn_logf(r2);
          fx -= w * dx;
          fy -= w * dy;
        }
        phi += (double)fp;
        ex += (double)fx;
        ey += (double)fy;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_p2p2d_f32_shallow(FmmArgs a) {
  const int64_t jt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = jt < a.n ? jt : a.n - 1;
  const int L = a.lt.L, d = a.depth[j];
  const bool live = jt < a.n && d < L;  // depth L: the direct kernel
  const uint64_t lm = __ballot(live);
  if (lm == 0) return;
  const uint32_t key = local2(a.keys[j], L);
  const int ltx = (int)compact2(key), lty = (int)compact2(key >> 1);
  const uint32_t bk = key >> (2 * (L - d));  // level-d box
  const float sL = (float)a.lt.s[L];
  const float4 t = a.pts[j];
  const int f = __ffsll((unsigned long long)lm) - 1;
  const uint32_t b0 = __builtin_amdgcn_readlane(bk, f);
  const int d0 = __builtin_amdgcn_readlane(d, f);
  double phi = 0.0, ex = 0.0, ey = 0.0;
  if (__ballot(live && (bk != b0 || d != d0)) == 0) {
    shallow_sum(a, L, d0, (int)compact2(b0), (int)compact2(b0 >> 1), ltx, lty, t, sL, phi, ex, ey);
  } else if (live) {
    shallow_sum(a, L, d, (int)compact2(bk), (int)compact2(bk >> 1), ltx, lty, t, sL, phi, ex, ey);
  }
  if (!live) return;
  phi -= (double)t.z * (double)__builtin_amdgcn_logf(kP2pEps);  // the target's own term
  a.near_pot[j] = phi * 0.34657359027997264;
  a.near_ex[j] = ex;
  a.near_ey[j] = ey;
}

void launch_p2p2d(const FmmArgs& a, bool leaf_local, hipStream_t st) {
  if (a.n <= 0) return;
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (a.depth) {
    // the uniform near field of depth d for the targets whose depth is d (the
    // others leave at once): FP64, one launch per level; FP32, the direct
    // kernel for depth L and one launch for every shallower depth
    if (leaf_local) {
      hipLaunchKernelGGL(k_p2p2d_f32, direct_grid(a.n), dim3(256), 0, st, a, 0, a.pts,
                         a.leaf_start, 0);
      if (a.lt.L > a.lt.kmin) hipLaunchKernelGGL(k_p2p2d_f32_shallow, grid, dim3(256), 0, st, a);
    } else {
      for (int d = a.lt.kmin; d <= a.lt.L; ++d) {
        FmmArgs b = a;
        b.lt.L = d;
        hipLaunchKernelGGL(k_p2p2d_f64, grid, dim3(256), 0, st, b, 2 * (a.lt.L - d));
      }
    }
    return;
  }
  if (leaf_local) {
    const int tiled = a.lt.L >= 2 && a.p2p_over ? 1 : 0;
    if (tiled) {
      const int64_t tiles = (int64_t)a.lt.nsys << (2 * (a.lt.L - 2));
      const int cap = p2p2d_tile_cap(a.lt, a.n);
      const int64_t per = 8 * kXcdChunk;
      hipLaunchKernelGGL(k_p2p2d_f32_tile, dim3((unsigned)((tiles + per - 1) / per * per)),
                         dim3(kP2pThreads),
                         (size_t)(cap + kP2pPad) * sizeof(float4), st, a, cap);
    }
    hipLaunchKernelGGL(k_p2p2d_f32, direct_grid(a.n), dim3(256), 0, st, a, tiled, a.pts,
                       a.leaf_start, 0);
  } else {
    hipLaunchKernelGGL(k_p2p2d_f64, grid, dim3(256), 0, st, a, 0);
  }
}

}  // namespace sffmm
