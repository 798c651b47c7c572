// fmm2d.hip -- FP64 passes of the shift-free FMM for the 2D log kernel.
//
// Box vectors are complex Laurent coefficients of order p about each box
// centre, scaled by the box side s_k (Section 2.2.1, the vector space V; the
// map from a particle to its coefficients does not depend on the level, the
// Note closing Section 2.2.2):
//   A_0 = sum q,   A_m = -(1/m) sum q w^m,   w = (z - z_b) / s_k.
// Pass structure (no M2M, no L2L):
//   p2m : every level's box vectors straight from the Morton-sorted particles
//         (U-bar-1, U-bar-2 realised without a shift);
//   m2l : every level's local coefficients as the sum over the interaction list
//         of operator x source vector (D-bar-1);
//   l2p : every level's local polynomial evaluated at the particles and summed
//         over levels in FP64 (D-bar-2 and F(v) = L_{m^l}(v));
//   p2p : the near field (E-2), fused with near + far and the unsort.
#include "fmm_internal.h"

namespace sffmm {

__device__ __forceinline__ uint32_t d_compact2(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0F0F0F0Fu;
  v = (v | (v >> 4)) & 0x00FF00FFu;
  v = (v | (v >> 8)) & 0x0000FFFFu;
  return v;
}

__device__ __forceinline__ uint32_t d_spread2(uint32_t v) {
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__device__ __forceinline__ int level_of_box(const LevelTable& lt, int64_t g) {
  int k = lt.kmin;
  while (k < lt.L && g >= lt.off[k + 1]) ++k;
  return k;
}

// Wave-wide sum (64 lanes) by butterfly exchange; every lane gets the total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// ---------------------------------------------------------------------------
// P2M.  One wave per (level, box, slice).  Coarse levels split every box into
// a fixed number of slices so that every level offers thousands of waves; the
// slice partials are added in slice order by k_p2m_slices (deterministic, no
// floating-point atomics).
// ---------------------------------------------------------------------------
struct P2mPlan {
  int nlev;
  int32_t slices[kMaxLevels2D + 1];
  int64_t wave_off[kMaxLevels2D + 2];
  int64_t part_off[kMaxLevels2D + 1];  // in boxes*slices units
};

static P2mPlan make_p2m_plan(const LevelTable& lt) {
  P2mPlan pl{};
  int64_t w = 0, po = 0;
  for (int k = lt.kmin; k <= lt.L; ++k) {
    const int64_t nb = (int64_t)1 << (2 * k);
    int64_t s = 1;
    while (nb * s < 4096) s *= 4;
    pl.slices[k] = (int32_t)s;
    pl.wave_off[k] = w;
    pl.part_off[k] = po;
    w += nb * s;
    if (s > 1) po += nb * s;
  }
  pl.wave_off[lt.L + 1] = w;
  pl.nlev = lt.L - lt.kmin + 1;
  return pl;
}

size_t p2m2d_partial_entries(const LevelTable& lt, int cs) {
  if (lt.L < lt.kmin) return 1;
  P2mPlan pl = make_p2m_plan(lt);
  int64_t tot = 0;
  for (int k = lt.kmin; k <= lt.L; ++k)
    if (pl.slices[k] > 1) tot += ((int64_t)1 << (2 * k)) * pl.slices[k];
  return (size_t)(tot * cs + 1);
}

template <int PB>
__global__ __launch_bounds__(256) void k_p2m2d_f64(Fmm2dArgs a, P2mPlan pl) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const LevelTable& lt = a.lt;
  if (wid >= pl.wave_off[lt.L + 1]) return;
  int k = lt.kmin;
  while (k < lt.L && wid >= pl.wave_off[k + 1]) ++k;
  const int64_t local = wid - pl.wave_off[k];
  const int S = pl.slices[k];
  const int64_t b = local / S;
  const int j = (int)(local - b * S);
  const int sh = 2 * (lt.L - k);
  const int64_t s0 = a.leaf_start[b << sh], s1 = a.leaf_start[(b + 1) << sh];
  const int64_t len = s1 - s0;
  const int64_t lo = s0 + len * j / S, hi = s0 + len * (j + 1) / S;
  const uint32_t bx = d_compact2((uint32_t)b), by = d_compact2((uint32_t)b >> 1);
  const double cx = lt.origin[0] + lt.s[k] * ((double)bx + 0.5);
  const double cy = lt.origin[1] + lt.s[k] * ((double)by + 0.5);
  const double is = lt.inv_s[k];
  const int p = a.p;
  double re[PB + 1], im[PB + 1];
#pragma unroll
  for (int m = 0; m <= PB; ++m) re[m] = im[m] = 0.0;
  for (int64_t i = lo + lane; i < hi; i += 64) {
    const double q = a.qs[i];
    const double wr = (a.xs[i] - cx) * is, wi = (a.ys[i] - cy) * is;
    re[0] += q;
    double pr = q * wr, pi = q * wi;  // q w^m
#pragma unroll
    for (int m = 1; m <= PB; ++m) {
      if (m <= p) {
        re[m] += pr;
        im[m] += pi;
        const double nr = pr * wr - pi * wi;
        pi = pr * wi + pi * wr;
        pr = nr;
      }
    }
  }
  double* out;
  if (S == 1)
    out = a.mom + (lt.off[k] + b) * a.cs;
  else
    out = a.partial + (pl.part_off[k] + b * S + j) * a.cs;
#pragma unroll
  for (int m = 0; m <= PB; ++m) {
    if (m <= p) {
      const double sr = wave_sum(re[m]), si = wave_sum(im[m]);
      const double f = m == 0 ? 1.0 : -1.0 / (double)m;
      if (lane == 0) {
        out[2 * m] = sr * f;
        out[2 * m + 1] = si * f;
      }
    }
  }
}

__global__ void k_p2m_slices(Fmm2dArgs a, P2mPlan pl, int k) {
  const int64_t nb = (int64_t)1 << (2 * k);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nc = 2 * (a.p + 1);
  if (g >= nb * nc) return;
  const int64_t b = g / nc;
  const int c = (int)(g - b * nc);
  const int S = pl.slices[k];
  const double* src = a.partial + (pl.part_off[k] + b * S) * a.cs + c;
  double acc = 0.0;
  for (int j = 0; j < S; ++j) acc += src[(int64_t)j * a.cs];
  a.mom[(a.lt.off[k] + b) * a.cs + c] = acc;
}

template <int PB>
static void p2m_dispatch(const Fmm2dArgs& a, const P2mPlan& pl, hipStream_t st) {
  const int64_t waves = pl.wave_off[a.lt.L + 1];
  hipLaunchKernelGGL(k_p2m2d_f64<PB>, dim3((waves + 3) / 4), dim3(256), 0, st, a, pl);
  for (int k = a.lt.kmin; k <= a.lt.L; ++k)
    if (pl.slices[k] > 1) {
      const int64_t cnt = ((int64_t)1 << (2 * k)) * 2 * (a.p + 1);
      hipLaunchKernelGGL(k_p2m_slices, dim3((cnt + 255) / 256), dim3(256), 0, st, a, pl, k);
    }
}

#define SFFMM_PB_DISPATCH(fn, p, ...)          \
  do {                                         \
    if ((p) <= 8)                              \
      fn<8>(__VA_ARGS__);                      \
    else if ((p) <= 12)                        \
      fn<12>(__VA_ARGS__);                     \
    else if ((p) <= 16)                        \
      fn<16>(__VA_ARGS__);                     \
    else if ((p) <= 20)                        \
      fn<20>(__VA_ARGS__);                     \
    else if ((p) <= 24)                        \
      fn<24>(__VA_ARGS__);                     \
    else                                       \
      fn<30>(__VA_ARGS__);                     \
  } while (0)

void launch_p2m2d_f64(const Fmm2dArgs& a, hipStream_t st) {
  if (a.lt.L < a.lt.kmin) return;
  const P2mPlan pl = make_p2m_plan(a.lt);
  SFFMM_PB_DISPATCH(p2m_dispatch, a.p, a, pl, st);
}

// ---------------------------------------------------------------------------
// M2L reference kernel (FP64 VALU).  One thread per (target box, output
// coefficient l) over all levels in one launch.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_m2l2d_f64(Fmm2dArgs a) {
  const int P = a.p + 1;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.nbox_total * P) return;
  const int64_t tb = g / P;
  const int l = (int)(g - tb * P);
  const LevelTable& lt = a.lt;
  const int64_t gb = tb;  // levels are stored back to back from level kmin at box 0
  const int k = level_of_box(lt, gb);
  const uint32_t mort = (uint32_t)(gb - lt.off[k]);
  const int tx = (int)d_compact2(mort), ty = (int)d_compact2(mort >> 1);
  const int nb = 1 << k;
  const int xlo = (tx & 1) ? -3 : -2, ylo = (ty & 1) ? -3 : -2;
  double ar = 0.0, ai = 0.0, a0 = 0.0;
  for (int dy = ylo; dy <= ylo + 5; ++dy) {
    const int sy = ty + dy;
    if (sy < 0 || sy >= nb) continue;
    for (int dx = xlo; dx <= xlo + 5; ++dx) {
      const int sx = tx + dx;
      if (sx < 0 || sx >= nb) continue;
      if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
      const int64_t src = lt.off[k] + (d_spread2(sx) | (d_spread2(sy) << 1));
      const double* A = a.mom + src * a.cs;
      const double* T = a.op + ((size_t)((dx + 3) + 7 * (dy + 3)) * P + l) * P * 2;
      for (int m = 0; m < P; ++m) {
        const double tr = T[2 * m], ti = T[2 * m + 1];
        const double xr = A[2 * m], xi = A[2 * m + 1];
        ar += tr * xr - ti * xi;
        ai += tr * xi + ti * xr;
      }
      a0 += A[0];
    }
  }
  if (l == 0) ar += lt.log_s[k] * a0;
  a.loc[gb * a.cs + 2 * l] = ar;
  a.loc[gb * a.cs + 2 * l + 1] = ai;
}

void launch_m2l2d_f64(const Fmm2dArgs& a, hipStream_t st) {
  if (a.nbox_total <= 0) return;
  const int64_t thr = a.nbox_total * (a.p + 1);
  hipLaunchKernelGGL(k_m2l2d_f64, dim3((thr + 255) / 256), dim3(256), 0, st, a);
}

// ---------------------------------------------------------------------------
// L2P: one thread per sorted particle, every level, FP64 accumulation.
// ---------------------------------------------------------------------------
template <int PB>
__global__ __launch_bounds__(256) void k_l2p2d_f64(Fmm2dArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const LevelTable& lt = a.lt;
  const uint32_t key = a.keys[j];
  const uint32_t lx = d_compact2(key), ly = d_compact2(key >> 1);
  const double x = a.xs[j], y = a.ys[j];
  const int p = a.p;
  double phi = 0.0, ex = 0.0, ey = 0.0;
  for (int k = lt.kmin; k <= lt.L; ++k) {
    const int sh = lt.L - k;
    const double cx = lt.origin[0] + lt.s[k] * ((double)(lx >> sh) + 0.5);
    const double cy = lt.origin[1] + lt.s[k] * ((double)(ly >> sh) + 0.5);
    const double is = lt.inv_s[k];
    const double wr = (x - cx) * is, wi = (y - cy) * is;
    const double* B = a.loc + (lt.off[k] + (key >> (2 * sh))) * a.cs;
    double gr = 0.0, gi = 0.0, dr = 0.0, di = 0.0;
#pragma unroll
    for (int l = PB; l >= 0; --l) {
      if (l <= p) {
        const double ndr = dr * wr - di * wi + gr;
        di = dr * wi + di * wr + gi;
        dr = ndr;
        const double ngr = gr * wr - gi * wi + B[2 * l];
        gi = gr * wi + gi * wr + B[2 * l + 1];
        gr = ngr;
      }
    }
    phi += gr;
    ex -= dr * is;
    ey += di * is;
  }
  a.far_pot[j] = phi;
  a.far_ex[j] = ex;
  a.far_ey[j] = ey;
}

template <int PB>
static void l2p_dispatch(const Fmm2dArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_l2p2d_f64<PB>, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
}

void launch_l2p2d_f64(const Fmm2dArgs& a, hipStream_t st) {
  if (a.n <= 0) return;
  SFFMM_PB_DISPATCH(l2p_dispatch, a.p, a, st);
}

// ---------------------------------------------------------------------------
// P2P + combine + unsort: one thread per sorted target, sources from the
// target's leaf and its adjacent leaves.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_p2p2d_f64(Fmm2dArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const LevelTable& lt = a.lt;
  const uint32_t key = a.keys[j];
  const int lx = (int)d_compact2(key), ly = (int)d_compact2(key >> 1);
  const int nl = 1 << lt.L;
  const double x = a.xs[j], y = a.ys[j];
  double phi = 0.0, ex = 0.0, ey = 0.0;
  for (int ny = ly - 1; ny <= ly + 1; ++ny) {
    if (ny < 0 || ny >= nl) continue;
    for (int nx = lx - 1; nx <= lx + 1; ++nx) {
      if (nx < 0 || nx >= nl) continue;
      const uint32_t nk = d_spread2(nx) | (d_spread2(ny) << 1);
      const int32_t i0 = a.leaf_start[nk], i1 = a.leaf_start[nk + 1];
      for (int32_t i = i0; i < i1; ++i) {
        if (i == j) continue;
        const double dx = x - a.xs[i], dy = y - a.ys[i];
        const double r2 = dx * dx + dy * dy;
        if (r2 == 0.0) continue;
        const double q = a.qs[i];
        phi += q * 0.5 * log(r2);
        const double w = q / r2;
        ex -= w * dx;
        ey -= w * dy;
      }
    }
  }
  const int64_t o = a.perm[j];
  a.pot[o] = phi + a.far_pot[j];
  if (a.field) {
    a.field[2 * o] = ex + a.far_ex[j];
    a.field[2 * o + 1] = ey + a.far_ey[j];
  }
}

void launch_p2p2d_f64(const Fmm2dArgs& a, hipStream_t st) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(k_p2p2d_f64, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
}

}  // namespace sffmm
