// points2d.hip -- far-field passes of the 2D log kernel with the paper's fixed
// point-charge box vectors (Appendix STEP1-STEP3 in the square box; layout in
// points2d.h): n points per axis (the paper's 4 at (-2, -1, 1, 2) s / 5, or n
// = 2..8 Chebyshev points), d = n^2 per box, point i + n j.
//   P2M (STEP2): a charge q at w = (x - c) / s adds q f_i(5 w_x) f_j(5 w_y) to
//     point i + n j, f the Lagrange weights of the node set,
//       f_i(u) = c_i prod_{m != i} (u - a_m),  c_i = 1 / prod_{m != i} (a_i - a_m).
//   M2L (STEP3): the locals are the potentials at the box's points of the
//     point charges of its interaction list,
//       L_i = sum_o sum_j G_o[i][j] M_j(t + o),
//       G_o[i][j] = log s_k + log |(a_i - a_j) / 5 - o|,
//     on the matrix cores: one workgroup per 16 same-parity target boxes (a
//     4 x 4 block of stride 2), its four waves taking every fourth offset,
//     K = N = d padded to DP (a multiple of 16), DP / 4 16x16x4 steps per
//     16 outputs and offset; in FP32 each offset's product is added into FP64
//     sums, as in the 3D contraction.
//   L2P: the potential at x is sum f_i(5 w_x) f_j(5 w_y) L_{i+nj} over levels,
//     the field minus its gradient (d/dx = (5 / s) d/du), then the near field
//     is added and the outputs go to input order.
#include <cmath>
#include <vector>

#include "device_common.h"
#include "points2d.h"

namespace sffmm {

int points2d_row(int n) { return (n * n + 15) / 16 * 16; }

M2lLayout points2d_layout(int n, int L) {
  const int dp = points2d_row(n);
  M2lLayout ly{};
  ly.p = n;  // points per axis
  ly.nr = n * n;
  ly.kpad = dp;
  ly.npad = dp;
  ly.stride = dp * dp;
  ly.cs = dp;
  ly.lstride = dp * dp * (L + 1);
  return ly;
}

void build_points2d_operators(int node_set, int n, double* out) {
  double a[kPointsMaxN];
  if (!point_nodes(node_set, n, a)) return;
  for (int i = 0; i < n; ++i) a[i] /= 5.0;  // in units of the box side
  const int d = n * n, dp = points2d_row(n);
  for (int dy = -3; dy <= 3; ++dy)
    for (int dx = -3; dx <= 3; ++dx) {
      double* W = out + (size_t)((dx + 3) + 7 * (dy + 3)) * dp * dp;
      for (int e = 0; e < dp * dp; ++e) W[e] = 0.0;
      if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
      for (int t = 0; t < d; ++t)
        for (int s = 0; s < d; ++s) {
          const double rx = a[t % n] - a[s % n] - dx, ry = a[t / n] - a[s / n] - dy;
          W[t * dp + s] = 0.5 * std::log(rx * rx + ry * ry);
        }
    }
}

void build_points2d_lane_pack(int node_set, int n, const LevelTable& lt, double* out) {
  const int d = n * n, dp = points2d_row(n), ks = dp / 4, nbk = dp / 16;
  std::vector<double> G0((size_t)49 * dp * dp);
  build_points2d_operators(node_set, n, G0.data());
  for (int k = 0; k <= lt.L; ++k) {
    const double ls = std::log(lt.s[k]);
    for (int slot = 0; slot < 49; ++slot) {
      const int dx = slot % 7 - 3, dy = slot / 7 - 3;
      const bool adj = std::abs(dx) <= 1 && std::abs(dy) <= 1;
      double* P = out + ((size_t)k * 49 + slot) * dp * dp;
      for (int nb = 0; nb < nbk; ++nb)
        for (int s = 0; s < ks; ++s)
          for (int l = 0; l < 64; ++l) {
            const int i = 16 * nb + l % 16, j = (l / 16) * ks + s;  // output, source point
            P[(nb * ks + s) * 64 + l] =
                adj || i >= d || j >= d ? 0.0 : G0[((size_t)slot * dp + i) * dp + j] + ls;
          }
    }
  }
}

namespace {

typedef float p2fx4 __attribute__((ext_vector_type(4)));
typedef double p2dx4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma2p;
template <>
struct Mfma2p<float> {
  using acc_t = p2fx4;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma2p<double> {
  using acc_t = p2dx4;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Accumulator register r of lane group g holds output row (target) 4g + r in
// FP32 and g + 4r in FP64; its column is the lane's output point l % 16 of its
// block of 16.
template <typename T>
__device__ __forceinline__ int prow(int r, int g) {
  return sizeof(T) == 8 ? g + 4 * r : 4 * g + r;
}

// Offset of the particle from the centre of its level-k box, in units of s_k
// (FP32 modes: from the leaf-local record, exact leaf-to-box offsets).
template <typename T, bool LL>
__device__ __forceinline__ void box_w(const LevelTable& lt, int k, uint32_t lx, uint32_t ly,
                                      float xl, float yl, double x, double y, T& wx, T& wy) {
  const int sh = lt.L - k;
  if (LL) {
    const T sL = (T)lt.s[lt.L], is = (T)lt.inv_s[k];
    wx = ((T)xl + leaf_to_box<T>(lx, sh) * sL) * is;
    wy = ((T)yl + leaf_to_box<T>(ly, sh) * sL) * is;
  } else {
    const double cx = lt.origin[0] + lt.s[k] * ((double)(lx >> sh) + 0.5);
    const double cy = lt.origin[1] + lt.s[k] * ((double)(ly >> sh) + 0.5);
    wx = (T)((x - cx) * lt.inv_s[k]);
    wy = (T)((y - cy) * lt.inv_s[k]);
  }
}

// P2M (plan of device_common.h): G lanes per slice of a box accumulate the d
// point charges in registers, a butterfly adds the lanes, S > 1 slices leave
// partial rows for k_points2d_slices.  The row's padding (d .. DP - 1) is never
// written: it keeps the zeros the plan cleared it to.
template <typename T, int N, bool LL>
__global__ __launch_bounds__(256) void k_p2m2d_points(FmmArgs a, P2mPlan pl, PtsNodes nd) {
  constexpr int D = N * N;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if ((t & ~(int64_t)63) >= pl.thr_off[pl.khi + 1]) return;  // whole wave beyond the end
  const LevelTable& lt = a.lt;
  int k = pl.klo;
  while (k < pl.khi && t >= pl.thr_off[k + 1]) ++k;
  const int G = pl.G[k], S = pl.S[k];
  const int64_t local = t - pl.thr_off[k];
  const int64_t nb = (int64_t)1 << (2 * k);
  const int64_t b = local / (G * S);
  const bool valid = b < nb;
  const int rem = (int)(local - b * G * S);
  const int j = rem / G, r = rem - (rem / G) * G;
  const int sh = lt.L - k;
  T acc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = (T)0;
  if (valid) {
    const int64_t s0 = a.leaf_start[b << (2 * sh)], s1 = a.leaf_start[(b + 1) << (2 * sh)];
    const int64_t len = s1 - s0;
    const int64_t lo = s0 + len * j / S, hi = s0 + len * (j + 1) / S;
    const T is = (T)lt.inv_s[k], sL = (T)lt.s[lt.L];
    T cx = 0, cy = 0;
    if (!LL) {
      cx = (T)(lt.origin[0] + lt.s[k] * ((double)compact2((uint32_t)b) + 0.5));
      cy = (T)(lt.origin[1] + lt.s[k] * ((double)compact2((uint32_t)b >> 1) + 0.5));
    }
    for (int64_t i = lo + r; i < hi; i += G) {
      T q, wx, wy;
      if (LL) {
        const float4 pt = a.pts[i];
        const uint32_t lb = __float_as_uint(pt.w);  // the leaf's column | row << 16
        q = (T)pt.z;
        wx = ((T)pt.x + leaf_to_box<T>(lb & 0xFFFFu, sh) * sL) * is;
        wy = ((T)pt.y + leaf_to_box<T>(lb >> 16, sh) * sL) * is;
      } else {
        q = (T)a.qs[i];
        wx = ((T)a.xs[i] - cx) * is;
        wy = ((T)a.ys[i] - cy) * is;
      }
      T fx[N], fy[N];
      lagn<N>(nd, wx, fx);
      lagn<N>(nd, wy, fy);
#pragma unroll
      for (int jj = 0; jj < N; ++jj) {
        const T qj = q * fy[jj];
#pragma unroll
        for (int ii = 0; ii < N; ++ii) acc[ii + N * jj] += fx[ii] * qj;
      }
    }
  }
  for (int dd = 1; dd < G; dd <<= 1) {
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] += __shfl_xor(acc[i], dd, 64);
  }
  if (!valid || r != 0) return;
  const int cs = a.cs;
  T* out;
  if (S == 1)
    out = (sizeof(T) == 8 ? (T*)a.mom64 : (T*)a.mom32) + (lt.off[k] + b) * cs;
  else
    out = (sizeof(T) == 8 ? (T*)a.part64 : (T*)a.part32) + (pl.part_off[k] + b * S + j) * cs;
#pragma unroll
  for (int i = 0; i < D; ++i) out[i] = acc[i];
}

// Slice partials of level k added up: one wave per (box, point), lane l taking
// slices l, l + 64, ... in order, then a fixed butterfly across the wave.
template <typename T>
__global__ __launch_bounds__(256) void k_points2d_slices(FmmArgs a, P2mPlan pl, int k, int d) {
  const int64_t nb = (int64_t)1 << (2 * k);
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wv >= nb * d) return;  // whole waves
  const int64_t b = wv / d;
  const int c = (int)(wv - b * d);
  const int S = pl.S[k];
  const T* part = sizeof(T) == 8 ? (const T*)a.part64 : (const T*)a.part32;
  T* mom = sizeof(T) == 8 ? (T*)a.mom64 : (T*)a.mom32;
  const T* src = part + (pl.part_off[k] + b * S) * a.cs + c;
  T acc = 0;
  for (int j = lane; j < S; j += 64) acc += src[(int64_t)j * a.cs];
#pragma unroll
  for (int dd = 32; dd >= 1; dd >>= 1) acc += __shfl_xor(acc, dd, 64);
  if (lane == 0) mom[(a.lt.off[k] + b) * a.cs + c] = acc;
}

// M2L: workgroup t of level k takes tile t: parity class par = t / nblk^2 and
// block bl of that class; lane i (= lane % 16) of each wave holds target
// (tx0 + 2 (i & 3) + px, ty0 + 2 (i >> 2) + py) and lane group g = lane / 16
// the source points g KS .. g KS + KS - 1 of its row.  The 27 offsets of a
// parity class lie in the 6 x 6 window [xlo, xlo + 5] x [ylo, ylo + 5] (xlo =
// -2 - px: the children of the parent's neighbours) without the 9 adjacent
// ones; wave w takes the offsets w, w + 4, ... of that list (four chains of
// loads and matrix-core steps in flight per tile instead of one), and the four
// partial products are added in LDS in wave order (the same order on every run).
struct Pts2Tiles {
  int klo, khi;
  int64_t off[kMaxLevels2D + 2];  // first tile of level k
};
constexpr int kPts2Waves = 4;  // waves per tile

template <typename T, int DP>
__global__ __launch_bounds__(64 * kPts2Waves) void k_m2l2d_points(FmmArgs a, Pts2Tiles tt) {
  using acc_t = typename Mfma2p<T>::acc_t;
  constexpr bool kF64 = sizeof(T) == 8;
  constexpr int KS = DP / 4, NB = DP / 16;
  __shared__ double part[kPts2Waves - 1][NB][4][64];
  const int64_t tile = blockIdx.x;  // the grid holds exactly the tiles
  int k = tt.klo;
  while (k < tt.khi && tile >= tt.off[k + 1]) ++k;
  const int n = 1 << k, nblk = n >= 8 ? n / 8 : 1;
  const int64_t local = tile - tt.off[k];
  const int par = (int)(local / ((int64_t)nblk * nblk));
  const int bl = (int)(local - (int64_t)par * nblk * nblk);
  const int px = par & 1, py = par >> 1;
  const int tx0 = 8 * (bl % nblk), ty0 = 8 * (bl / nblk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 15, g = lane >> 4;
  const int tx = tx0 + 2 * (i & 3) + px, ty = ty0 + 2 * (i >> 2) + py;
  const bool tin = tx < n && ty < n;
  const int xlo = px ? -3 : -2, ylo = py ? -3 : -2;
  const int cs = a.cs;
  const T* mom = (kF64 ? (const T*)a.mom64 : (const T*)a.mom32) + a.lt.off[k] * cs;
  const T* ops = (kF64 ? (const T*)a.opl64 : (const T*)a.opl32) + (size_t)k * 49 * DP * DP;
  acc_t acc[NB];
  double sum[NB][4];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    acc[nb] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) sum[nb][r] = 0.0;
  }
  int e = 0;  // position in the offset list
  for (int oy = ylo; oy < ylo + 6; ++oy)
    for (int ox = xlo; ox < xlo + 6; ++ox) {
      if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1) continue;  // adjacent: the near field
      if (e++ % kPts2Waves != wave) continue;
      const int sx = tx + ox, sy = ty + oy;
      const bool ok = tin && sx >= 0 && sy >= 0 && sx < n && sy < n;
      T av[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) av[s] = (T)0;
      if (ok) {
        const T* A = mom + (int64_t)(spread2((uint32_t)sx) | (spread2((uint32_t)sy) << 1)) * cs +
                     KS * g;
#pragma unroll
        for (int s = 0; s < KS; ++s) av[s] = A[s];
      }
      const T* W = ops + (size_t)((ox + 3) + 7 * (oy + 3)) * DP * DP + lane;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int s = 0; s < KS; ++s)
          acc[nb] = Mfma2p<T>::op(av[s], W[(nb * KS + s) * 64], acc[nb]);
      if constexpr (!kF64) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) sum[nb][r] += (double)acc[nb][r];
          acc[nb] = acc_t{0, 0, 0, 0};
        }
      }
    }
  if constexpr (kF64) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) sum[nb][r] = acc[nb][r];
  }
  if (wave > 0) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[wave - 1][nb][r][lane] = sum[nb][r];
  }
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int w = 1; w < kPts2Waves; ++w)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) sum[nb][r] += part[w - 1][nb][r][lane];
  T* loc = (kF64 ? (T*)a.loc64 : (T*)a.loc32) + a.lt.off[k] * cs;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = prow<T>(r, g);
    const int gx = tx0 + 2 * (row & 3) + px, gy = ty0 + 2 * (row >> 2) + py;
    if (gx < n && gy < n) {
      T* dst = loc + (int64_t)(spread2((uint32_t)gx) | (spread2((uint32_t)gy) << 1)) * cs + i;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) dst[16 * nb] = (T)sum[nb][r];
    }
  }
}

// One level's potential and gradient (in units of 1 / s_k through u) at w.
template <int N, typename T>
__device__ __forceinline__ void eval_points2(const PtsNodes& nd, const T* B, T wx, T wy, T& F,
                                             T& Gx, T& Gy) {
  T fx[N], dfx[N], fy[N], dfy[N];
  lagnd<N>(nd, wx, fx, dfx);
  lagnd<N>(nd, wy, fy, dfy);
  F = Gx = Gy = (T)0;
#pragma unroll
  for (int jj = 0; jj < N; ++jj) {
    T g = 0, gd = 0;
#pragma unroll
    for (int ii = 0; ii < N; ++ii) {
      const T v = B[ii + N * jj];
      g += fx[ii] * v;
      gd += dfx[ii] * v;
    }
    F += fy[jj] * g;
    Gx += fy[jj] * gd;
    Gy += dfy[jj] * g;
  }
}

template <int N, bool LL>
__global__ __launch_bounds__(256) void k_l2p2d_points(FmmArgs a, PtsNodes nd) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const LevelTable& lt = a.lt;
  const int L = lt.L;
  const uint32_t key = a.keys[j];
  const uint32_t lx = compact2(local2(key, L)), ly = compact2(local2(key, L) >> 1);
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
  const int cs = a.cs;
  for (int k = lt.kmin; k <= L; ++k) {
    const uint32_t box = key >> (2 * (L - k));
    const double d5 = 5.0 * lt.inv_s[k];  // d/dx = (5 / s_k) d/du
    if (k < lt.split) {
      double wx, wy, F, Gx, Gy;
      box_w<double, LL>(lt, k, lx, ly, xl, yl, x, y, wx, wy);
      eval_points2<N, double>(nd, a.loc64 + (lt.off[k] + box) * cs, wx, wy, F, Gx, Gy);
      phi += F;
      ex -= Gx * d5;
      ey -= Gy * d5;
    } else {
      float wx, wy, F, Gx, Gy;
      box_w<float, LL>(lt, k, lx, ly, xl, yl, x, y, wx, wy);
      eval_points2<N, float>(nd, a.loc32 + (lt.off[k] + box) * cs, wx, wy, F, Gx, Gy);
      phi += (double)F;
      ex -= (double)(Gx * (float)d5);
      ey -= (double)(Gy * (float)d5);
    }
  }
  const int64_t o = a.perm[j];
  a.pot[o] = phi + a.near_pot[j];
  if (a.field) {
    a.field[2 * o] = ex + a.near_ex[j];
    a.field[2 * o + 1] = ey + a.near_ey[j];
  }
}

template <int N>
void p2m_points_n(const FmmArgs& a, bool ll, bool f64, hipStream_t st) {
  const PtsNodes nd = make_nodes(a.basis, N);
  const P2mPlan pl = make_p2m_plan(2, a.klo, a.khi, a.n);
  const int64_t thr = pl.thr_off[a.khi + 1];
  const dim3 grid((unsigned)((thr + 255) / 256));
  if (f64) {
    if (ll)
      hipLaunchKernelGGL((k_p2m2d_points<double, N, true>), grid, dim3(256), 0, st, a, pl, nd);
    else
      hipLaunchKernelGGL((k_p2m2d_points<double, N, false>), grid, dim3(256), 0, st, a, pl, nd);
  } else {
    hipLaunchKernelGGL((k_p2m2d_points<float, N, true>), grid, dim3(256), 0, st, a, pl, nd);
  }
  for (int k = a.klo; k <= a.khi; ++k)
    if (pl.S[k] > 1) {
      const int64_t waves = ((int64_t)1 << (2 * k)) * (N * N);
      const dim3 sg((unsigned)((waves * 64 + 255) / 256));
      if (f64)
        hipLaunchKernelGGL(k_points2d_slices<double>, sg, dim3(256), 0, st, a, pl, k, N * N);
      else
        hipLaunchKernelGGL(k_points2d_slices<float>, sg, dim3(256), 0, st, a, pl, k, N * N);
    }
}

template <int N>
void l2p_points_n(const FmmArgs& a, bool ll, hipStream_t st) {
  const PtsNodes nd = make_nodes(a.basis, N);
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (ll)
    hipLaunchKernelGGL((k_l2p2d_points<N, true>), grid, dim3(256), 0, st, a, nd);
  else
    hipLaunchKernelGGL((k_l2p2d_points<N, false>), grid, dim3(256), 0, st, a, nd);
}

template <int DP>
void m2l_points_dp(const FmmArgs& a, const Pts2Tiles& tt, bool fp64, hipStream_t st) {
  const dim3 grid((unsigned)tt.off[tt.khi + 1]), block(64 * kPts2Waves);
  if (fp64)
    hipLaunchKernelGGL((k_m2l2d_points<double, DP>), grid, block, 0, st, a, tt);
  else
    hipLaunchKernelGGL((k_m2l2d_points<float, DP>), grid, block, 0, st, a, tt);
}

}  // namespace

#define SFFMM_PTS2_N(fn, n, ...)           \
  do {                                     \
    switch (n) {                           \
      case 2: fn<2>(__VA_ARGS__); break;   \
      case 3: fn<3>(__VA_ARGS__); break;   \
      case 4: fn<4>(__VA_ARGS__); break;   \
      case 5: fn<5>(__VA_ARGS__); break;   \
      case 6: fn<6>(__VA_ARGS__); break;   \
      case 7: fn<7>(__VA_ARGS__); break;   \
      default: fn<8>(__VA_ARGS__); break;  \
    }                                      \
  } while (0)

void launch_p2m2d_points(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st) {
  if (a.khi < a.klo || a.n <= 0) return;
  SFFMM_PTS2_N(p2m_points_n, a.p, a, leaf_local, fp64, st);
}

void launch_m2l2d_points(const FmmArgs& a, bool fp64, hipStream_t st) {
  if (a.khi < a.klo) return;
  Pts2Tiles tt{};
  tt.klo = a.klo;
  tt.khi = a.khi;
  int64_t t = 0;
  for (int k = a.klo; k <= a.khi; ++k) {
    tt.off[k] = t;
    const int64_t n = (int64_t)1 << k, nblk = n >= 8 ? n / 8 : 1;
    t += 4 * nblk * nblk;
  }
  tt.off[a.khi + 1] = t;
  switch (points2d_row(a.p)) {
    case 16: m2l_points_dp<16>(a, tt, fp64, st); break;
    case 32: m2l_points_dp<32>(a, tt, fp64, st); break;
    case 48: m2l_points_dp<48>(a, tt, fp64, st); break;
    default: m2l_points_dp<64>(a, tt, fp64, st); break;
  }
}

void launch_l2p2d_points(const FmmArgs& a, bool leaf_local, hipStream_t st) {
  if (a.n <= 0) return;
  SFFMM_PTS2_N(l2p_points_n, a.p, a, leaf_local, st);
}

}  // namespace sffmm
