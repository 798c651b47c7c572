// points2d.hip -- far-field passes of the 2D log kernel with the paper's fixed
// point-charge box vectors (Appendix STEP1-STEP3 in the square box; layout in
// points2d.h).
//   P2M (STEP2): a charge q at w = (x - c) / s adds q f_i(5 w_x) f_j(5 w_y) to
//     point i + 4 j, f the cubic Lagrange weights of the node set (lag4).
//   M2L (STEP3): the locals are the potentials at the box's points of the
//     point charges of its interaction list,
//       L_i = sum_o sum_j G_o[i][j] M_j(t + o),
//       G_o[i][j] = log s_k + log |(a_i - a_j) / 5 - o|,
//     on the matrix cores: one workgroup per 16 same-parity target boxes (a
//     4 x 4 block of stride 2), its four waves taking every fourth offset,
//     K = 16 source points, N = 16 output points, four 16x16x4 steps per
//     offset; in FP32 each offset's product is added into FP64 sums, as in
//     the 3D contraction.
//   L2P: the potential at x is sum f_i(5 w_x) f_j(5 w_y) L_{i+4j} over levels,
//     the field minus its gradient (d/dx = (5 / s) d/du), then the near field
//     is added and the outputs go to input order.
#include <cmath>
#include <vector>

#include "device_common.h"
#include "points2d.h"

namespace sffmm {

M2lLayout points2d_layout(int L) {
  M2lLayout ly{};
  ly.p = 4;  // points per axis
  ly.nr = kPoints2D;
  ly.kpad = kPoints2D;
  ly.npad = kPoints2D;
  ly.stride = kPoints2D * kPoints2D;
  ly.cs = kPoints2D;
  ly.lstride = kPoints2D * kPoints2D * (L + 1);
  return ly;
}

void build_points2d_operators(int node_set, double* out) {
  double a[4];  // node offsets in units of the box side
  for (int i = 0; i < 4; ++i) a[i] = point_node(node_set, i) / 5.0;
  for (int dy = -3; dy <= 3; ++dy)
    for (int dx = -3; dx <= 3; ++dx) {
      double* W = out + (size_t)((dx + 3) + 7 * (dy + 3)) * 256;
      for (int e = 0; e < 256; ++e) W[e] = 0.0;
      if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
      for (int t = 0; t < 16; ++t)
        for (int s = 0; s < 16; ++s) {
          const double rx = a[t & 3] - a[s & 3] - dx, ry = a[t >> 2] - a[s >> 2] - dy;
          W[t * 16 + s] = 0.5 * std::log(rx * rx + ry * ry);
        }
    }
}

void build_points2d_lane_pack(int node_set, const LevelTable& lt, double* out) {
  std::vector<double> G0((size_t)49 * 256);
  build_points2d_operators(node_set, G0.data());
  for (int k = 0; k <= lt.L; ++k) {
    const double ls = std::log(lt.s[k]);
    for (int slot = 0; slot < 49; ++slot) {
      const int dx = slot % 7 - 3, dy = slot / 7 - 3;
      const bool adj = std::abs(dx) <= 1 && std::abs(dy) <= 1;
      double* P = out + ((size_t)k * 49 + slot) * 256;
      for (int s = 0; s < 4; ++s)
        for (int l = 0; l < 64; ++l) {
          const int i = l % 16, j = 4 * (l / 16) + s;
          P[64 * s + l] = adj ? 0.0 : G0[(size_t)slot * 256 + i * 16 + j] + ls;
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
// FP32 and g + 4r in FP64; its column is the lane's output point l % 16.
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

// P2M (plan of device_common.h): G lanes per slice of a box accumulate the 16
// point charges in registers, a butterfly adds the lanes, S > 1 slices leave
// partial rows for k_points2d_slices.
template <typename T, int NS, bool LL>
__global__ __launch_bounds__(256) void k_p2m2d_points(FmmArgs a, P2mPlan pl) {
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
  T acc[kPoints2D];
#pragma unroll
  for (int i = 0; i < kPoints2D; ++i) acc[i] = (T)0;
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
      T fx[4], fy[4];
      lag4<NS>(wx, fx);
      lag4<NS>(wy, fy);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const T qj = q * fy[jj];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) acc[ii + 4 * jj] += fx[ii] * qj;
      }
    }
  }
  for (int d = 1; d < G; d <<= 1) {
#pragma unroll
    for (int i = 0; i < kPoints2D; ++i) acc[i] += __shfl_xor(acc[i], d, 64);
  }
  if (!valid || r != 0) return;
  const int cs = a.cs;
  T* out;
  if (S == 1)
    out = (sizeof(T) == 8 ? (T*)a.mom64 : (T*)a.mom32) + (lt.off[k] + b) * cs;
  else
    out = (sizeof(T) == 8 ? (T*)a.part64 : (T*)a.part32) + (pl.part_off[k] + b * S + j) * cs;
#pragma unroll
  for (int i = 0; i < kPoints2D; ++i) out[i] = acc[i];
}

// Slice partials of level k added up: one wave per (box, point), lane l taking
// slices l, l + 64, ... in order, then a fixed butterfly across the wave.
template <typename T>
__global__ __launch_bounds__(256) void k_points2d_slices(FmmArgs a, P2mPlan pl, int k) {
  const int64_t nb = (int64_t)1 << (2 * k);
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wv >= nb * kPoints2D) return;  // whole waves
  const int64_t b = wv / kPoints2D;
  const int c = (int)(wv - b * kPoints2D);
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

// M2L: workgroup t of level k takes tile t: parity class par = t / nblk^2 and
// block bl of that class; lane i (= lane % 16) of each wave holds target
// (tx0 + 2 (i & 3) + px, ty0 + 2 (i >> 2) + py).  The 27 offsets of a parity
// class lie in the 6 x 6 window [xlo, xlo + 5] x [ylo, ylo + 5] (xlo = -2 - px:
// the children of the parent's neighbours) without the 9 adjacent ones; wave w
// takes the offsets w, w + 4, ... of that list (four chains of loads and
// matrix-core steps in flight per tile instead of one), and the four partial
// products are added in LDS in wave order (the same order on every run).
struct Pts2Tiles {
  int klo, khi;
  int64_t off[kMaxLevels2D + 2];  // first tile of level k
};
constexpr int kPts2Waves = 4;  // waves per tile

template <typename T>
__global__ __launch_bounds__(64 * kPts2Waves) void k_m2l2d_points(FmmArgs a, Pts2Tiles tt) {
  using acc_t = typename Mfma2p<T>::acc_t;
  constexpr bool kF64 = sizeof(T) == 8;
  __shared__ double part[kPts2Waves - 1][4][64];
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
  const T* ops = (kF64 ? (const T*)a.opl64 : (const T*)a.opl32) + (size_t)k * 49 * 256;
  acc_t acc = {0, 0, 0, 0};
  double sum[4] = {0.0, 0.0, 0.0, 0.0};
  int e = 0;  // position in the offset list
  for (int oy = ylo; oy < ylo + 6; ++oy)
    for (int ox = xlo; ox < xlo + 6; ++ox) {
      if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1) continue;  // adjacent: the near field
      if (e++ % kPts2Waves != wave) continue;
      const int sx = tx + ox, sy = ty + oy;
      const bool ok = tin && sx >= 0 && sy >= 0 && sx < n && sy < n;
      T av[4] = {(T)0, (T)0, (T)0, (T)0};
      if (ok) {
        const T* A = mom + (int64_t)(spread2((uint32_t)sx) | (spread2((uint32_t)sy) << 1)) * cs +
                     4 * g;
#pragma unroll
        for (int s = 0; s < 4; ++s) av[s] = A[s];
      }
      const T* W = ops + (size_t)((ox + 3) + 7 * (oy + 3)) * 256 + lane;
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = Mfma2p<T>::op(av[s], W[64 * s], acc);
      if constexpr (!kF64) {
#pragma unroll
        for (int r = 0; r < 4; ++r) sum[r] += (double)acc[r];
        acc = acc_t{0, 0, 0, 0};
      }
    }
  if constexpr (kF64) {
#pragma unroll
    for (int r = 0; r < 4; ++r) sum[r] = acc[r];
  }
  if (wave > 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wave - 1][r][lane] = sum[r];
  }
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int w = 1; w < kPts2Waves; ++w)
#pragma unroll
    for (int r = 0; r < 4; ++r) sum[r] += part[w - 1][r][lane];
  T* loc = (kF64 ? (T*)a.loc64 : (T*)a.loc32) + a.lt.off[k] * cs;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = prow<T>(r, g);
    const int gx = tx0 + 2 * (row & 3) + px, gy = ty0 + 2 * (row >> 2) + py;
    if (gx < n && gy < n)
      loc[(int64_t)(spread2((uint32_t)gx) | (spread2((uint32_t)gy) << 1)) * cs + i] = (T)sum[r];
  }
}

// One level's potential and gradient (in units of 1 / s_k through u) at w.
template <int NS, typename T>
__device__ __forceinline__ void eval_points2(const T* B, T wx, T wy, T& F, T& Gx, T& Gy) {
  T fx[4], dfx[4], fy[4], dfy[4];
  lag4d<NS>(wx, fx, dfx);
  lag4d<NS>(wy, fy, dfy);
  F = Gx = Gy = (T)0;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    T g = 0, gd = 0;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const T v = B[ii + 4 * jj];
      g += fx[ii] * v;
      gd += dfx[ii] * v;
    }
    F += fy[jj] * g;
    Gx += fy[jj] * gd;
    Gy += dfy[jj] * g;
  }
}

template <int NS, bool LL>
__global__ __launch_bounds__(256) void k_l2p2d_points(FmmArgs a) {
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
      eval_points2<NS, double>(a.loc64 + (lt.off[k] + box) * cs, wx, wy, F, Gx, Gy);
      phi += F;
      ex -= Gx * d5;
      ey -= Gy * d5;
    } else {
      float wx, wy, F, Gx, Gy;
      box_w<float, LL>(lt, k, lx, ly, xl, yl, x, y, wx, wy);
      eval_points2<NS, float>(a.loc32 + (lt.off[k] + box) * cs, wx, wy, F, Gx, Gy);
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

template <int NS>
void p2m_points_ns(const FmmArgs& a, bool ll, bool f64, hipStream_t st) {
  const P2mPlan pl = make_p2m_plan(2, a.klo, a.khi, a.n);
  const int64_t thr = pl.thr_off[a.khi + 1];
  const dim3 grid((unsigned)((thr + 255) / 256));
  if (f64) {
    if (ll)
      hipLaunchKernelGGL((k_p2m2d_points<double, NS, true>), grid, dim3(256), 0, st, a, pl);
    else
      hipLaunchKernelGGL((k_p2m2d_points<double, NS, false>), grid, dim3(256), 0, st, a, pl);
  } else {
    hipLaunchKernelGGL((k_p2m2d_points<float, NS, true>), grid, dim3(256), 0, st, a, pl);
  }
  for (int k = a.klo; k <= a.khi; ++k)
    if (pl.S[k] > 1) {
      const int64_t waves = ((int64_t)1 << (2 * k)) * kPoints2D;
      const dim3 sg((unsigned)((waves * 64 + 255) / 256));
      if (f64)
        hipLaunchKernelGGL(k_points2d_slices<double>, sg, dim3(256), 0, st, a, pl, k);
      else
        hipLaunchKernelGGL(k_points2d_slices<float>, sg, dim3(256), 0, st, a, pl, k);
    }
}

template <int NS>
void l2p_points_ns(const FmmArgs& a, bool ll, hipStream_t st) {
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (ll)
    hipLaunchKernelGGL((k_l2p2d_points<NS, true>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_l2p2d_points<NS, false>), grid, dim3(256), 0, st, a);
}

}  // namespace

void launch_p2m2d_points(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st) {
  if (a.khi < a.klo || a.n <= 0) return;
  if (a.basis == 2)
    p2m_points_ns<2>(a, leaf_local, fp64, st);
  else
    p2m_points_ns<1>(a, leaf_local, fp64, st);
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
  const dim3 grid((unsigned)t), block(64 * kPts2Waves);
  if (fp64)
    hipLaunchKernelGGL(k_m2l2d_points<double>, grid, block, 0, st, a, tt);
  else
    hipLaunchKernelGGL(k_m2l2d_points<float>, grid, block, 0, st, a, tt);
}

void launch_l2p2d_points(const FmmArgs& a, bool leaf_local, hipStream_t st) {
  if (a.n <= 0) return;
  if (a.basis == 2)
    l2p_points_ns<2>(a, leaf_local, st);
  else
    l2p_points_ns<1>(a, leaf_local, st);
}

}  // namespace sffmm
