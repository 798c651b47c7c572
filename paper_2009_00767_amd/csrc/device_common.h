// device_common.h -- Morton-code helpers, leaf-centre offsets, the P2M work
// plan and the point-charge (Lagrange) weights shared by the 2D and 3D kernels.
#pragma once

#include "fmm_internal.h"

namespace sffmm {

__device__ __forceinline__ uint32_t compact2(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0F0F0F0Fu;
  v = (v | (v >> 4)) & 0x00FF00FFu;
  v = (v | (v >> 8)) & 0x0000FFFFu;
  return v;
}

__device__ __forceinline__ uint32_t spread2(uint32_t v) {
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x000003FFu;
  return v;
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Offset of a leaf centre from the centre of its level-k ancestor, along one
// axis, in units of s_L: (r + 1/2) - 2^(L-k) / 2 with r the leaf index inside
// the ancestor.  Exact in FP32 and FP64.
template <typename T>
__device__ __forceinline__ T leaf_to_box(uint32_t leaf, int sh) {
  const uint32_t r = leaf & ((1u << sh) - 1u);
  return (T)r + (T)0.5 - (T)(1u << sh) * (T)0.5;
}

// P2M work plan: per level, G lanes per box (a power of two <= 64 giving each
// lane about 16 particles) and S waves (slices) per box when it holds far more
// than a wave's share.  Level thread ranges start on wave boundaries.
struct P2mPlan {
  int klo, khi;
  int32_t G[kMaxLevels2D + 1];
  int32_t S[kMaxLevels2D + 1];
  int64_t thr_off[kMaxLevels2D + 2];
  int64_t part_off[kMaxLevels2D + 1];
};

inline P2mPlan make_p2m_plan(int dim, int klo, int khi, int64_t n, int nsys = 1) {
  P2mPlan pl{};
  pl.klo = klo;
  pl.khi = khi;
  int64_t t = 0, po = 0;
  for (int k = klo; k <= khi; ++k) {
    const int64_t nb = (int64_t)nsys << (dim * k);
    const int64_t avg = n / nb;
    int64_t G = 1, S = 1;
    if (avg > 24) {
      while (G < 64 && G * 16 < avg) G *= 2;
      if (avg > 2048)
        while (S < 1024 && S * 1024 < avg) S *= 2;
    }
    pl.G[k] = (int32_t)G;
    pl.S[k] = (int32_t)S;
    pl.thr_off[k] = t;
    pl.part_off[k] = po;
    t += (nb * G * S + 63) / 64 * 64;
    if (S > 1) po += nb * S;
  }
  pl.thr_off[khi + 1] = t;
  return pl;
}

inline size_t p2m_partial_rows(int dim, int klo, int khi, int64_t maxn, int nsys = 1) {
  if (khi < klo) return 0;
  const P2mPlan pl = make_p2m_plan(dim, klo, khi, maxn, nsys);
  int64_t rows = 0;
  for (int k = klo; k <= khi; ++k)
    if (pl.S[k] > 1) rows += ((int64_t)nsys << (dim * k)) * pl.S[k];
  return (size_t)rows;
}

// Low 2k bits of a stacked 2D key / box index: the Morton code inside its system.
__device__ __forceinline__ uint32_t local2(uint32_t v, int k) {
  return v & ((k >= 16) ? 0xFFFFFFFFu : ((1u << (2 * k)) - 1u));
}

// Deals blocks round-robin over the 8 XCDs the way the hardware dispatches them
// and maps them back so that each XCD owns one contiguous range of work items.
// Adaptive depth: particles in the 3 x 3 level-k boxes around box (bx, by) of
// a one-system 2D tree of depth L (leaf_start: the level-L leaf offsets; a
// level-k box spans the leaf keys [b << 2 (L - k), (b + 1) << 2 (L - k))).
__device__ __forceinline__ int64_t around_count2(const int32_t* leaf_start, int L, int k, int bx,
                                                 int by) {
  const int nb = 1 << k, sh = 2 * (L - k);
  int64_t c = 0;
  for (int y = by - 1; y <= by + 1; ++y) {
    if (y < 0 || y >= nb) continue;
    for (int x = bx - 1; x <= bx + 1; ++x) {
      if (x < 0 || x >= nb) continue;
      const int64_t b = (int64_t)(spread2((uint32_t)x) | (spread2((uint32_t)y) << 1));
      c += leaf_start[(b + 1) << sh] - leaf_start[b << sh];
    }
  }
  return c;
}

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t q8 = nblocks / 8, r8 = nblocks % 8;
  const int64_t xcd = bid % 8, idx = bid / 8;
  return xcd * q8 + (xcd < r8 ? xcd : r8) + idx;
}

// Fixed point-charge basis (Appendix STEP1-STEP2): 4 points per axis at
// a_n s / 5 from the box centre (node set NS: the paper's a = (-2, -1, 1, 2),
// or Chebyshev points), point i + 4 j + 16 l.  A charge at w = (r - r_b) / s
// becomes the 64 charges q f_i(5 w_x) f_j(5 w_y) f_l(5 w_z), f the cubic
// Lagrange basis of those nodes; with d_n = u - a_n and c_n the inverse
// denominators:
//   f = (d_1 d_2 d_3 c_0, d_0 d_2 d_3 c_1, d_0 d_1 d_3 c_2, d_0 d_1 d_2 c_3).
template <int NS, typename T>
__device__ __forceinline__ void lag4(T w, T (&f)[4]) {
  constexpr T a0 = (T)point_node(NS, 0), a1 = (T)point_node(NS, 1), a2 = (T)point_node(NS, 2),
              a3 = (T)point_node(NS, 3);
  constexpr T c0 = (T)point_node_inv_den(NS, 0), c1 = (T)point_node_inv_den(NS, 1),
              c2 = (T)point_node_inv_den(NS, 2), c3 = (T)point_node_inv_den(NS, 3);
  const T u = (T)5 * w;
  const T d0 = u - a0, d1 = u - a1, d2 = u - a2, d3 = u - a3;
  const T d23 = d2 * d3, d01 = d0 * d1;
  f[0] = d1 * d23 * c0;
  f[1] = d0 * d23 * c1;
  f[2] = d01 * d3 * c2;
  f[3] = d01 * d2 * c3;
}

// the weights and their derivatives in u
template <int NS, typename T>
__device__ __forceinline__ void lag4d(T w, T (&f)[4], T (&df)[4]) {
  constexpr T a0 = (T)point_node(NS, 0), a1 = (T)point_node(NS, 1), a2 = (T)point_node(NS, 2),
              a3 = (T)point_node(NS, 3);
  constexpr T c0 = (T)point_node_inv_den(NS, 0), c1 = (T)point_node_inv_den(NS, 1),
              c2 = (T)point_node_inv_den(NS, 2), c3 = (T)point_node_inv_den(NS, 3);
  const T u = (T)5 * w;
  const T d0 = u - a0, d1 = u - a1, d2 = u - a2, d3 = u - a3;
  const T d23 = d2 * d3, d01 = d0 * d1, d13 = d1 * d3, d12 = d1 * d2, d03 = d0 * d3,
          d02 = d0 * d2;
  f[0] = d1 * d23 * c0;
  f[1] = d0 * d23 * c1;
  f[2] = d01 * d3 * c2;
  f[3] = d01 * d2 * c3;
  df[0] = (d23 + d13 + d12) * c0;
  df[1] = (d23 + d03 + d02) * c1;
  df[2] = (d13 + d03 + d01) * c2;
  df[3] = (d12 + d02 + d01) * c3;
}

// acc[i + 4 j + 16 l] += q f_i(x) f_j(y) f_l(z)
template <int NS, typename T>
__device__ __forceinline__ void points_accumulate(T (&acc)[64], T q, T wx, T wy, T wz) {
  T fx[4], fy[4], fz[4];
  lag4<NS>(wx, fx);
  lag4<NS>(wy, fy);
  lag4<NS>(wz, fz);
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const T ql = q * fz[l];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T qjl = ql * fy[j];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i + 4 * j + 16 * l] += fx[i] * qjl;
    }
  }
}

}  // namespace sffmm
