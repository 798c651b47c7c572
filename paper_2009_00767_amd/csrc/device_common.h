// device_common.h -- Morton-code helpers, leaf-centre offsets and the P2M work
// plan shared by the 2D and 3D kernels.
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
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t q8 = nblocks / 8, r8 = nblocks % 8;
  const int64_t xcd = bid % 8, idx = bid / 8;
  return xcd * q8 + (xcd < r8 ? xcd : r8) + idx;
}

}  // namespace sffmm
