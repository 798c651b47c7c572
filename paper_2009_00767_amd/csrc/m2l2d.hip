// m2l2d.hip -- the interaction-list contraction (D-bar-1 of Section 2.2.1) for
// the 2D log kernel on the matrix cores.
//
// For a target box t at level k the local coefficients are
//   B(t) = sum_{o in IL(t)} T_o A(t + o),
// with T_o the level-independent operator of offset o (built once, in FP64,
// see operators.cpp).  The 27 offsets of an interior box depend only on the
// parities of its indices, so the 16 same-parity targets of an 8 x 8 tile share
// one operator per offset: their 16 x 2p outputs form a dense product
//   C[16 x N] += A_o[16 x K] . W_o[K x N]
// per offset, which runs as v_mfma 16x16x4 instructions (FP32 or FP64).
//
// Workgroup = one 8 x 8 tile of target boxes at one level (all levels in one
// launch); the 14 x 14 source halo of box vectors is staged in LDS; wave w
// handles the targets with index parities (w & 1, w >> 1).  Blocks are mapped
// to tiles so that each XCD (blocks are dealt round-robin to the 8 XCDs) works
// on one contiguous Morton range of tiles and so reuses its L2.
//
// The K dimension is permuted so that lane group g = lane / 16 supplies the
// consecutive input values g*KS .. g*KS + KS - 1 of its row: every MFMA step s
// contracts the four values {g*KS + s}.  The real-only coefficient A_0 and the
// Re B_0 output are handled by VALU fused multiply-adds beside the MFMAs.
#include "device_common.h"

namespace sffmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename T>
struct Mfma16;
template <>
struct Mfma16<float> {
  using acc_t = floatx4;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma16<double> {
  using acc_t = doublex4;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

struct M2lTiles {
  int klo, khi;
  int64_t off[kMaxLevels2D + 2];  // first tile of level k
  int64_t ntiles;
};

constexpr int kHalo = 14;  // 8 targets + 3 on each side

// Output row held in accumulator register r by lane group g: 4g + r for the
// FP32 16x16x4 MFMA, g + 4r for the FP64 one (checked on gfx950).  Row i is the
// target (2 (i & 3) + px, 2 (i >> 2) + py) of the wave's parity class.
template <typename T>
__device__ __forceinline__ int crow_x(int r, int g) {
  return sizeof(T) == 8 ? 2 * g : 2 * r;
}
template <typename T>
__device__ __forceinline__ int crow_y(int r, int g) {
  return sizeof(T) == 8 ? 2 * r : 2 * g;
}

// BF = true (T = float): the dense block of coefficients 1..p runs as
// v_mfma_f32_16x16x32_bf16 on BF16-rounded inputs and operators (K padded to a
// multiple of 32, lane group g supplying KB consecutive values); the A_0 and
// Re B_0 terms stay in FP32.
template <typename T, int KS, int NB, bool BF>
__global__ __launch_bounds__(256) void k_m2l2d_mfma(FmmArgs a, M2lTiles tt, M2lLayout ly) {
  constexpr int KB = BF ? (KS + 7) / 8 * 8 : KS;  // values per lane group
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* halo = reinterpret_cast<T*>(smem_raw);
  using acc_t = typename Mfma16<T>::acc_t;
  constexpr bool kF64 = sizeof(T) == 8;

  const int64_t tile = xcd_remap(blockIdx.x, tt.ntiles);
  int k = tt.klo;
  while (k < tt.khi && tile >= tt.off[k + 1]) ++k;
  const int n = 1 << k;
  const int64_t tper = k >= 3 ? ((int64_t)1 << (2 * (k - 3))) : 1;  // tiles per system
  const int64_t tg = tile - tt.off[k];
  const uint32_t sys = (uint32_t)(tg / tper), tl = (uint32_t)(tg - (int64_t)sys * tper);
  const uint32_t sysb = sys << (2 * k);  // system bits of this level's box indices
  const int tx0 = 8 * (int)compact2(tl), ty0 = 8 * (int)compact2(tl >> 1);
  const int cs = ly.cs, pb = ly.p;  // layout order (the order bucket)
  const T* mom = (kF64 ? (const T*)a.mom64 : (const T*)a.mom32) + a.lt.off[k] * cs;
  T* loc = (kF64 ? (T*)a.loc64 : (T*)a.loc32) + a.lt.off[k] * cs;
  const T* ops = kF64 ? (const T*)a.op64 : (const T*)a.op32;

  // Stage the source halo (zeros outside the grid).
  for (int e = threadIdx.x; e < kHalo * kHalo * cs; e += 256) {
    const int hb = e / cs, c = e - hb * cs;
    const int sx = tx0 - 3 + hb % kHalo, sy = ty0 - 3 + hb / kHalo;
    T v = (T)0;
    if (sx >= 0 && sy >= 0 && sx < n && sy < n)
      v = mom[(int64_t)(sysb | spread2(sx) | (spread2(sy) << 1)) * cs + c];
    halo[e] = v;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int px = w & 1, py = w >> 1;
  const int i = lane & 15, g = lane >> 4;
  const int ix = 2 * (i & 3) + px, iy = 2 * (i >> 2) + py;  // A-row target of this lane
  acc_t acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = acc_t{0, 0, 0, 0};
  T b0p = 0, a0s = 0;
  const int xlo = px ? -3 : -2, ylo = py ? -3 : -2;
  const int kpad = ly.kpad, npad = ly.npad;
  // This level's order pk <= pb: the moments above pk are zero and the locals
  // above pk are never read, so only the K values below 2 pk (ksr per lane
  // group, consecutive) and the output blocks below 2 pk (nbr) are formed.
  const int pk = a.ord[k];
  const int ksr = BF ? (pk + 15) / 16 * 8 : (pk + 1) / 2;
  const int nbr = (pk + 7) / 8;

  for (int dy = ylo; dy <= ylo + 5; ++dy) {
    for (int dx = xlo; dx <= xlo + 5; ++dx) {
      if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
      const T* W = ops + (size_t)((dx + 3) + 7 * (dy + 3)) * ly.stride;
      const T* row = halo + ((iy + dy + 3) * kHalo + (ix + dx + 3)) * cs;
      // K values g * ksr + s, s < ksr, of this lane group (all below 2 pb + 2
      // and zero from 2 pk on)
      T av[KB];
#pragma unroll
      for (int s = 0; s < KB; ++s)
        av[s] = (s < ksr && g * ksr + s < 2 * pb) ? row[g * ksr + s] : (T)0;
      if constexpr (BF) {
        const __bf16* Wh = a.op16 + (size_t)((dx + 3) + 7 * (dy + 3)) * ly.npad * ly.kbf;
#pragma unroll
        for (int c = 0; c < KB / 8; ++c) {
          if (8 * c < ksr) {
            bf16x8 ab;
#pragma unroll
            for (int e = 0; e < 8; ++e) ab[e] = (__bf16)av[8 * c + e];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              if (nb < nbr) {
                const bf16x8 bb = *reinterpret_cast<const bf16x8*>(Wh + (16 * nb + i) * ly.kbf +
                                                                   g * ksr + 8 * c);
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, acc[nb], 0, 0, 0);
              }
            }
          }
        }
      } else {
        T bv[NB][KS];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int s = 0; s < KS; ++s)
            bv[nb][s] = (nb < nbr && s < ksr) ? W[(16 * nb + i) * kpad + g * ksr + s] : (T)0;
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            if (nb < nbr && s < ksr) acc[nb] = Mfma16<T>::op(av[s], bv[nb][s], acc[nb]);
      }
      // Re B_0 from the coefficients m >= 1 (this lane's share of the K range)
      const T* c0 = W + npad * kpad;
      const T* r0 = c0 + npad;
#pragma unroll
      for (int s = 0; s < KB; ++s)
        if (s < ksr && g * ksr + s < 2 * pb) b0p += r0[g * ksr + s] * av[s];
      if (g == 0) {
        const T a0 = row[2 * pb];
        b0p += r0[kpad] * a0;  // Re log(-u)
        a0s += a0;
      }
      // outputs l >= 1 from A_0 for the four C rows this lane holds
      T c0v[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) c0v[nb] = nb < nbr ? c0[16 * nb + i] : (T)0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int cx = crow_x<T>(r, g) + px, cy = crow_y<T>(r, g) + py;
        const T a0r = halo[((cy + dy + 3) * kHalo + (cx + dx + 3)) * cs + 2 * pb];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          if (nb < nbr) acc[nb][r] += c0v[nb] * a0r;
      }
    }
  }
  b0p += __shfl_xor(b0p, 16, 64);
  b0p += __shfl_xor(b0p, 32, 64);
  a0s += __shfl_xor(a0s, 16, 64);
  a0s += __shfl_xor(a0s, 32, 64);
  const T b0 = b0p + (T)a.lt.log_s[k] * a0s;

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gx = tx0 + crow_x<T>(r, g) + px, gy = ty0 + crow_y<T>(r, g) + py;
    if (gx < n && gy < n) {
      T* dst = loc + (int64_t)(sysb | spread2(gx) | (spread2(gy) << 1)) * cs;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int j = 16 * nb + i;
        if (j < 2 * pb) dst[j] = acc[nb][r];
      }
    }
  }
  if (g == 0) {
    const int gx = tx0 + ix, gy = ty0 + iy;
    if (gx < n && gy < n) {
      T* dst = loc + (int64_t)(sysb | spread2(gx) | (spread2(gy) << 1)) * cs;
      dst[2 * pb] = b0;
      dst[2 * pb + 1] = (T)0;  // Im B_0 enters neither the potential nor the field
    }
  }
}

template <typename T, int KS, int NB, bool BF>
static void m2l_launch(const FmmArgs& a, const M2lTiles& tt, const M2lLayout& ly,
                       hipStream_t st) {
  const size_t lds = (size_t)kHalo * kHalo * ly.cs * sizeof(T);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_m2l2d_mfma<T, KS, NB, BF>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_m2l2d_mfma<T, KS, NB, BF>), dim3(tt.ntiles), dim3(256), lds, st, a, tt,
                     ly);
}

template <typename T, bool BF>
static void m2l_dispatch_t(const FmmArgs& a, const M2lTiles& tt, const M2lLayout& ly,
                           hipStream_t st) {
  switch (ly.kpad) {  // kpad = 2 PB, PB the order bucket
    case 16: m2l_launch<T, 4, 1, BF>(a, tt, ly, st); break;
    case 24: m2l_launch<T, 6, 2, BF>(a, tt, ly, st); break;
    case 32: m2l_launch<T, 8, 2, BF>(a, tt, ly, st); break;
    case 40: m2l_launch<T, 10, 3, BF>(a, tt, ly, st); break;
    case 48: m2l_launch<T, 12, 3, BF>(a, tt, ly, st); break;
    default: m2l_launch<T, 15, 4, BF>(a, tt, ly, st); break;
  }
}

void launch_m2l2d(const FmmArgs& a, bool fp64, hipStream_t st, bool bf16) {
  if (a.khi < a.klo) return;
  M2lTiles tt{};
  tt.klo = a.klo;
  tt.khi = a.khi;
  int64_t t = 0;
  for (int k = a.klo; k <= a.khi; ++k) {
    tt.off[k] = t;
    const int64_t side = k >= 3 ? ((int64_t)1 << (k - 3)) : 1;
    t += side * side * a.lt.nsys;
  }
  tt.off[a.khi + 1] = t;
  tt.ntiles = t;
  const M2lLayout ly = m2l2d_layout(order_bucket(a.p));
  if (fp64)
    m2l_dispatch_t<double, false>(a, tt, ly, st);
  else if (bf16)
    m2l_dispatch_t<float, true>(a, tt, ly, st);
  else
    m2l_dispatch_t<float, false>(a, tt, ly, st);
}

}  // namespace sffmm
