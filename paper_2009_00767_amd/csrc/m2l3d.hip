// m2l3d.hip -- the interaction-list contraction (D-bar-1 of Section 2.2.1) for
// the 3D 1/r kernel on the matrix cores.
//
// L(t) = sum_{o in IL(t)} T_o M(t + o) with T_o the real (p+1)^2 x (p+1)^2
// operator of offset o (operators.cpp), or the 64 x 64 point-charge block of
// the fixed point-charge basis (Appendix STEP3; its degree-0 slot stays zero).  The 189 offsets of an interior box
// depend only on the parities of its indices, so one workgroup takes one parity
// class and a block of 4 x 4 x (NW MB) same-parity targets (an 8 x 8 x 2 NW MB
// box region) with NW waves: wave w owns the 16 targets of each of the
// z-layers w, w + NW, ... and, per offset, runs the dense products
// C[16 x N] += A_o[16 x K] . W_o[K x N] as v_mfma 16x16x4 instructions, each
// operator value read from LDS serving MB of them.  The operators stream from
// beyond the L2 (the 3D pack outgrows an XCD's L2), so the more targets a
// workgroup holds, the less operator traffic per target.
// The operator of the next offset is prefetched into registers while the
// current one is in use and double-buffered in LDS, in the lane-major order in
// which the MFMA steps consume it (conflict-free LDS reads); source moments are
// read straight from global memory (each is used by one target per offset).
// The degree-0 input enters as one more MFMA step (K = 1, lane group 0); the
// degree-0 output uses VALU fused multiply-adds.
#include "device_common.h"
#include "points3d.h"

namespace sffmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Mfma16x;
template <>
struct Mfma16x<float> {
  using acc_t = floatx4;
  using vec_t = floatx4;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma16x<double> {
  using acc_t = doublex4;
  using vec_t = doublex2;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// LDS of a workgroup: the operator slot double-buffered where two fit the
// 160 KB of a CU, else one buffer (the 128 x 128 point-charge operators of
// n = 5 in FP64), refilled between two barriers.
template <typename T, int KS, int NB>
__host__ __device__ constexpr int m2l3_lds_slots() {
  return 2 * (64 * (NB * (KS + 1) + KS) + 4) * (int)sizeof(T) <= 160 * 1024 ? 2 : 1;
}

struct M2l3Tiles {
  int klo, khi;
  int64_t off[kMaxLevels3D + 2];  // first block of level k
  int64_t nblocks;
  int nsplit[kMaxLevels3D + 2];     // offset chunks per tile at level k (1: no split)
  int64_t pbase[kMaxLevels3D + 2];  // level k's first box row in the partial buffer
};

// Accumulator register r of lane group g holds output row 4g + r (FP32) or
// g + 4r (FP64); row i is the target (2 (i & 3) + px, 2 (i >> 2) + py, 2w + pz).
template <typename T>
__device__ __forceinline__ int crow3(int r, int g) {
  return sizeof(T) == 8 ? g + 4 * r : 4 * g + r;
}

template <typename T, int KS, int NB, int MB, int NW, bool SPLIT>
__global__ __launch_bounds__(64 * NW) void k_m2l3d_mfma(FmmArgs a, M2l3Tiles tt, M2lLayout ly) {
  using acc_t = typename Mfma16x<T>::acc_t;
  using vec_t = typename Mfma16x<T>::vec_t;
  constexpr int VW = sizeof(vec_t) / sizeof(T);  // values per vector load
  constexpr int WGLB = 64 * (NB * (KS + 1) + KS) + 4;  // lane-major slot (operators.cpp)
  constexpr int WLDS = WGLB;
  constexpr int NV = WGLB / VW;                    // vectors per slot
  constexpr int NT = 64 * NW;
  constexpr int ZL = NW * MB;  // same-parity z-layers per block
  constexpr int PRE = (NV + NT - 1) / NT;
  constexpr bool kDB = m2l3_lds_slots<T, KS, NB>() == 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* wb0 = reinterpret_cast<T*>(smem_raw);
  T* wb1 = kDB ? wb0 + WLDS : wb0;

  const int64_t blk = xcd_remap(blockIdx.x, tt.nblocks);
  int k = tt.klo;
  while (k < tt.khi && blk >= tt.off[k + 1]) ++k;
  // small levels: ns workgroups per tile, each over its own chunk of the 189
  // offsets, writing FP64 partial sums (added in chunk order by k_m2l3d_reduce)
  const int ns = SPLIT ? kM2l3Split : 1;
  const int chunk = SPLIT ? (int)((blk - tt.off[k]) % ns) : 0;
  const int64_t local = SPLIT ? (blk - tt.off[k]) / ns : blk - tt.off[k];
  const int n = 1 << k;
  // blocks per parity: nxy x nxy x nz.  With nz = nxy or nxy / 2 (or nxy <= 2)
  // a 3D Morton index below nxy^2 nz decodes to x, y < nxy and z < nz, and the
  // blocks run in Morton order; with fewer z blocks (nz = nxy / 4, sixteen
  // layers per workgroup) the top Morton bits would also bound y, so there the
  // z block is the slab index and x, y run in 2D Morton order within it.
  const int nxy = n >= 8 ? n / 8 : 1;
  const int nz = n >= 2 * ZL ? n / (2 * ZL) : 1;
  const int64_t per = (int64_t)nxy * nxy * nz;
  const int par = (int)(local / per);
  const uint32_t bm = (uint32_t)(local - (int64_t)par * per);
  const int px = par & 1, py = (par >> 1) & 1, pz = par >> 2;
  int tx0, ty0, tz0;
  if (2 * nz >= nxy) {
    tx0 = 8 * (int)compact3(bm);
    ty0 = 8 * (int)compact3(bm >> 1);
    tz0 = 2 * ZL * (int)compact3(bm >> 2);
  } else {
    const uint32_t slab = bm / (uint32_t)(nxy * nxy), r = bm - slab * (uint32_t)(nxy * nxy);
    tx0 = 8 * (int)compact2(r);
    ty0 = 8 * (int)compact2(r >> 1);
    tz0 = 2 * ZL * (int)slab;
  }
  const int cs = ly.cs;
  constexpr bool kF64 = sizeof(T) == 8;
  const T* mom = (kF64 ? (const T*)a.mom64 : (const T*)a.mom32) + a.lt.off[k] * cs;
  T* loc = (kF64 ? (T*)a.loc64 : (T*)a.loc32) + a.lt.off[k] * cs;
  const T* ops = kF64 ? (const T*)a.opl64 : (const T*)a.opl32;
  const int i00 = ly.nr - 1;  // index of the degree-0 value

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int tx = tx0 + 2 * (i & 3) + px, ty = ty0 + 2 * (i >> 2) + py;
  int tzm[MB];  // the z of this lane's target in each of the wave's layers
#pragma unroll
  for (int m = 0; m < MB; ++m) tzm[m] = tz0 + 2 * (w + NW * m) + pz;
  const int xlo = px ? -3 : -2, ylo = py ? -3 : -2, zlo = pz ? -3 : -2;

  // offset q (0..215 over the 6 x 6 x 6 range; 27 of them are adjacent).  Along
  // x the window runs in steps of two, 0 2 4 1 3 5: consecutive offsets then
  // read sources of the same x parity, three quarters of them the same boxes,
  // which the L2 still holds.
  auto xstep = [](int r) { return r < 3 ? 2 * r : 2 * r - 5; };
  auto slot_of = [&](int q, int& dx, int& dy, int& dz) -> int {
    dx = xlo + xstep(q % 6);
    dy = ylo + (q / 6) % 6;
    dz = zlo + q / 36;
    return (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);
  };
  auto adjacent = [&](int q, int xl, int yl, int zl) {
    const int dx = xl + xstep(q % 6), dy = yl + (q / 6) % 6, dz = zl + q / 36;
    return dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
  };
  auto next_q = [&](int q) {
    do ++q;
    while (q < 216 && adjacent(q, xlo, ylo, zlo));
    return q;
  };
  auto nth_q = [&](int m) {  // the m-th (from 0) offset of the list, 216 past its end
    int q = -1;
    for (int e = 0; e <= m; ++e) q = next_q(q);
    return q;
  };
  const int q_stop = SPLIT ? nth_q((chunk + 1) * 189 / ns) : 216;
  // FP32: each offset's contribution is formed in the MFMA accumulators and
  // added into FP64 sums (the 189-offset sum is not left to FP32 rounding).
  acc_t acc[MB][NB];
  double sum[MB][NB][4];
  double b0p[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    b0p[m] = 0.0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      acc[m][nb] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) sum[m][nb][r] = 0.0;
    }
  }

  // W of offset q: global slot -> registers (fetch) -> LDS (store), lane-major as in memory
#define SFFMM_FETCH(qq)                                                                      \
  {                                                                                          \
    int fx, fy, fz;                                                                          \
    const vec_t* W = reinterpret_cast<const vec_t*>(ops + (size_t)slot_of(qq, fx, fy, fz) *  \
                                                                 WGLB);                     \
    _Pragma("unroll") for (int u = 0; u < PRE; ++u) {                                        \
      const int e = tid + NT * u;                                                            \
      pre[u] = W[e < NV ? e : NV - 1];                                                       \
    }                                                                                        \
  }
#define SFFMM_STORE(buf)                                                                     \
  {                                                                                          \
    _Pragma("unroll") for (int u = 0; u < PRE; ++u) {                                        \
      const int e = (tid + NT * u) * VW;                                                     \
      if (e < WGLB) *reinterpret_cast<vec_t*>((buf) + e) = pre[u];                           \
    }                                                                                        \
  }
  vec_t pre[PRE];
  int q = SPLIT ? nth_q(chunk * 189 / ns) : next_q(-1);
  SFFMM_FETCH(q);
  SFFMM_STORE(wb0);
  __syncthreads();
  T* cur = wb0;
  T* nxt = wb1;
  // source row of offset qq for this lane's target in layer tz (zeros outside
  // the grid); in FP64 the next offset's is loaded while the current one is
  // contracted
#define SFFMM_LOADA(qq, tz, AV, A0)                                                          \
  {                                                                                          \
    int ex, ey, ez;                                                                          \
    (void)slot_of(qq, ex, ey, ez);                                                           \
    const int sx = tx + ex, sy = ty + ey, sz = (tz) + ez;                                    \
    const bool ok = sx >= 0 && sy >= 0 && sz >= 0 && sx < n && sy < n && sz < n && tx < n && \
                    ty < n && (tz) < n;                                                      \
    const T* A = mom + (ok ? (int64_t)(spread3(sx) | (spread3(sy) << 1) | (spread3(sz) << 2)) * cs : 0); \
    if constexpr ((KS * sizeof(T)) % 16 == 0) {                                              \
      const vec_t* Av = reinterpret_cast<const vec_t*>(A + g * KS);                          \
      _Pragma("unroll") for (int u = 0; u < KS / VW; ++u) {                                  \
        const vec_t v = Av[u];                                                               \
        _Pragma("unroll") for (int c = 0; c < VW; ++c) AV[VW * u + c] = ok ? v[c] : (T)0;    \
      }                                                                                      \
    } else {                                                                                 \
      _Pragma("unroll") for (int s = 0; s < KS; ++s) AV[s] = ok ? A[g * KS + s] : (T)0;      \
    }                                                                                        \
    A0 = ok ? A[i00] : (T)0;                                                                 \
  }
  // (FP64 with one layer only: in FP32, or with two layers, the registers of
  // a second row cost more than the latency they hide; not for K = 128)
  constexpr bool kPrefA = kF64 && MB == 1 && KS < 32;
  T avn[KS], a0n = 0;
  if (kPrefA) SFFMM_LOADA(q, tzm[0], avn, a0n);
  while (q < q_stop) {
    const int qn = next_q(q);
    if (qn < q_stop) SFFMM_FETCH(qn);
    T av[MB][KS], a0[MB];
    if (kPrefA) {
#pragma unroll
      for (int s = 0; s < KS; ++s) av[0][s] = avn[s];
      a0[0] = a0n;
      if (qn < q_stop) SFFMM_LOADA(qn, tzm[0], avn, a0n);
    } else {
#pragma unroll
      for (int m = 0; m < MB; ++m) SFFMM_LOADA(q, tzm[m], av[m], a0[m]);
    }
    const T* Wl = cur;
    if constexpr (KS == 32) {
      // one layer per wave and one wave per SIMD: the NB output blocks in the
      // inner loop, so consecutive products go to independent accumulators
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[0][nb] = Mfma16x<T>::op(av[0][s], Wl[((size_t)nb * (KS + 1) + s) * 64 + lane],
                                      acc[0][nb]);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)  // the degree-0 input step (K = 1, lane group 0)
        acc[0][nb] = Mfma16x<T>::op(g == 0 ? a0[0] : (T)0,
                                    Wl[((size_t)nb * (KS + 1) + KS) * 64 + lane], acc[0][nb]);
    } else {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const T* Wb = Wl + (size_t)nb * (KS + 1) * 64 + lane;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const T wv = Wb[s * 64];
#pragma unroll
          for (int m = 0; m < MB; ++m) acc[m][nb] = Mfma16x<T>::op(av[m][s], wv, acc[m][nb]);
        }
        const T wv = Wb[KS * 64];
#pragma unroll
        for (int m = 0; m < MB; ++m)  // the degree-0 input step (K = 1, lane group 0)
          acc[m][nb] = Mfma16x<T>::op(g == 0 ? a0[m] : (T)0, wv, acc[m][nb]);
      }
    }
    const T* R = Wl + (size_t)NB * (KS + 1) * 64;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      T b0o = 0;
#pragma unroll
      for (int s = 0; s < KS; ++s) b0o += R[s * 64 + lane] * av[m][s];
      if (g == 0) b0o += R[KS * 64] * a0[m];  // degree 0 -> degree 0
      b0p[m] += (double)b0o;
    }
    if constexpr (!kF64) {
#pragma unroll
      for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) sum[m][nb][r] += (double)acc[m][nb][r];
          acc[m][nb] = acc_t{0, 0, 0, 0};
        }
    }
    if constexpr (!kDB) __syncthreads();  // every wave done with the one buffer
    if (qn < q_stop) SFFMM_STORE(nxt);
    __syncthreads();
    T* t = cur;
    cur = nxt;
    nxt = t;
    q = qn;
  }
#undef SFFMM_FETCH
#undef SFFMM_STORE
#undef SFFMM_LOADA
  const int nout = ly.nr - 1;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    double b0 = b0p[m];
    b0 += __shfl_xor(b0, 16, 64);
    b0 += __shfl_xor(b0, 32, 64);
    const int tz = tzm[m];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ci = crow3<T>(r, g);
      const int gx = tx0 + 2 * (ci & 3) + px, gy = ty0 + 2 * (ci >> 2) + py;
      // the C rows of this lane belong to the wave's layer (all lanes share tz)
      if (gx < n && gy < n && tz < n) {
        const int64_t bx = (int64_t)(spread3(gx) | (spread3(gy) << 1) | (spread3(tz) << 2));
        if constexpr (SPLIT) {
          double* pdst = a.m2l_part + ((int64_t)chunk * kM2l3SplitBoxes + tt.pbase[k] + bx) * cs;
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int j = 16 * nb + i;
            if (j < nout) pdst[j] = kF64 ? (double)acc[m][nb][r] : sum[m][nb][r];
          }
        } else {
          T* dst = loc + bx * cs;
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int j = 16 * nb + i;
            if (j < nout) dst[j] = kF64 ? (T)acc[m][nb][r] : (T)sum[m][nb][r];
          }
        }
      }
    }
    if (g == 0 && tx < n && ty < n && tz < n) {
      const int64_t bx = (int64_t)(spread3(tx) | (spread3(ty) << 1) | (spread3(tz) << 2));
      if constexpr (SPLIT)
        a.m2l_part[((int64_t)chunk * kM2l3SplitBoxes + tt.pbase[k] + bx) * cs + i00] = b0;
      else
        loc[bx * cs + i00] = (T)b0;
    }
  }
}

// loc[b][j] = sum over chunks c (in order) of the partial rows of level k
template <typename T>
__global__ void k_m2l3d_reduce(const double* part, T* loc, int64_t nbox, int cs, int nr, int ns,
                               int64_t pbase) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nbox * nr) return;
  const int64_t b = g / nr;
  const int j = (int)(g - b * nr);
  double s = 0.0;
  for (int c = 0; c < ns; ++c) s += part[((int64_t)c * kM2l3SplitBoxes + pbase + b) * cs + j];
  loc[b * cs + j] = (T)s;
}

template <typename T, int KS, int NB, int MB, int NW, bool SPLIT>
static void m2l3_launch(const FmmArgs& a, const M2l3Tiles& tt, const M2lLayout& ly,
                        hipStream_t st) {
  const size_t lds = (size_t)m2l3_lds_slots<T, KS, NB>() * (64 * (NB * (KS + 1) + KS) + 4) *
                     sizeof(T);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_m2l3d_mfma<T, KS, NB, MB, NW, SPLIT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_m2l3d_mfma<T, KS, NB, MB, NW, SPLIT>), dim3(tt.nblocks), dim3(64 * NW), lds,
                     st, a, tt, ly);
  if (SPLIT)
    for (int k = tt.klo; k <= tt.khi; ++k) {
      const int64_t nbox = (int64_t)1 << (3 * k), cnt = nbox * ly.nr;
      T* loc = (sizeof(T) == 8 ? (T*)a.loc64 : (T*)a.loc32) + a.lt.off[k] * ly.cs;
      hipLaunchKernelGGL(k_m2l3d_reduce<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
                         a.m2l_part, loc, nbox, ly.cs, ly.nr, tt.nsplit[k], tt.pbase[k]);
    }
}

// Tile variant mb: 4 mb layers of 16 targets per workgroup (mb = 4: eight
// waves of two layers; FP32 only, the FP64 registers of two layers leave room
// for one wave per SIMD).
template <typename T, int KS, int NB, bool SPLIT>
static void m2l3_mb(const FmmArgs& a, const M2l3Tiles& tt, const M2lLayout& ly, hipStream_t st) {
  if constexpr (KS == 32) {  // K = N = 128: one layer per wave, one workgroup per CU
    m2l3_launch<T, KS, NB, 1, 4, SPLIT>(a, tt, ly, st);
  } else {
    if constexpr (sizeof(T) == 4) {
      if (a.m2l_mb == 4) {
        m2l3_launch<T, KS, NB, 2, 8, SPLIT>(a, tt, ly, st);
        return;
      }
    }
    if (a.m2l_mb == 2)
      m2l3_launch<T, KS, NB, 2, 4, SPLIT>(a, tt, ly, st);
    else
      m2l3_launch<T, KS, NB, 1, 4, SPLIT>(a, tt, ly, st);
  }
}

template <typename T, int KS, int NB>
static void m2l3_split(const FmmArgs& a, const M2l3Tiles& tt, const M2lLayout& ly, bool split,
                       hipStream_t st) {
  if (split)
    m2l3_mb<T, KS, NB, true>(a, tt, ly, st);
  else
    m2l3_mb<T, KS, NB, false>(a, tt, ly, st);
}

bool m2l3d_variant_ok(int mb, bool fp64) { return mb == 1 || mb == 2 || (mb == 4 && !fp64); }

void launch_m2l3d(const FmmArgs& a, bool fp64, hipStream_t st) {
  if (a.khi < a.klo) return;
  const M2lLayout ly = a.basis ? points3d_layout_n(a.p) : m2l3d_layout(order_bucket3(a.p));
  const int mb = ly.kpad == 128 ? 1 : m2l3d_variant_ok(a.m2l_mb, fp64) ? a.m2l_mb : 1;
  const int zl = 4 * mb;  // same-parity z-layers per block
  FmmArgs am = a;
  am.m2l_mb = mb;
  // levels 2 and 3 have 8 tiles each: their own launch splits each tile's
  // offsets over kM2l3Split workgroups; the larger levels run unsplit
  const int ksplit = a.m2l_part ? std::min(a.khi, kM2l3SplitLevel) : a.klo - 1;
  for (int part = 0; part < 2; ++part) {
    const bool split = part == 0;
    const int klo = split ? a.klo : std::max(a.klo, ksplit + 1);
    const int khi = split ? ksplit : a.khi;
    if (khi < klo) continue;
    M2l3Tiles tt{};
    tt.klo = klo;
    tt.khi = khi;
    int64_t t = 0;
    for (int k = klo; k <= khi; ++k) {
      tt.off[k] = t;
      const int n = 1 << k;
      const int64_t nxy = n >= 8 ? n / 8 : 1, nz = n >= 2 * zl ? n / (2 * zl) : 1;
      tt.nsplit[k] = split ? kM2l3Split : 1;
      tt.pbase[k] = k == 3 ? 64 : 0;
      t += 8 * nxy * nxy * nz * tt.nsplit[k];
    }
    tt.off[khi + 1] = t;
    tt.nblocks = t;
    if (a.basis && ly.kpad == 128) {  // 125 point charges: K = N = 128
      if (fp64)
        m2l3_split<double, 32, 8>(am, tt, ly, split, st);
      else
        m2l3_split<float, 32, 8>(am, tt, ly, split, st);
    } else if (a.basis) {  // up to 64 point charges: K = N = 64
      if (fp64)
        m2l3_split<double, 16, 4>(am, tt, ly, split, st);
      else
        m2l3_split<float, 16, 4>(am, tt, ly, split, st);
    } else if (ly.p == 4) {
      if (fp64)
        m2l3_split<double, 6, 2>(am, tt, ly, split, st);
      else
        m2l3_split<float, 6, 2>(am, tt, ly, split, st);
    } else {
      if (fp64)
        m2l3_split<double, 20, 5>(am, tt, ly, split, st);
      else
        m2l3_split<float, 20, 5>(am, tt, ly, split, st);
    }
  }
}

}  // namespace sffmm
