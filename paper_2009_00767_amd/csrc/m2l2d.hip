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
  int remap;  // deal tiles to the XCDs in contiguous ranges
};

constexpr int kHalo = 14;  // 8 targets + 3 on each side (x); 8 MB + 6 rows (y)

// Output row held in accumulator register r by lane group g: 4g + r for the
// FP32 16x16x4 MFMA, g + 4r for the FP64 one (checked on gfx950).  Row i is the
// target (2 (i & 3) + px, 2 (i >> 2) + py) of the wave's parity class.  In both,
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
template <typename T>
__device__ __forceinline__ int crow_x(int r, int g) {
  return sizeof(T) == 8 ? 2 * g : 2 * r;
}
template <typename T>
__device__ __forceinline__ int crow_y(int r, int g) {
  return sizeof(T) == 8 ? 2 * r : 2 * g;
}

// Tile of one workgroup: 8 x (8 MB) target boxes of one level.  Wave w takes
// the targets of parity class (w & 1, w >> 1): MB blocks of 16 targets that
// share every operator load (MB, the tile height and the tile order are the
// tuning parameters; the arithmetic of each target is the same for every
// choice).  MB = 1 tiles are visited in Morton order, taller tiles row by row.
//
// K runs in natural order: MFMA step s contracts the values 4s..4s+3 of each
// source row, lane group g supplying value 4s + g (FP32 / FP64 16x16x4), and
// only the steps below this level's order are issued.  The source halo sits in
// LDS as four parity planes (the targets of one wave read sources of one
// parity for a given offset), coefficient-major, plane rows 8 boxes wide and
// the coefficient stride congruent to 4 modulo 32 banks: the 16 targets of a
// lane group read 16 distinct banks and two lane groups tile all 32.
// The operators come from the lane-major pack: one coalesced dword per lane
// and step, the A_0 column as one more K = 1 step (lane group 0 only).
template <int MB>
struct HaloGeom {
  static constexpr int HY = 8 * MB + 6;        // halo rows
  static constexpr int PSZ = 8 * (4 * MB + 3); // boxes per parity plane (8-wide rows)
  static constexpr int KST = 4 * PSZ + 4;      // per coefficient; = 4 mod 32
};

// FULL: every level of the launch runs at the layout order (pk = pb), so the
// step and block counts are the compile-time KS, NB and no guard is emitted.
template <typename T, int KS, int NB, int MB, bool FULL>
__global__ __launch_bounds__(256) void k_m2l2d_mfma(FmmArgs a, M2lTiles tt, M2lLayout ly) {
  using G = HaloGeom<MB>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* halo = reinterpret_cast<T*>(smem_raw);
  using acc_t = typename Mfma16<T>::acc_t;
  constexpr bool kF64 = sizeof(T) == 8;

  const int64_t tile = tt.remap ? xcd_remap(blockIdx.x, tt.ntiles) : (int64_t)blockIdx.x;
  int k = tt.klo;
  while (k < tt.khi && tile >= tt.off[k + 1]) ++k;
  const int n = 1 << k;
  const int ntx = (n + 7) / 8, nty = (n + 8 * MB - 1) / (8 * MB);
  const int64_t tper = (int64_t)ntx * nty;  // tiles per system
  const int64_t tg = tile - tt.off[k];
  const uint32_t sys = (uint32_t)(tg / tper), tl = (uint32_t)(tg - (int64_t)sys * tper);
  const uint32_t sysb = sys << (2 * k);  // system bits of this level's box indices
  int tx0, ty0;
  if (MB == 1) {
    tx0 = 8 * (int)compact2(tl);
    ty0 = 8 * (int)compact2(tl >> 1);
  } else {
    tx0 = 8 * (int)(tl % (uint32_t)ntx);
    ty0 = 8 * MB * (int)(tl / (uint32_t)ntx);
  }
  if (a.depth && k > a.lt.kmin) {
    // adaptive depth: a level-k local is read only by particles whose depth
    // reaches k, i.e. in a box whose parent is open; a tile with no such box
    // is left alone
    int act = 0;
    const int t = threadIdx.x;
    if (t < 16 * MB) {
      const int px = (tx0 >> 1) + (t & 3), py = (ty0 >> 1) + (t >> 2), np = n >> 1;
      if (px < np && py < np)
        act = a.adapt_open[adapt_open_off(k - 1) + (spread2(px) | (spread2(py) << 1))] & 1;
    }
    if (!__syncthreads_or(act)) return;
  }
  const int cs = ly.cs, pb = ly.p;  // layout order (the order bucket)
  const T* mom = (kF64 ? (const T*)a.mom64 : (const T*)a.mom32) + a.lt.off[k] * cs;
  T* loc = (kF64 ? (T*)a.loc64 : (T*)a.loc32) + a.lt.off[k] * cs;
  const T* ops = kF64 ? (const T*)a.opl64 : (const T*)a.opl32;

  // Stage the source halo (zeros outside the grid) into the parity planes, four
  // consecutive values of one box row per thread.  A row holds cs = 2 pb + 4 =
  // 4 (KS + 1) values for every order bucket (pb even: kpad = 2 pb = 4 KS), so
  // the index arithmetic has compile-time divisors, and rows are 16-byte aligned.
  constexpr int CS4 = KS + 1;
  for (int e = threadIdx.x; e < kHalo * G::HY * CS4; e += 256) {
    const int hb = e / CS4, c4 = e - hb * CS4;
    const int lx = hb % kHalo, lyy = hb / kHalo;
    const int sx = tx0 - 3 + lx, sy = ty0 - 3 + lyy;
    T v[4] = {(T)0, (T)0, (T)0, (T)0};
    if (sx >= 0 && sy >= 0 && sx < n && sy < n) {
      const T* src = mom + (int64_t)(sysb | spread2(sx) | (spread2(sy) << 1)) * (4 * CS4) + 4 * c4;
      if constexpr (kF64) {
        const double2 u0 = reinterpret_cast<const double2*>(src)[0];
        const double2 u1 = reinterpret_cast<const double2*>(src)[1];
        v[0] = u0.x;
        v[1] = u0.y;
        v[2] = u1.x;
        v[3] = u1.y;
      } else {
        const float4 u = *reinterpret_cast<const float4*>(src);
        v[0] = u.x;
        v[1] = u.y;
        v[2] = u.z;
        v[3] = u.w;
      }
    }
    T* dst = halo + 4 * c4 * G::KST + (((lyy & 1) << 1) | (lx & 1)) * G::PSZ + (lyy >> 1) * 8 +
             (lx >> 1);
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[j * G::KST] = v[j];
  }
  __syncthreads();

  // the wave index is uniform: in a scalar register every offset slot and
  // operator address derived from it stays scalar
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int px = w & 1, py = w >> 1;
  const int i = lane & 15, g = lane >> 4;
  const int ix = 2 * (i & 3) + px, iy = 2 * (i >> 2) + py;  // A-row target of this lane
  acc_t acc[MB][NB];
  T b0p[MB], a0s[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    b0p[mb] = a0s[mb] = (T)0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = acc_t{0, 0, 0, 0};
  }
  const int xlo = px ? -3 : -2, ylo = py ? -3 : -2;
  // This level's order pk <= pb: the moments above pk are zero and the locals
  // above pk are never read, so only the steps below 2 pk (ksr) and the output
  // blocks below 2 pk (nbr) are formed.
  const int pk = FULL ? pb : a.ord[k];
  const int ksr = FULL ? KS : (pk + 1) / 2;
  const int nbr = FULL ? NB : (pk + 7) / 8;
  const int a0k = 2 * pb;  // coefficient 0 sits after the pb complex ones

  // The 27 offsets of this wave's parity class: the 6 x 6 window (dx, dy) =
  // (wx + xlo, wy + ylo) minus the 3 x 3 near block, in row-major window order.
  uint64_t todo = (1ull << 36) - 1;
  {
    const int nx0 = px ? 2 : 1, ny0 = py ? 2 : 1;
    for (int yy = 0; yy < 3; ++yy)
      for (int xx = 0; xx < 3; ++xx) todo &= ~(1ull << ((ny0 + yy) * 6 + nx0 + xx));
  }

  // Operator registers of one offset (the next offset's are loaded while the
  // current one is contracted): dense B steps, the A_0 step, Re B_0 weights and
  // Re log(-u).
#define SFFMM_M2L_LOADW(WI, BV, C0, R0, RL)                                                   \
  {                                                                                           \
    const int slot_ = ((WI) % 6 + xlo + 3) + 7 * ((WI) / 6 + ylo + 3);                        \
    const T* P_ = ops + (size_t)slot_ * ly.lstride;                                           \
    _Pragma("unroll") for (int nb = 0; nb < NB; ++nb) {                                       \
      _Pragma("unroll") for (int st = 0; st < KS; ++st) {                                     \
        BV[nb][st] = (nb < nbr && st < ksr) ? P_[((size_t)nb * (KS + 1) + st) * 64 + lane]    \
                                            : (T)0;                                           \
      }                                                                                       \
    }                                                                                         \
    _Pragma("unroll") for (int nb = 0; nb < NB; ++nb) {                                       \
      C0[nb] = nb < nbr ? P_[((size_t)nb * (KS + 1) + KS) * 64 + lane] : (T)0;                \
    }                                                                                         \
    const T* R_ = P_ + (size_t)NB * (KS + 1) * 64;                                            \
    _Pragma("unroll") for (int st = 0; st < KS; ++st) {                                       \
      R0[st] = st < ksr ? R_[(size_t)st * 64 + lane] : (T)0;                                  \
    }                                                                                         \
    RL = R_[(size_t)KS * 64];                                                                 \
  }

  // One offset.  FP32 / FP64: step s multiplies A = source value 4s + g of the
  // lane's target row by the pack's B step; BF16: chunk c takes the lane's 8
  // values 32c + 8g .. 32c + 8g + 7.  Re B_0 accumulates r0[4s + g] times the
  // same values; the A_0 step adds A_0 c0^T.
#define SFFMM_M2L_STEP(WI, BV, C0, R0, RL)                                                    \
  {                                                                                           \
    const int dx_ = (WI) % 6 + xlo, dy_ = (WI) / 6 + ylo;                                     \
    T a0v[MB];                                                                                \
    _Pragma("unroll") for (int mb = 0; mb < MB; ++mb) {                                       \
      const int lx_ = ix + dx_ + 3, ly_ = iy + 8 * mb + dy_ + 3;                              \
      const T* hp = halo + (((ly_ & 1) << 1) | (lx_ & 1)) * G::PSZ + (ly_ >> 1) * 8 + (lx_ >> 1); \
      a0v[mb] = g == 0 ? hp[a0k * G::KST] : (T)0;                                             \
      _Pragma("unroll") for (int st = 0; st < KS; ++st) {                                     \
        if (st < ksr) {                                                                       \
          const T av = hp[(4 * st + g) * G::KST];                                             \
          _Pragma("unroll") for (int nb = 0; nb < NB; ++nb) {                                 \
            if (nb < nbr) acc[mb][nb] = Mfma16<T>::op(av, BV[nb][st], acc[mb][nb]);           \
          }                                                                                   \
          b0p[mb] += R0[st] * av;                                                             \
        }                                                                                     \
      }                                                                                       \
      b0p[mb] += (g == 0 ? RL : (T)0) * a0v[mb];                                              \
      a0s[mb] += a0v[mb];                                                                     \
      _Pragma("unroll") for (int nb = 0; nb < NB; ++nb) {                                     \
        if (nb < nbr) acc[mb][nb] = Mfma16<T>::op(a0v[mb], C0[nb], acc[mb][nb]);              \
      }                                                                                       \
    }                                                                                         \
  }

  T bvA[NB][KS], bvB[NB][KS], c0A[NB], c0B[NB], r0A[KS], r0B[KS], rlA, rlB;
  // the largest FP64 blocks have no registers for a second set
  constexpr bool kPipe = NB * KS * sizeof(T) / 4 <= 96;
  int wcur = __builtin_ctzll(todo);
  todo &= todo - 1;
  SFFMM_M2L_LOADW(wcur, bvA, c0A, r0A, rlA);
  if (!kPipe) {
    for (;;) {
      SFFMM_M2L_STEP(wcur, bvA, c0A, r0A, rlA);
      if (!todo) break;
      wcur = __builtin_ctzll(todo);
      todo &= todo - 1;
      SFFMM_M2L_LOADW(wcur, bvA, c0A, r0A, rlA);
    }
  }
  // The next offset's operators are loaded on every path, past the last offset
  // too (a repeat of the current one, never used): with the same loads in
  // flight on every path the compiler's wait before a step covers only the
  // older set, and the newer set's latency hides behind the step.
  while (kPipe) {
    const bool more = todo != 0;
    const int wnext = more ? __builtin_ctzll(todo) : wcur;
    todo &= todo - 1;
    SFFMM_M2L_LOADW(wnext, bvB, c0B, r0B, rlB);
    SFFMM_M2L_STEP(wcur, bvA, c0A, r0A, rlA);
    if (!more) break;
    const bool more2 = todo != 0;
    wcur = more2 ? __builtin_ctzll(todo) : wnext;
    todo &= todo - 1;
    SFFMM_M2L_LOADW(wcur, bvA, c0A, r0A, rlA);
    SFFMM_M2L_STEP(wnext, bvB, c0B, r0B, rlB);
    if (!more2) break;
  }
#undef SFFMM_M2L_LOADW
#undef SFFMM_M2L_STEP
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    T bp = b0p[mb], as = a0s[mb];
    bp += __shfl_xor(bp, 16, 64);
    bp += __shfl_xor(bp, 32, 64);
    as += __shfl_xor(as, 16, 64);
    as += __shfl_xor(as, 32, 64);
    const T b0 = bp + (T)a.lt.log_s[k] * as;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gx = tx0 + crow_x<T>(r, g) + px, gy = ty0 + crow_y<T>(r, g) + py + 8 * mb;
      if (gx < n && gy < n) {
        T* dst = loc + (int64_t)(sysb | spread2(gx) | (spread2(gy) << 1)) * cs;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int j = 16 * nb + i;
          if (j < 2 * pb) dst[j] = acc[mb][nb][r];
        }
      }
    }
    if (g == 0) {
      const int gx = tx0 + ix, gy = ty0 + iy + 8 * mb;
      if (gx < n && gy < n) {
        T* dst = loc + (int64_t)(sysb | spread2(gx) | (spread2(gy) << 1)) * cs;
        dst[2 * pb] = b0;
        dst[2 * pb + 1] = (T)0;  // Im B_0 enters neither the potential nor the field
      }
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 mode: every product of an offset, the A_0 terms and Re B_0 included,
// runs as v_mfma_f32_16x16x32_bf16 steps with FP32 accumulation.  Output column
// 0 of the products is Re B_0 and column 1 + j output value j; the K order
// (the BF16 operator pack in operators.cpp) is
//   0..5           the real A_0 as the cross products hi.hi, hi.mid, mid.hi,
//                  hi.lo, mid.mid, lo.hi of three-part BF16 splits of A_0 and of
//                  the operator's A_0 entries: the A_0 terms, the largest of the
//                  far field, to FP32 accuracy;
//   6 + k          input value k (re/im of coefficients 1..pb) rounded to BF16;
//   6 + 2pb + ...  for the leading ms coefficients (the largest terms after A_0)
//                  the low parts of the inputs against the high parts of the
//                  operator, then the high parts against the low parts: two-term
//                  splits on both sides, in K positions the chunk would pad.
//
// The source halo sits in LDS as BF16 rows in that K order, KC chunks of 32
// values per box, in four parity planes of 7-box rows.  Lane (i, g) reads the
// 16-byte part 4c + g of its target's source row with one ds_read_b128 per
// chunk c; the parts of a row are rotated by (bx & 3) | ((by & 1) << 2) of the
// box's plane coordinates, so that the boxes of 8 consecutive lanes (4 columns
// by 2 rows of one plane) fall in 8 distinct 16-byte bank groups.  The FP32 A_0
// values, for the level term log s * sum A_0 of Re B_0, sit in a plane of
// their own.  One operator load (NBB x KC parts per lane) serves the MB blocks
// of 16 targets of the wave.
template <int MB, int KC>
struct BfHalo {
  static constexpr int PW = 7;                   // boxes per plane row
  static constexpr int PSZ = PW * (4 * MB + 3);  // boxes per parity plane
  static constexpr int NBOX = 4 * PSZ;
  static constexpr int P = 4 * KC;               // 16-byte parts per row
  static constexpr int RB = 16 * P;              // bytes per row
  static constexpr size_t bytes() { return (size_t)NBOX * (RB + 4); }
};

__device__ __forceinline__ int bf_rot(int bx, int by) { return (bx & 3) | ((by & 1) << 2); }

template <int PB, int MB, bool FULL>
__global__ __launch_bounds__(256) void k_m2l2d_bf16(FmmArgs a, M2lTiles tt, M2lLayout ly) {
  constexpr int KC = bf16_chunks(PB), NBB = (1 + 2 * PB + 15) / 16, MS = bf16_split(PB);
  constexpr int KQ = 6 + 2 * PB + 4 * MS;  // K positions in use
  using H = BfHalo<MB, KC>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* rows = smem_raw;
  float* a0p = reinterpret_cast<float*>(smem_raw + (size_t)H::NBOX * H::RB);

  const int64_t tile = tt.remap ? xcd_remap(blockIdx.x, tt.ntiles) : (int64_t)blockIdx.x;
  int k = tt.klo;
  while (k < tt.khi && tile >= tt.off[k + 1]) ++k;
  const int n = 1 << k;
  const int ntx = (n + 7) / 8, nty = (n + 8 * MB - 1) / (8 * MB);
  const int64_t tper = (int64_t)ntx * nty;
  const int64_t tg = tile - tt.off[k];
  const uint32_t sys = (uint32_t)(tg / tper), tl = (uint32_t)(tg - (int64_t)sys * tper);
  const uint32_t sysb = sys << (2 * k);
  int tx0, ty0;
  if (MB == 1) {
    tx0 = 8 * (int)compact2(tl);
    ty0 = 8 * (int)compact2(tl >> 1);
  } else {
    tx0 = 8 * (int)(tl % (uint32_t)ntx);
    ty0 = 8 * MB * (int)(tl / (uint32_t)ntx);
  }
  if (a.depth && k > a.lt.kmin) {
    // adaptive depth: a level-k local is read only by particles whose depth
    // reaches k, i.e. in a box whose parent is open; a tile with no such box
    // is left alone
    int act = 0;
    const int t = threadIdx.x;
    if (t < 16 * MB) {
      const int px = (tx0 >> 1) + (t & 3), py = (ty0 >> 1) + (t >> 2), np = n >> 1;
      if (px < np && py < np)
        act = a.adapt_open[adapt_open_off(k - 1) + (spread2(px) | (spread2(py) << 1))] & 1;
    }
    if (!__syncthreads_or(act)) return;
  }
  constexpr int cs = 2 * PB + 4, pb = PB;  // values per box row (ly.cs)
  const float* mom = a.mom32 + a.lt.off[k] * cs;
  float* loc = a.loc32 + a.lt.off[k] * cs;

  // Stage the halo: one float4 of one box's FP32 row per task, its values
  // written as BF16 pairs at their K positions (the float4 holding A_0 also
  // writes the six A_0 slots and the zero tail).  The loads of a batch of tasks
  // are issued before any is used.
  constexpr int HY = 8 * MB + 6;
  constexpr int C4 = cs / 4;
  constexpr int NT = kHalo * HY * C4;
  constexpr int IT = (NT + 255) / 256;
  constexpr int BATCH = IT < 8 ? IT : 8;
  auto put2 = [&](unsigned char* row, int rot, int kq, float x0, float x1) {
    // BF16 pair at the even K position kq of a row (parts rotated by rot)
    const int part = kq >> 3;
    __bf16* d = reinterpret_cast<__bf16*>(row + ((part + rot) % H::P) * 16 + (kq & 7) * 2);
    d[0] = (__bf16)x0;
    d[1] = (__bf16)x1;
  };
  for (int it0 = 0; it0 < IT; it0 += BATCH) {
    float4 u[BATCH];
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      const int e = threadIdx.x + 256 * (it0 + b);
      u[b] = float4{0.f, 0.f, 0.f, 0.f};
      if (e < NT) {
        const int hb = e / C4, t = e - hb * C4;
        const int sx = tx0 - 3 + hb % kHalo, sy = ty0 - 3 + hb / kHalo;
        if (sx >= 0 && sy >= 0 && sx < n && sy < n)
          u[b] = reinterpret_cast<const float4*>(
              mom + (int64_t)(sysb | spread2(sx) | (spread2(sy) << 1)) * cs)[t];
      }
    }
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      const int e = threadIdx.x + 256 * (it0 + b);
      if (e >= NT) continue;
      const int hb = e / C4, t = e - hb * C4;
      const int lx = hb % kHalo, lyy = hb / kHalo;
      const int bx = lx >> 1, by = lyy >> 1;
      const int pos = (((lyy & 1) << 1) | (lx & 1)) * H::PSZ + by * H::PW + bx;
      unsigned char* row = rows + (size_t)pos * H::RB;
      const int rot = bf_rot(bx, by);
      const float v[4] = {u[b].x, u[b].y, u[b].z, u[b].w};
      if (4 * t < 2 * pb) {
#pragma unroll
        for (int h = 0; h < 4; h += 2) {
          const int kk = 4 * t + h;  // input value index
          put2(row, rot, 6 + kk, v[h], v[h + 1]);
          if (kk < 2 * MS) {
            const float h0 = (float)(__bf16)v[h], h1 = (float)(__bf16)v[h + 1];
            put2(row, rot, 6 + 2 * pb + kk, v[h] - h0, v[h + 1] - h1);
            put2(row, rot, 6 + 2 * pb + 2 * MS + kk, v[h], v[h + 1]);
          }
        }
      } else {  // the float4 of A_0 (re, im = 0, padding)
        const float a0 = v[0];
        const float hi = (float)(__bf16)a0;
        const float mid = (float)(__bf16)(a0 - hi);
        const float lo = a0 - hi - mid;
        put2(row, rot, 0, hi, hi);
        put2(row, rot, 2, mid, hi);
        put2(row, rot, 4, mid, lo);
#pragma unroll
        for (int kq = KQ; kq < 32 * KC; kq += 2) put2(row, rot, kq, 0.f, 0.f);
        a0p[pos] = a0;
      }
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int px = w & 1, py = w >> 1;
  const int i = lane & 15, g = lane >> 4;
  const int ix = 2 * (i & 3) + px, iy = 2 * (i >> 2) + py;  // A-row target of this lane
  floatx4 acc[MB][NBB];
  float a0s[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    a0s[mb] = 0.f;
#pragma unroll
    for (int nb = 0; nb < NBB; ++nb) acc[mb][nb] = floatx4{0, 0, 0, 0};
  }
  const int xlo = px ? -3 : -2, ylo = py ? -3 : -2;
  // This level's order pk <= pb: output blocks beyond 1 + 2 pk outputs are not
  // formed (the locals above pk are never read); every chunk is (each holds
  // split slots of the leading coefficients).
  const int pk = FULL ? pb : a.ord[k];
  const int ksr = KC;
  const int nbr = FULL ? NBB : (1 + 2 * pk + 15) / 16;
  uint64_t todo = (1ull << 36) - 1;
  {
    const int nx0 = px ? 2 : 1, ny0 = py ? 2 : 1;
    for (int yy = 0; yy < 3; ++yy)
      for (int xx = 0; xx < 3; ++xx) todo &= ~(1ull << ((ny0 + yy) * 6 + nx0 + xx));
  }
  const bf16x8 bzero = {};

#define SFFMM_BF_LOADW(WI, BB)                                                                \
  {                                                                                           \
    const int slot_ = ((WI) % 6 + xlo + 3) + 7 * ((WI) / 6 + ylo + 3);                        \
    const __bf16* Ph_ = a.op16 + (size_t)slot_ * ly.l16;                                      \
    _Pragma("unroll") for (int nb = 0; nb < NBB; ++nb) {                                      \
      _Pragma("unroll") for (int c = 0; c < KC; ++c) {                                        \
        BB[nb][c] = (nb < nbr && c < ksr)                                                     \
                        ? *reinterpret_cast<const bf16x8*>(Ph_ +                               \
                                                           ((size_t)(nb * KC + c) * 64 + lane) * 8) \
                        : bzero;                                                              \
      }                                                                                       \
    }                                                                                         \
  }
#define SFFMM_BF_STEP(WI, BB)                                                                 \
  {                                                                                           \
    const int dx_ = (WI) % 6 + xlo, dy_ = (WI) / 6 + ylo;                                     \
    _Pragma("unroll") for (int mb = 0; mb < MB; ++mb) {                                       \
      const int lx_ = ix + dx_ + 3, ly_ = iy + 8 * mb + dy_ + 3;                              \
      const int bx_ = lx_ >> 1, by_ = ly_ >> 1;                                               \
      const int pos_ = (((ly_ & 1) << 1) | (lx_ & 1)) * H::PSZ + by_ * H::PW + bx_;           \
      const unsigned char* rp_ = rows + (size_t)pos_ * H::RB;                                 \
      const int rot_ = bf_rot(bx_, by_);                                                      \
      a0s[mb] += a0p[pos_];                                                                   \
      _Pragma("unroll") for (int c = 0; c < KC; ++c) {                                        \
        if (c < ksr) {                                                                        \
          const bf16x8 av =                                                                   \
              *reinterpret_cast<const bf16x8*>(rp_ + ((4 * c + g + rot_) % H::P) * 16);       \
          _Pragma("unroll") for (int nb = 0; nb < NBB; ++nb) {                                \
            if (nb < nbr)                                                                     \
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, BB[nb][c], acc[mb][nb], \
                                                                    0, 0, 0);                 \
          }                                                                                   \
        }                                                                                     \
      }                                                                                       \
    }                                                                                         \
  }

  // the next offset's operators are loaded while the current one is contracted
  // (past the last offset a repeat of the current one, never used)
  bf16x8 bbA[NBB][KC], bbB[NBB][KC];
  int wcur = __builtin_ctzll(todo);
  todo &= todo - 1;
  SFFMM_BF_LOADW(wcur, bbA);
  for (;;) {
    const bool more = todo != 0;
    const int wnext = more ? __builtin_ctzll(todo) : wcur;
    todo &= todo - 1;
    SFFMM_BF_LOADW(wnext, bbB);
    SFFMM_BF_STEP(wcur, bbA);
    if (!more) break;
    const bool more2 = todo != 0;
    wcur = more2 ? __builtin_ctzll(todo) : wnext;
    todo &= todo - 1;
    SFFMM_BF_LOADW(wcur, bbA);
    SFFMM_BF_STEP(wnext, bbB);
    if (!more2) break;
  }
#undef SFFMM_BF_LOADW
#undef SFFMM_BF_STEP
  const float lsk = (float)a.lt.log_s[k];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // C register r of lane group g is the target row 4 g + r, whose A_0 sum
      // lane 4 g + r holds
      const float as = __shfl(a0s[mb], 4 * g + r, 64);
      const int gx = tx0 + 2 * r + px, gy = ty0 + 2 * g + py + 8 * mb;
      if (gx < n && gy < n) {
        float* dst = loc + (int64_t)(sysb | spread2(gx) | (spread2(gy) << 1)) * cs;
#pragma unroll
        for (int nb = 0; nb < NBB; ++nb) {
          const int col = 16 * nb + i;
          if (col == 0) {
            dst[2 * pb] = acc[mb][0][r] + lsk * as;
            dst[2 * pb + 1] = 0.f;  // Im B_0 enters neither the potential nor the field
          } else if (col - 1 < 2 * pb) {
            dst[col - 1] = acc[mb][nb][r];
          }
        }
      }
    }
  }
}

// LDS bytes of one workgroup (the source halo in parity planes).
static size_t m2l2d_lds(const M2lLayout& ly, int mb, bool fp64) {
  const size_t kst = (size_t)4 * 8 * (4 * mb + 3) + 4;
  return kst * ly.cs * (fp64 ? 8 : 4);
}

template <int KC>
static size_t m2l2d_bf16_lds(int mb) {
  switch (mb) {
    case 1: return BfHalo<1, KC>::bytes();
    case 2: return BfHalo<2, KC>::bytes();
    case 3: return BfHalo<3, KC>::bytes();
    case 4: return BfHalo<4, KC>::bytes();
    default: return BfHalo<8, KC>::bytes();
  }
}

static size_t m2l2d_bf16_lds_kc(int kc, int mb) {
  return kc == 1 ? m2l2d_bf16_lds<1>(mb) : kc == 2 ? m2l2d_bf16_lds<2>(mb) : m2l2d_bf16_lds<3>(mb);
}

template <typename T, int KS, int NB, int MB, bool FULL>
static void m2l_launch_f(const FmmArgs& a, const M2lTiles& tt, const M2lLayout& ly,
                         hipStream_t st) {
  const size_t lds = m2l2d_lds(ly, MB, sizeof(T) == 8);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_m2l2d_mfma<T, KS, NB, MB, FULL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_m2l2d_mfma<T, KS, NB, MB, FULL>), dim3(tt.ntiles), dim3(256), lds, st, a,
                     tt, ly);
}

template <typename T, int KS, int NB, int MB>
static void m2l_launch(const FmmArgs& a, const M2lTiles& tt, const M2lLayout& ly,
                       hipStream_t st) {
  if (a.ord_full)
    m2l_launch_f<T, KS, NB, MB, true>(a, tt, ly, st);
  else
    m2l_launch_f<T, KS, NB, MB, false>(a, tt, ly, st);
}

// Tile heights compiled per (precision, bucket): MB = 1 everywhere; 2, 3, 4 and
// 8 where the accumulators, the operator block and the halo still fit (FP64: MB
// 2 up to bucket 20, MB 3 up to bucket 16; MB 8: FP32 up to bucket 16).
template <typename T, int KS, int NB>
static void m2l_mb(const FmmArgs& a, const M2lTiles& tt, const M2lLayout& ly, hipStream_t st) {
  constexpr bool kF64 = sizeof(T) == 8;
  const int mb = a.m2l_mb;
  if (mb == 8 && !kF64 && KS <= 8) {
    m2l_launch<T, KS, NB, ((kF64 || KS > 8) ? 1 : 8)>(a, tt, ly, st);
  } else if (mb == 3 && (!kF64 || KS <= 8)) {
    m2l_launch<T, KS, NB, ((kF64 && KS > 8) ? 1 : 3)>(a, tt, ly, st);
  } else if (mb == 4 && !kF64) {
    m2l_launch<T, KS, NB, (kF64 ? 1 : 4)>(a, tt, ly, st);
  } else if (mb == 2 && (!kF64 || KS <= 10)) {
    m2l_launch<T, KS, NB, ((kF64 && KS > 10) ? 1 : 2)>(a, tt, ly, st);
  } else {
    m2l_launch<T, KS, NB, 1>(a, tt, ly, st);
  }
}

template <int PB, int MB>
static void m2l_bf16_launch(const FmmArgs& a, const M2lTiles& tt, const M2lLayout& ly,
                            hipStream_t st) {
  const size_t lds = BfHalo<MB, bf16_chunks(PB)>::bytes();
  auto kfull = k_m2l2d_bf16<PB, MB, true>;
  auto kpart = k_m2l2d_bf16<PB, MB, false>;
  auto kern = a.ord_full ? kfull : kpart;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(kern, dim3(tt.ntiles), dim3(256), lds, st, a, tt, ly);
}

// BF16 tile heights: MB = 1, 2, 3, 4 and 8 where the BF16 halo fits (MB 8 up
// to two chunks per row).
template <int PB>
static void m2l_bf16_mb(const FmmArgs& a, const M2lTiles& tt, const M2lLayout& ly,
                        hipStream_t st) {
  switch (a.m2l_mb) {
    case 8: m2l_bf16_launch<PB, (bf16_chunks(PB) <= 2 ? 8 : 1)>(a, tt, ly, st); break;
    case 4: m2l_bf16_launch<PB, 4>(a, tt, ly, st); break;
    case 3: m2l_bf16_launch<PB, 3>(a, tt, ly, st); break;
    case 2: m2l_bf16_launch<PB, 2>(a, tt, ly, st); break;
    default: m2l_bf16_launch<PB, 1>(a, tt, ly, st); break;
  }
}

bool m2l2d_variant_ok(int mb, bool fp64, int pb, bool bf16) {
  const M2lLayout ly = m2l2d_layout(pb);
  if (mb != 1 && mb != 2 && mb != 3 && mb != 4 && mb != 8) return false;
  if (bf16) return m2l2d_bf16_lds_kc(ly.kbf / 32, mb) <= 147456;
  if (fp64 && (mb >= 4 || (mb == 2 && ly.kpad / 4 > 10) || (mb == 3 && ly.kpad / 4 > 8)))
    return false;
  if (mb == 8 && ly.kpad / 4 > 8) return false;
  return m2l2d_lds(ly, mb, fp64) <= 147456;  // leave LDS to spare out of 160 KB
}

template <typename T>
static void m2l_dispatch_t(const FmmArgs& a, const M2lTiles& tt, const M2lLayout& ly,
                           hipStream_t st) {
  switch (ly.kpad) {  // kpad = 2 PB, PB the order bucket
    case 16: m2l_mb<T, 4, 1>(a, tt, ly, st); break;
    case 24: m2l_mb<T, 6, 2>(a, tt, ly, st); break;
    case 32: m2l_mb<T, 8, 2>(a, tt, ly, st); break;
    case 40: m2l_mb<T, 10, 3>(a, tt, ly, st); break;
    case 48: m2l_mb<T, 12, 3>(a, tt, ly, st); break;
    default: m2l_mb<T, 15, 4>(a, tt, ly, st); break;
  }
}

static void m2l_dispatch_bf16(const FmmArgs& a, const M2lTiles& tt, const M2lLayout& ly,
                              hipStream_t st) {
  switch (ly.p) {  // the order bucket
    case 8: m2l_bf16_mb<8>(a, tt, ly, st); break;
    case 12: m2l_bf16_mb<12>(a, tt, ly, st); break;
    case 16: m2l_bf16_mb<16>(a, tt, ly, st); break;
    case 20: m2l_bf16_mb<20>(a, tt, ly, st); break;
    case 24: m2l_bf16_mb<24>(a, tt, ly, st); break;
    default: m2l_bf16_mb<30>(a, tt, ly, st); break;
  }
}

// Levels of at most 4 x 4 boxes per system (level 2, kept in FP64 in the FP32
// modes): the contraction on the VALU with one workgroup per target box and one
// thread per (output value, interaction-list source) dot product; the partial
// sums are added over the sources in list order (deterministic).  A single tile
// of the matrix-core kernel would need a 14 x 14 LDS halo for 16 targets and
// would wait for LDS behind the main contraction's workgroups.
constexpr int kSmallMaxOut = 2 * 30 + 1;
__global__ __launch_bounds__(256) void k_m2l2d_small(FmmArgs a, int k, M2lLayout ly) {
  __shared__ double part[27][kSmallMaxOut];
  __shared__ int srcs[27], slots[27];
  __shared__ int nsrc;
  const int n = 1 << k, nt = n * n;
  const uint32_t sys = blockIdx.x / nt;
  const int t = (int)(blockIdx.x - sys * nt);
  const uint32_t sysb = sys << (2 * k);
  const int tx = t % n, ty = t / n;
  const int pk = a.ord[k], pb = ly.p, cs = ly.cs, kpad = ly.kpad, npad = ly.npad;
  const int nout = 2 * pb + 1;  // re / im of l = 1..pb, then Re B_0
  const double* mom = a.mom64 + a.lt.off[k] * cs;
  double* loc = a.loc64 + a.lt.off[k] * cs;
  if (threadIdx.x == 0) {
    // interaction list of (tx, ty) inside the grid, in row-major window order
    const int xlo = (tx & 1) ? -3 : -2, ylo = (ty & 1) ? -3 : -2;
    int c = 0;
    for (int dy = ylo; dy <= ylo + 5; ++dy)
      for (int dx = xlo; dx <= xlo + 5; ++dx) {
        if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
        const int sx = tx + dx, sy = ty + dy;
        if (sx < 0 || sy < 0 || sx >= n || sy >= n) continue;
        srcs[c] = (int)(sysb | spread2(sx) | (spread2(sy) << 1));
        slots[c] = (dx + 3) + 7 * (dy + 3);
        ++c;
      }
    nsrc = c;
  }
  __syncthreads();
  const int ns = nsrc;
  for (int e = threadIdx.x; e < ns * nout; e += blockDim.x) {
    const int si = e / nout, j = e - (e / nout) * nout;
    const bool b0 = j == 2 * pb;
    double acc = 0.0;
    if (b0 || j < 2 * pk) {
      const double* src = mom + (int64_t)srcs[si] * cs;
      const double* W = a.op64 + (size_t)slots[si] * ly.stride;
      const double* c0 = W + npad * kpad;
      const double* r0 = c0 + npad;
      const double* wr = b0 ? r0 : W + (size_t)j * kpad;
      double s0 = 0.0, s1 = 0.0;
      int kk = 0;
      for (; kk + 1 < 2 * pk; kk += 2) {
        s0 += wr[kk] * src[kk];
        s1 += wr[kk + 1] * src[kk + 1];
      }
      if (kk < 2 * pk) s0 += wr[kk] * src[kk];
      acc = (s0 + s1) + (b0 ? r0[kpad] : c0[j]) * src[2 * pb];
    }
    part[si][j] = acc;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nout; j += blockDim.x) {
    double acc = 0.0, a0s = 0.0;
    for (int si = 0; si < ns; ++si) {
      acc += part[si][j];
      if (j == 2 * pb) a0s += mom[(int64_t)srcs[si] * cs + 2 * pb];
    }
    double* dst = loc + (int64_t)(sysb | spread2(tx) | (spread2(ty) << 1)) * cs;
    if (j == 2 * pb) {
      dst[2 * pb] = acc + a.lt.log_s[k] * a0s;
      dst[2 * pb + 1] = 0.0;  // Im B_0 enters neither the potential nor the field
    } else {
      dst[j] = acc;  // zero above the level's order
    }
  }
}

void launch_m2l2d(const FmmArgs& a, bool fp64, hipStream_t st, bool bf16) {
  if (a.khi < a.klo) return;
  if (fp64 && a.khi <= 2) {
    const M2lLayout ly = m2l2d_layout(order_bucket(a.p));
    for (int k = a.klo; k <= a.khi; ++k)
      hipLaunchKernelGGL(k_m2l2d_small, dim3((unsigned)(a.lt.nsys << (2 * k))), dim3(256), 0, st,
                         a, k, ly);
    return;
  }
  const M2lLayout ly = m2l2d_layout(order_bucket(a.p));
  FmmArgs b = a;
  if (!m2l2d_variant_ok(b.m2l_mb, fp64, ly.p, bf16 && !fp64)) b.m2l_mb = 1;
  const int mb = b.m2l_mb;
  M2lTiles tt{};
  tt.klo = a.klo;
  tt.khi = a.khi;
  tt.remap = a.m2l_remap;
  int64_t t = 0;
  for (int k = a.klo; k <= a.khi; ++k) {
    tt.off[k] = t;
    const int64_t n = (int64_t)1 << k;
    t += ((n + 7) / 8) * ((n + 8 * mb - 1) / (8 * mb)) * a.lt.nsys;
  }
  tt.off[a.khi + 1] = t;
  tt.ntiles = t;
  if (fp64)
    m2l_dispatch_t<double>(b, tt, ly, st);
  else if (bf16)
    m2l_dispatch_bf16(b, tt, ly, st);
  else
    m2l_dispatch_t<float>(b, tt, ly, st);
}

}  // namespace sffmm
