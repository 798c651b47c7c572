// fmm_internal.h -- plan layout and kernel launchers shared by the host API and
// the HIP kernels of the shift-free FMM library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fmm.h"

namespace sffmm {

constexpr int kMaxLevels2D = 12;
constexpr int kMaxLevels3D = 8;
constexpr int kMaxOrder2D = 30;
constexpr int kMaxOrder3D = 12;
constexpr int kRadixTile = 2048;  // keys per workgroup in a radix pass (256 threads x 8)

// Per-level geometry handed to the kernels by value.
struct LevelTable {
  int32_t L;                 // finest level
  int32_t kmin;              // coarsest level with an interaction list (2)
  int64_t off[kMaxLevels2D + 2];  // first box of level k in the per-level coefficient arrays
  double side;               // box side S
  double origin[3];
  double s[kMaxLevels2D + 1];      // side of a level-k box, S / 2^k (exact in binary)
  double inv_s[kMaxLevels2D + 1];  // 2^k / S
  double log_s[kMaxLevels2D + 1];  // log(S / 2^k) (2D multipole-to-local constant)
  double leaf_scale;         // 2^L / S, the leaf-coordinate factor
};

struct fmm_plan_impl;

// ----- sort.hip -----
// keys/vals for n particles (n > 0): Morton key of the leaf, identity values;
// flags out-of-domain / NaN positions in *flag (bit 0).
void launch_bin(int dim, const double* pos, int64_t n, const LevelTable& lt, uint32_t* keys,
                int32_t* vals, int32_t* flag, hipStream_t st);
// Stable LSD radix sort of (keys, vals) by the low `bits` bits; returns which
// buffer pair holds the result (0: keys/vals, 1: keys_alt/vals_alt).
int radix_sort(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n,
               int bits, int32_t* hist, int32_t* scan_tmp, hipStream_t st);
size_t radix_hist_entries(int64_t maxn);
size_t scan_tmp_entries(int64_t count);
// leaf_start[l] = first sorted position with key >= l, l in [0, nleaf].
void launch_leaf_bounds(const uint32_t* sorted_keys, int64_t n, int64_t nleaf, int32_t* leaf_start,
                        hipStream_t st);
// Gathers sorted FP64 SoA coordinates and charges.
void launch_gather_f64(int dim, const double* pos, const double* q, const int32_t* perm, int64_t n,
                       double* xs, double* ys, double* zs, double* qs, hipStream_t st);
// Gathers FP32 leaf-local coordinates (x - leaf centre) and charges as float4.
void launch_gather_f32(int dim, const double* pos, const double* q, const int32_t* perm,
                       const uint32_t* sorted_keys, int64_t n, const LevelTable& lt,
                       float4* pts, hipStream_t st);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);

// ----- fmm2d.hip -----
struct Fmm2dArgs {
  LevelTable lt;
  int p;             // order
  int cs;            // coefficient stride (reals per box)
  int64_t n;
  int64_t nbox_total;  // boxes over levels kmin..L
  const uint32_t* keys;     // sorted leaf keys
  const int32_t* leaf_start;
  const int32_t* perm;
  const double* xs;
  const double* ys;
  const double* qs;
  double* mom;       // [nbox_total][cs]
  double* loc;       // [nbox_total][cs]
  double* partial;   // P2M slice partials
  const double* op;  // [49][P][P][2] complex operators by offset slot (dx+3) + 7 (dy+3)
  double* far_pot;
  double* far_ex;
  double* far_ey;
  double* pot;       // caller output (input order)
  double* field;     // caller output or NULL
};
void launch_p2m2d_f64(const Fmm2dArgs& a, hipStream_t st);
void launch_m2l2d_f64(const Fmm2dArgs& a, hipStream_t st);
void launch_l2p2d_f64(const Fmm2dArgs& a, hipStream_t st);
void launch_p2p2d_f64(const Fmm2dArgs& a, hipStream_t st);
size_t p2m2d_partial_entries(const LevelTable& lt, int cs);

// ----- operators.cpp -----
// 2D multipole-to-local operators in FP64, one complex (p+1)x(p+1) matrix per
// offset slot (dx + 3) + 7 (dy + 3), dx, dy in [-3, 3]; entry [l][m] multiplies
// source coefficient m into target coefficient l (the log s_k term excluded).
void build_m2l2d_operators(int p, double* out /* [49][p+1][p+1][2] */);

}  // namespace sffmm
