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
constexpr int kMaxOrder3D = 8;
constexpr int kRadixTile = 2048;      // keys per workgroup in a radix pass (256 threads x 8)
constexpr int kLearnedMaxOrder = 24;  // the learned order picks p in 4..24

// Per-level geometry handed to the kernels by value.
struct LevelTable {
  int32_t L;     // finest level
  int32_t kmin;  // coarsest level with an interaction list (2)
  int32_t split; // first level whose coefficients are stored in FP32 (L + 1: none)
  int32_t nsys;  // independent systems of this depth stacked side by side (1: one system);
                 // leaf keys are (system << 2L) | Morton(leaf), level-k boxes (system << 2k) | Morton
  // first box of level k inside its coefficient array (the FP64 array for
  // k < split, the FP32 array for k >= split)
  int64_t off[kMaxLevels2D + 2];
  double side;                     // box side S
  double origin[3];
  double s[kMaxLevels2D + 1];      // side of a level-k box, S / 2^k (exact in binary)
  double inv_s[kMaxLevels2D + 1];  // 2^k / S
  double log_s[kMaxLevels2D + 1];  // log(S / 2^k) (2D multipole-to-local constant)
  double leaf_scale;               // 2^L / S, the leaf-coordinate factor
};

// Level table of a tree of depth L made of nsys stacked systems: levels below
// `split` (3 in the FP32 modes, L + 1 in FP64) in the FP64 coefficient array,
// the others in the FP32 one; *nbox64 / *nbox32 receive the boxes of each.
LevelTable level_table(int dim, bool f32, double side, const double* origin, int L, int nsys,
                       int64_t* nbox64, int64_t* nbox32);

// Point-charge node sets (Appendix STEP1; any distinct positions serve, and
// Discussion (1) names Chebyshev interpolation): the offsets of the four
// points per axis from the box centre, in units of s / 5.  Set 1: the paper's
// (-2, -1, 1, 2).  Set 2: the Chebyshev points of the first kind on the box,
// 2.5 cos((2i + 1) pi / 8).
__host__ __device__ constexpr double point_node(int set, int i) {
  return set == 2 ? (i == 0 ? -2.309698831278217 : i == 1 ? -0.9567085809127246
                     : i == 2 ? 0.9567085809127246 : 2.309698831278217)
                  : (i == 0 ? -2.0 : i == 1 ? -1.0 : i == 2 ? 1.0 : 2.0);
}
// 1 / prod_{k != i} (a_i - a_k): the denominator of the Lagrange weight f_i.
__host__ __device__ constexpr double point_node_inv_den(int set, int i) {
  double den = 1.0;
  for (int k = 0; k < 4; ++k)
    if (k != i) den *= point_node(set, i) - point_node(set, k);
  return 1.0 / den;
}

// Layout of the 2D multipole-to-local operator pack and of a box's coefficients.
struct M2lLayout {
  int p;
  int kpad;    // 2p rounded up to a multiple of 4 (MFMA K)
  int npad;    // 2p rounded up to a multiple of 16 (MFMA N)
  int stride;  // values per offset slot in the operator pack
  int cs;      // values per box: 2p + 2 rounded up to a multiple of 4
  int kbf;     // 2D BF16 products: 6 + 2p inputs padded to a multiple of 32
  int nbf;     // 2D BF16 products: 1 + 2p outputs padded to a multiple of 16
  int lstride; // 2D lane-major pack: values per offset slot (see operators.cpp)
  int l16;     // 2D lane-major BF16 pack: values per offset slot
  int nr;      // 3D: values per box vector (the last one is the degree-0 term)
};

// Caller buffers of a batched evaluation.  The kernels of its captured graph
// that touch them read the addresses from this device record, which a
// one-thread kernel rewrites before every replay, so a replay takes new buffer
// addresses without a new graph.
struct BatchIo {
  const double* pos;
  const double* q;
  double* pot;
  double* field;
};

// ----- sort.hip -----
// keys/vals for n particles (n > 0): Morton key of the leaf, identity values;
// out-of-domain / NaN positions set flag[0] = tag (the evaluation's tag, so
// that no kernel has to clear the flag before an evaluation).
// Also writes the per-tile histogram of the first radix digit into hist and,
// if rec is not NULL, the FP32 leaf-local record (x, y[, z], q) of every
// particle in input order.
void launch_bin(int dim, const double* pos, int64_t n, const LevelTable& lt, uint32_t* keys,
                int32_t* vals, int32_t* flag, int32_t tag, int32_t* hist, hipStream_t st,
                const double* q = nullptr, float4* rec = nullptr, int hist_shift = 0);
// Stable LSD radix sort of (keys, vals) by the low `bits` bits; returns which
// buffer pair holds the result (0: keys/vals, 1: keys_alt/vals_alt).
// hist: radix_hist_entries(maxn) ints (per-tile digit counts); tot: 256 ints.
// first_hist_done: hist already holds the first pass's tile histograms.
// recs / recs_alt (optional): per-particle records moved with the keys; the
// sorted records end in the buffer of the returned parity.
int radix_sort(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n,
               int bits, int32_t* hist, int32_t* tot, hipStream_t st,
               bool first_hist_done = false, float4* recs = nullptr, float4* recs_alt = nullptr);
size_t radix_hist_entries(int64_t maxn);
// Keys of 9..16 bits whose mean high-digit bucket fits the LDS stage: a first
// pass by the high digit key >> 8 (its tile histograms in hist, from
// launch_bin with hist_shift = 8), then a stable sort of each bucket by the low 8 bits
// that also writes leaf_start[0..nleaf] (single system, nleaf = 2^bits).  The
// result is in keys / vals / recs, the same order as radix_sort's.
// parts: radix_two_digit_parts() ints of scratch (digit counts of the parts of
// buckets beyond the LDS stage).
bool radix_two_digit(int64_t n, int bits);
size_t radix_two_digit_parts();
void radix_sort_two_digit(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                          int64_t n, int bits, int32_t* hist, int32_t* tot, int32_t* leaf_start,
                          int64_t nleaf, int32_t* parts, hipStream_t st, float4* recs,
                          float4* recs_alt);
// leaf_start[l] = first sorted position with key >= l, l in [0, nleaf].
void launch_leaf_bounds(const uint32_t* sorted_keys, int64_t n, int64_t nleaf, int32_t* leaf_start,
                        hipStream_t st);
// Gathers sorted FP64 SoA coordinates and charges.
// io (optional): take pos and q from the batched evaluation's record instead.
void launch_gather_f64(int dim, const double* pos, const double* q, const int32_t* perm, int64_t n,
                       double* xs, double* ys, double* zs, double* qs, hipStream_t st,
                       const BatchIo* io = nullptr);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
// Batched 2D: keys (rank << 2 lmax) | Morton scaled to lmax, see sort.hip; also
// the first radix digit's tile histograms into hist (as launch_bin).
// io (optional): take pos and q from the batched evaluation's record instead.
void launch_bin_batched(const double* pos, int64_t n, const int64_t* sys_off, int nsys,
                        const int32_t* info, const LevelTable& lt, int lmax, uint32_t* keys,
                        int32_t* vals, int32_t* flag, int32_t tag, int32_t* hist,
                        hipStream_t st, const double* q = nullptr, float4* rec = nullptr,
                        const BatchIo* io = nullptr);
void launch_rekey(uint32_t* keys, int64_t n, int r0, int L, int lmax, hipStream_t st);

// ----- fmm2d.hip / m2l2d.hip -----
struct FmmArgs {
  LevelTable lt;
  int p;        // order (3D; 2D: the largest order, which fixes the layout bucket)
  int basis;    // 3D: 0 solid harmonics, else fixed point charges (4 x 4 x 4 per box) of
                // node set `basis` (1 the paper's, 2 Chebyshev points)
  const int32_t* ord;  // 2D: device [levels + 1], the order of each level's expansions
  int ord_full;        // 2D: every level's order equals the layout bucket (host-known)
  int m2l_mb;          // 2D M2L tile: 8 x (8 m2l_mb) targets per workgroup (1, 2, 4, 8)
  int m2l_remap;       // 2D M2L: deal tiles to the XCDs in contiguous ranges
  int cs;       // coefficient stride (values per box)
  int klo, khi; // levels handled by one launch
  int64_t n;
  const uint32_t* keys;  // sorted leaf keys
  const int32_t* leaf_start;
  const int32_t* perm;
  const double* xs;      // FP64 mode: sorted absolute coordinates and charges
  const double* ys;
  const double* zs;
  const double* qs;
  const float4* pts;     // FP32 mode: sorted leaf-local (x, y, q, 0) / (x, y, z, q)
  double* mom64;         // levels < split
  double* loc64;
  float* mom32;          // levels >= split
  float* loc32;
  double* part64;        // P2M slice partials
  float* part32;
  const double* op64;    // operator packs [49][stride]
  const float* op32;
  const double* opl64;   // lane-major packs [49 (2D) or 343 (3D)][lstride]
  const float* opl32;
  const __bf16* op16;    // 2D lane-major BF16 dense blocks [49][l16]
  double* near_pot;      // near field in sorted order (P2P -> L2P combine)
  double* near_ex;
  double* near_ey;
  double* near_ez;
  double* m2l_part;      // 3D M2L: partial sums of the split small levels (m2l3d_partial_entries)
  uint8_t* p2p_over;     // 2D FP32 near field: per 4 x 4-leaf tile, halo too large to stage
  double* pot;           // caller output (input order)
  double* field;         // caller output or NULL
  const BatchIo* io;     // batched graphs: the outputs come from this record instead
  // Adaptive depth (2D, one system, depth != NULL): a particle's tree goes
  // deeper while the 3 x 3 boxes around its box hold more than adapt_near
  // particles, down to lt.L.
  int64_t adapt_near;
  const uint8_t* depth;  // depth of every sorted particle (NULL: uniform)
  // adapt_open[adapt_open_off(k) + b], levels kmin..L - 1, Morton order: bit 0
  // (open) the trees of the particles of level-k box b go below level k (the
  // 3 x 3 boxes around it hold more than adapt_near particles and k < L); bit 1
  // some box of the 3 x 3 around b is open
  const uint8_t* adapt_open;
};
__host__ __device__ constexpr int64_t adapt_open_off(int k) { return (((int64_t)1 << (2 * k)) - 1) / 3; }
// P2M for levels a.klo..a.khi; leaf_local selects the FP32 leaf-local inputs,
// fp64 the storage of that level range.
void launch_p2m2d(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st);
// partial rows for nsys stacked systems totalling at most maxn particles
size_t p2m2d_partial_entries(const LevelTable& lt, int klo, int khi, int64_t maxn, int cs);
// M2L (MFMA) for levels a.klo..a.khi in FP64, FP32 or (FP32 with) BF16 inputs.
void launch_m2l2d(const FmmArgs& a, bool fp64, hipStream_t st, bool bf16 = false);
// Whether tile height mb is compiled and fits the LDS for this precision and bucket.
bool m2l2d_variant_ok(int mb, bool fp64, int pb, bool bf16);
void launch_l2p2d(const FmmArgs& a, bool leaf_local, hipStream_t st);
void launch_p2p2d(const FmmArgs& a, bool leaf_local, hipStream_t st);
// Adaptive depth: the open flags of levels kmin..L - 1 (one launch per level,
// coarse to fine), then every sorted particle's depth.
void launch_adapt_depth(const FmmArgs& a, uint8_t* open, uint8_t* depth, hipStream_t st);

// ----- fmm3d.hip / m2l3d.hip (same argument block, 3D layouts) -----
void launch_p2m3d(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st);
size_t p2m3d_partial_entries(int klo, int khi, int64_t maxn, int cs);
// 3D M2L; a.m2l_mb: 4 a.m2l_mb layers of 16 targets per workgroup.
void launch_m2l3d(const FmmArgs& a, bool fp64, hipStream_t st);
bool m2l3d_variant_ok(int mb, bool fp64);
// Levels 2..kM2l3SplitLevel (8 tiles each) run their 189 offsets as kM2l3Split
// chunks on as many workgroups; partial rows for the 64 + 512 boxes of those levels.
constexpr int kM2l3Split = 27, kM2l3SplitLevel = 3, kM2l3SplitBoxes = 64 + 512;
inline size_t m2l3d_partial_entries(int cs) { return (size_t)kM2l3Split * kM2l3SplitBoxes * cs; }
void launch_l2p3d(const FmmArgs& a, bool leaf_local, hipStream_t st);
void launch_p2p3d(const FmmArgs& a, bool leaf_local, hipStream_t st);

// ----- rootframe.hip (point charges in the root frame, FP64) -----
// rv: [boxes of levels 2..L][64] FP64, level k at lt.off[k] (the FP64 plan's
// offsets).  Upward: U-bar-1 and U-bar-2 into rv, then each box's own charges
// M_m v_m into the moment rows (levels a.klo..a.khi); downward: the
// contraction's locals back to root-frame linear forms in rv, then the
// parent-to-child additions; eval: F(v) at every particle plus the near field,
// scattered to input order.
void launch_root_upward(const FmmArgs& a, double* rv, hipStream_t st);
void launch_root_downward(const FmmArgs& a, double* rv, hipStream_t st);
void launch_root_eval(const FmmArgs& a, const double* rv, hipStream_t st);

// ----- order.hip (learned order, 2D) -----
// One system of an evaluation as seen by the order selection: its sorted range,
// depth, depth-group row of the order table, its chunk blocks and its index.
struct OrderSys {
  int32_t start, n, L, group, blk0, nblk, id, pad;
};
int order_chunk();  // sorted positions per partial block
// keys: sorted keys whose level-k box is key >> 2 (kbits - k); q in input order
// (read through perm).  Raises ord[group * ord_cols + k] to the chosen order
// (the rows must be cleared first); feat_out (optional) [id][13][3].
// io (optional): take q from the batched evaluation's record instead.
void launch_order_select(const OrderSys* sys, int nsys, int total_blocks, const uint32_t* keys,
                         const int32_t* perm, const double* q, int kbits, const float* w,
                         double* pq, int32_t* pcnt, float log10_budget, int32_t* ord, int ord_cols,
                         float* feat_out, hipStream_t st, const BatchIo* io = nullptr);
// Writes one order-selection record to device memory from a kernel argument
// (no host staging buffer).
void launch_set_ordsys(OrderSys* dst, const OrderSys& v, hipStream_t st);
// Batched evaluations: writes the caller's buffer addresses into *io and checks
// the caller's device system tables against the prepared ones (offsets [nsys +
// 1]; depths, or the default depth rule when levels is NULL): flag[2] = tag on
// any difference, else 0.  One workgroup.
void launch_batch_begin(BatchIo* io, const double* pos, const double* q, double* pot,
                        double* field, const int64_t* off, const int32_t* levels,
                        const int64_t* prep_off, const int32_t* prep_info, int nsys, int lmax,
                        int32_t* flag, int32_t tag, hipStream_t st);
int64_t mlp_grad_waves(int64_t m);
void launch_mlp_forward(const float* w, const float* x, int64_t m, float* y, hipStream_t st);
// part: [round_up(mlp_grad_waves(m), 4)][FMM_MLP_NPARAM], part_loss the same count
void launch_mlp_grad(const float* w, const float* x, const float* t, int64_t m, float* part,
                     double* part_loss, float* grad, float* loss, hipStream_t st);
void launch_mlp_adam(float* w, const float* g, float* m1, float* m2, int step, float lr,
                     hipStream_t st);
// Relative L2 difference of pot against ref over every particle of each of
// nsys systems (device offsets sys_off [nsys + 1] into the concatenated
// arrays; NULL: one system of n) into err_out[1 + s], the largest into
// err_out[0]; any above tol (or NaN): flag[1] = tag and ref copied into pot /
// field.  err_out holds nsys + 1 values.
void launch_judge(double* pot, double* field, const double* rpot, const double* rfield, int64_t n,
                  int dim, const int64_t* sys_off, int nsys, double tol, int32_t* flag,
                  int32_t tag, double* err_out, hipStream_t st);

// Kernels are instantiated for a few order buckets; an order p runs with the
// layout of its bucket (coefficients above p are zero).
__host__ __device__ inline int order_bucket(int p) {
  return p <= 8 ? 8 : p <= 12 ? 12 : p <= 16 ? 16 : p <= 20 ? 20 : p <= 24 ? 24 : 30;
}

// 2D BF16 products of order bucket pb: chunks of 32 K positions, enough for
// the 6 A_0 slots, the 2 pb input values and the two-term splits of at least
// the leading 4 coefficients (4 K positions each); ms, the number of leading
// coefficients (re/im of 1..ms) whose splits fill the chunks.
__host__ __device__ constexpr int bf16_chunks(int pb) {
  return (6 + 2 * pb + 4 * (pb < 4 ? pb : 4) + 31) / 32;
}
__host__ __device__ constexpr int bf16_split(int pb) {
  return (32 * bf16_chunks(pb) - 6 - 2 * pb) / 4 < pb ? (32 * bf16_chunks(pb) - 6 - 2 * pb) / 4
                                                     : pb;
}

// ----- operators.cpp -----
// Layout for order bucket pb.
M2lLayout m2l2d_layout(int pb);
// 2D operator pack of order p in FP64, [49][ly.stride] (see operators.cpp).
void build_m2l2d_operators(int p, const M2lLayout& ly, double* out);
// Lane-major 2D packs for the matrix-core kernel, from the FP64 pack: per slot
// the B operand of every MFMA step in the order the 64 lanes hold it (see
// operators.cpp); the BF16 one rounded once from the FP64 values (through FP32).
void build_m2l2d_lane_pack(const M2lLayout& ly, const double* pack, double* out);
void build_m2l2d_bf16(const M2lLayout& ly, const double* pack, uint16_t* out);
// 3D: layout for order bucket pb and operator pack [343][ly.stride].
M2lLayout m2l3d_layout(int pb);
void build_m2l3d_operators(int p, const M2lLayout& ly, double* out);
void build_m2l3d_lane_pack(const M2lLayout& ly, const double* pack, double* out);
// 3D fixed point-charge basis: the layout (64 point charges and an unused,
// always-zero degree-0 slot, so that the 3D matrix-core kernel runs it as is)
// and its operator pack [343][ly.stride] in the same format.
M2lLayout points3d_layout();
void build_points3d_operators(const M2lLayout& ly, int node_set, double* out);
__host__ __device__ inline int order_bucket3(int p) { return p <= 4 ? 4 : p <= 8 ? 8 : 12; }

}  // namespace sffmm
