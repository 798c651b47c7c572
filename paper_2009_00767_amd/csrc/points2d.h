// points2d.h -- the 2D log kernel with the paper's fixed point-charge box
// vectors (Appendix STEP1-STEP3 in the square box): n points per axis at
// a_i s / 5 from the box centre (node set 1: the paper's (-2, -1, 1, 2), n =
// 4; node set 2: the n = 2..8 Chebyshev points of the first kind,
// 2.5 cos((2i + 1) pi / (2n)) ascending), d = n^2 per box, point i + n j
// (x offset index i, y index j).  The sort and the near field are the 2D
// kernel's.
#ifndef SFFMM_POINTS2D_H
#define SFFMM_POINTS2D_H

#include "fmm_internal.h"
#include "lagrange.h"

namespace sffmm {

constexpr int kPoints2DMaxN = kPointsMaxN;  // points per axis at most

// Values per box row: d padded to a multiple of 16 (the matrix-core K and N).
int points2d_row(int n);

// Box rows of points2d_row(n) values; the lane-major operator pack of level k
// and offset slot (dx + 3) + 7 (dy + 3) starts at ((k * 49) + slot) * DP^2, so
// lstride is DP^2 (L + 1) values per slot (levels 0..L).
M2lLayout points2d_layout(int n, int L);

// Unit-side operators G0_o[i][j] = log |(a_i - a_j) / 5 - o| (target point i,
// source point j of the box at offset o = source - target, in units of the
// box side), [49 slots][DP][DP] row-major; the adjacent offsets (|o| <= 1) and
// the padding hold zeros.
void build_points2d_operators(int node_set, int n, double* out);

// Lane-major packs for the matrix-core contraction, per level k = 0..L and
// slot: value [nb][s][l] (KS = DP / 4 steps s, lane l: output point
// 16 nb + l % 16, source point (l / 16) KS + s) is G0_o + log s_k (s_k =
// lt.s[k]) for real points, zero in the padding.
void build_points2d_lane_pack(int node_set, int n, const LevelTable& lt, double* out);

// The three far-field passes for levels a.klo..a.khi (a.basis: the node set,
// a.p: the points per axis).  P2M: leaf_local selects the FP32 leaf-local
// records as inputs, fp64 the storage of the level range.  L2P: every level
// kmin..L, near field added, outputs scattered to input order.
void launch_p2m2d_points(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st);
void launch_m2l2d_points(const FmmArgs& a, bool fp64, hipStream_t st);
void launch_l2p2d_points(const FmmArgs& a, bool leaf_local, hipStream_t st);

}  // namespace sffmm

#endif
