// points2d.h -- the 2D log kernel with the paper's fixed point-charge box
// vectors (Appendix STEP1-STEP3 in the square box): 4 x 4 points per box at
// a_i s / 5 from its centre, a_i from point_node (node set 1: the paper's
// (-2, -1, 1, 2); 2: the Chebyshev points), point i + 4 j (x offset index i,
// y index j).  The sort and the near field are the 2D kernel's.
#ifndef SFFMM_POINTS2D_H
#define SFFMM_POINTS2D_H

#include "fmm_internal.h"

namespace sffmm {

constexpr int kPoints2D = 16;  // point charges per box

// Box rows of 16 values; the lane-major operator pack of level k and offset
// slot (dx + 3) + 7 (dy + 3) starts at ((k * 49) + slot) * 256, so lstride is
// 256 (L + 1) values per slot (levels 0..L).
M2lLayout points2d_layout(int L);

// Unit-side operators G0_o[i][j] = log |(a_i - a_j) / 5 - o| (target point i,
// source point j of the box at offset o = source - target, in units of the
// box side), [49 slots][16 * 16] row-major; the adjacent offsets (|o| <= 1)
// hold zeros.
void build_points2d_operators(int node_set, double* out);

// Lane-major packs for the matrix-core contraction, per level k = 0..L and
// slot: value [s][l] (s < 4, lane l: output point i = l % 16, source point
// 4 (l / 16) + s) is G0_o[i][4 (l / 16) + s] + log s_k (s_k = lt.s[k]).
void build_points2d_lane_pack(int node_set, const LevelTable& lt, double* out);

// The three far-field passes for levels a.klo..a.khi (a.basis: the node set).
// P2M: leaf_local selects the FP32 leaf-local records as inputs, fp64 the
// storage of the level range.  L2P: every level kmin..L, near field added,
// outputs scattered to input order.
void launch_p2m2d_points(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st);
void launch_m2l2d_points(const FmmArgs& a, bool fp64, hipStream_t st);
void launch_l2p2d_points(const FmmArgs& a, bool leaf_local, hipStream_t st);

}  // namespace sffmm

#endif
