// points3d.h -- the 3D 1/r kernel with n x n x n fixed point charges per box
// for n other than 4 (Appendix STEP1-STEP3 with d = n^3; Discussion (4): d is
// a free parameter), at the n Chebyshev points of the first kind per axis
// (Discussion (1)); point i + n j + n^2 l at offsets (a_i, a_j, a_l) s / 5.
// The n = 4 sets run in the shared 3D passes of fmm3d.hip; the sort, the near
// field and the contraction (m2l3d.hip) are the 3D kernel's.
#ifndef SFFMM_POINTS3D_H
#define SFFMM_POINTS3D_H

#include "fmm_internal.h"
#include "lagrange.h"

namespace sffmm {

constexpr int kPoints3DMaxN = 5;  // points per axis at most (d = 125)

// Layout of a box row and of the contraction's operator pack: d = n^3 values
// padded to K = N = 64 for n <= 4 (the n = 4 layout) and to 128 for n = 5;
// the degree-0 slot of the harmonic format (index nr - 1) stays zero.
M2lLayout points3d_layout_n(int n);

// Operators of node set `node_set` with n points per axis in the harmonic
// pack format [343][ly.stride]: W_o[t][s] = 1 / |o + y_s - y_t| (unit box
// side, o the offset in box sides, y the point offsets) for real points t, s
// of non-adjacent offsets, zero elsewhere.
void build_points3d_operators_n(const M2lLayout& ly, int node_set, int n, double* out);

// P2M and L2P of the point charges for n in {2, 3, 5} (a.p; a.basis the node
// set).  P2M: leaf_local selects the FP32 leaf-local records as inputs, fp64
// the storage of the level range.  L2P: every level kmin..L, near field
// added, outputs scattered to input order.
void launch_p2m3d_points(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st);
void launch_l2p3d_points(const FmmArgs& a, bool leaf_local, hipStream_t st);

}  // namespace sffmm

#endif
