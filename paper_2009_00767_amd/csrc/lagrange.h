// lagrange.h -- node sets and Lagrange weights of the fixed point-charge box
// vectors (Appendix STEP1-STEP2; Discussion (1) and (4)): n points per axis at
// a_i s / 5 from the box centre, shared by the 2D and 3D point-charge passes.
//   node set 1: the paper's (-2, -1, 1, 2), n = 4;
//   node set 2: the n Chebyshev points of the first kind of the box,
//     a_i = -2.5 cos((2i + 1) pi / (2n)), ascending.
// A charge at w = (r - r_b) / s goes to the points with the weights
//   f_i(u) = c_i prod_{m != i} (u - a_m),  c_i = 1 / prod_{m != i} (a_i - a_m),
// u = 5 w, one factor per axis.
#ifndef SFFMM_LAGRANGE_H
#define SFFMM_LAGRANGE_H

#include <cmath>

#include "fmm_internal.h"

namespace sffmm {

constexpr int kPointsMaxN = 8;  // points per axis at most

// The node offsets a_0 < ... < a_{n-1} (units of s / 5) of node set `node_set`
// with n points per axis; false when that set has no such n.
inline bool point_nodes(int node_set, int n, double* a) {
  if (node_set == 1) {
    if (n != 4) return false;
    for (int i = 0; i < 4; ++i) a[i] = point_node(1, i);
    return true;
  }
  if (node_set != 2 || n < 2 || n > kPointsMaxN) return false;
  for (int i = 0; i < n; ++i) a[i] = -2.5 * std::cos((2.0 * i + 1.0) * M_PI / (2.0 * n));
  return true;
}

// The node set of a launch (a kernel argument): offsets a_i and the inverse
// denominators c_i of the weights.
struct PtsNodes {
  double a[kPointsMaxN];
  double c[kPointsMaxN];
};

inline PtsNodes make_nodes(int node_set, int n) {
  PtsNodes nd{};
  (void)point_nodes(node_set, n, nd.a);
  for (int i = 0; i < n; ++i) {
    double den = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != i) den *= nd.a[i] - nd.a[m];
    nd.c[i] = 1.0 / den;
  }
  return nd;
}

// f_i(u) for the N nodes (u = 5 w)
template <int N, typename T>
__device__ __forceinline__ void lagn(const PtsNodes& nd, T w, T (&f)[N]) {
  const T u = (T)5 * w;
  T dv[N];
#pragma unroll
  for (int m = 0; m < N; ++m) dv[m] = u - (T)nd.a[m];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T v = (T)nd.c[i];
#pragma unroll
    for (int m = 0; m < N; ++m)
      if (m != i) v *= dv[m];
    f[i] = v;
  }
}

// f_i(u) and df_i / du: the product and its derivative built one factor at a
// time, (v, v') <- (v (u - a_m), v' (u - a_m) + v)
template <int N, typename T>
__device__ __forceinline__ void lagnd(const PtsNodes& nd, T w, T (&f)[N], T (&df)[N]) {
  const T u = (T)5 * w;
  T dv[N];
#pragma unroll
  for (int m = 0; m < N; ++m) dv[m] = u - (T)nd.a[m];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T v = (T)nd.c[i], dd = (T)0;
#pragma unroll
    for (int m = 0; m < N; ++m)
      if (m != i) {
        dd = dd * dv[m] + v;
        v *= dv[m];
      }
    f[i] = v;
    df[i] = dd;
  }
}

}  // namespace sffmm

#endif
