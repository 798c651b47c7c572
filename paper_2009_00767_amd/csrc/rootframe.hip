// rootframe.hip -- the point-charge method in the root frame, as Section 2.2.1
// writes its passes with the Appendix's STEP4-STEP5 (FMM_ROOT_FRAME, FP64).
//
// Every box vector is a vector of the root box's 64 point charges: a particle
// c maps to v = q h_{m^0}(c), the same for every box containing it (the Note
// closing Section 2.2.2), so
//   U-bar-1  finest boxes:  v_m = sum of the v of its particles   (k_root_leaf)
//   U-bar-2  coarser boxes: v_m = sum of its 8 children's v        (k_root_up)
// The bilinear form of two boxes of an interaction list is
//   B_{mi,m}(v, v') = b(M_mi v, M_m v'),  M_m = (h_m(p_1) .. h_m(p_64))   (STEP4, STEP5)
// with b the pair sum of point charges.  D-bar-1 forms, per target box, the
// dual vector sum_{mi} M_m^T M_b^T M_mi v_mi: the transfer into each box's own
// frame (k_root_to_box), the box-frame contraction of the point-charge kernel
// (k_m2l3d_mfma, shared with the box-local form) and the transfer back
// (k_root_from_box).  D-bar-2 passes the dual vectors from parent to child by
// addition (k_root_down), and F(v) = L_{m^l}(v) is the dot product of the
// finest box's dual vector with the particle's root-frame weights
// (k_root_eval, with the near field added and the result scattered to input
// order).
//
// The transfers are exact in exact arithmetic (the root weights reproduce
// every cubic, and each h_m is one), but their entries grow about 8-fold per
// axis per level (h_m evaluated at root points far outside m), so rounding
// is amplified: the reason the paper asks for double precision (Discussion
// (3)).  Only FP64 plans take this form.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace sffmm {
namespace {

// 1D Lagrange weights f_a(u) of node set NS (the same formula as the box
// vectors of the point-charge basis use).
template <int NS>
__device__ __forceinline__ double lag1(int a, double u) {
  double num = 1.0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k != a) num *= u - point_node(NS, k);
  return num * point_node_inv_den(NS, a);
}

template <int NS>
__device__ __forceinline__ void lag1x4(double u, double (&f)[4], double (&df)[4]) {
  const double d0 = u - point_node(NS, 0), d1 = u - point_node(NS, 1),
               d2 = u - point_node(NS, 2), d3 = u - point_node(NS, 3);
  const double d23 = d2 * d3, d01 = d0 * d1, d13 = d1 * d3, d12 = d1 * d2, d03 = d0 * d3,
               d02 = d0 * d2;
  f[0] = d1 * d23 * point_node_inv_den(NS, 0);
  f[1] = d0 * d23 * point_node_inv_den(NS, 1);
  f[2] = d01 * d3 * point_node_inv_den(NS, 2);
  f[3] = d01 * d2 * point_node_inv_den(NS, 3);
  df[0] = (d23 + d13 + d12) * point_node_inv_den(NS, 0);
  df[1] = (d23 + d03 + d02) * point_node_inv_den(NS, 1);
  df[2] = (d13 + d03 + d01) * point_node_inv_den(NS, 2);
  df[3] = (d12 + d02 + d01) * point_node_inv_den(NS, 3);
}

// U-bar-1: one wave per finest box; lane l takes the box's particles l,
// l + 64, ... (sorted, FP64) and adds each one's 64 root-frame charges into
// registers (the weights of the box-vector kernels, in the root box's frame);
// the lanes' sums then meet in LDS and are added in lane order.
template <int NS>
__global__ __launch_bounds__(64) void k_root_leaf(FmmArgs a, double* __restrict__ rv) {
  __shared__ double red[64][65];
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const LevelTable& lt = a.lt;
  const double is = 1.0 / lt.side;  // w = (x - C0) / S
  const double cx = lt.origin[0] + 0.5 * lt.side, cy = lt.origin[1] + 0.5 * lt.side,
               cz = lt.origin[2] + 0.5 * lt.side;
  const int32_t i0 = a.leaf_start[b], i1 = a.leaf_start[b + 1];
  double acc[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) acc[i] = 0.0;
  for (int32_t i = i0 + lane; i < i1; i += 64)
    points_accumulate<NS, double>(acc, a.qs[i], (a.xs[i] - cx) * is, (a.ys[i] - cy) * is,
                                  (a.zs[i] - cz) * is);
#pragma unroll
  for (int i = 0; i < 64; ++i) red[lane][i] = acc[i];
  __syncthreads();
  double t = 0.0;
  for (int l = 0; l < 64; ++l) t += red[l][lane];
  rv[(lt.off[lt.L] + b) * 64 + lane] = t;
}

// U-bar-2 at level k: thread per (box, point); the children 8b .. 8b + 7 are
// the box's Morton successors.
__global__ __launch_bounds__(256) void k_root_up(LevelTable lt, int k, double* __restrict__ rv) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = (int64_t)1 << (3 * k);
  if (g >= nb * 64) return;
  const int64_t b = g >> 6;
  const int i = (int)(g & 63);
  const double* ch = rv + (lt.off[k + 1] + 8 * b) * 64 + i;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) acc += ch[64 * c];
  rv[(lt.off[k] + b) * 64 + i] = acc;
}

// The three 4 x 4 factors of M_m for box b of level k: T[d][a][a'] =
// f_a(u), u = 5 (P_a' - c_d) / s_k, P the root nodes along axis d and c the box
// centre.  Threads 0..47 of the block fill it.
template <int NS>
__device__ __forceinline__ void transfer_factors(const LevelTable& lt, int k, int64_t b,
                                                 double (*T)[4][4]) {
  const int t = threadIdx.x;
  if (t < 48) {
    const int d = t >> 4, aa = (t >> 2) & 3, ap = t & 3;
    const uint32_t ub = (uint32_t)b;
    const uint32_t ix = compact3(ub >> d);
    const double c = lt.origin[d] + lt.s[k] * ((double)ix + 0.5);
    const double P = lt.origin[d] + 0.5 * lt.side + point_node(NS, ap) * lt.side / 5.0;
    T[d][aa][ap] = lag1<NS>(aa, 5.0 * (P - c) * lt.inv_s[k]);
  }
}

// D-bar-1, first step: M_m v_m, the box's own 64 point charges, into the
// moment rows the contraction reads (degree-0 slot and padding zero).  One
// 64-thread block per box of the level range.
template <int NS>
__global__ __launch_bounds__(64) void k_root_to_box(FmmArgs a, const double* __restrict__ rv) {
  __shared__ double T[3][4][4];
  __shared__ double v[64];
  const LevelTable& lt = a.lt;
  int64_t gb = blockIdx.x;
  int k = a.klo;
  while (k < a.khi && gb >= ((int64_t)1 << (3 * k))) {
    gb -= (int64_t)1 << (3 * k);
    ++k;
  }
  const int64_t b = gb;
  const int i = threadIdx.x;
  transfer_factors<NS>(lt, k, b, T);
  v[i] = rv[(lt.off[k] + b) * 64 + i];
  __syncthreads();
  const int ia = i & 3, ib = (i >> 2) & 3, ic = i >> 4;
  double acc = 0.0;
  for (int j = 0; j < 64; ++j)
    acc += T[0][ia][j & 3] * T[1][ib][(j >> 2) & 3] * T[2][ic][j >> 4] * v[j];
  double* row = a.mom64 + (lt.off[k] + b) * a.cs;
  row[i] = acc;
  if (i < a.cs - 64) row[64 + i] = 0.0;
}

// D-bar-1, last step: M_m^T y_m / s_k, the box's linear form back in the root
// frame (y_m: the potentials at its points for a unit box side).
template <int NS>
__global__ __launch_bounds__(64) void k_root_from_box(FmmArgs a, double* __restrict__ rv) {
  __shared__ double T[3][4][4];
  __shared__ double y[64];
  const LevelTable& lt = a.lt;
  int64_t gb = blockIdx.x;
  int k = a.klo;
  while (k < a.khi && gb >= ((int64_t)1 << (3 * k))) {
    gb -= (int64_t)1 << (3 * k);
    ++k;
  }
  const int64_t b = gb;
  const int j = threadIdx.x;
  transfer_factors<NS>(lt, k, b, T);
  y[j] = a.loc64[(lt.off[k] + b) * a.cs + j];
  __syncthreads();
  const int ja = j & 3, jb = (j >> 2) & 3, jc = j >> 4;
  double acc = 0.0;
  for (int i = 0; i < 64; ++i)
    acc += T[0][i & 3][ja] * T[1][(i >> 2) & 3][jb] * T[2][i >> 4][jc] * y[i];
  rv[(lt.off[k] + b) * 64 + j] = acc * lt.inv_s[k];
}

// D-bar-2 at level k: L_child = L~_child + L_parent.
__global__ __launch_bounds__(256) void k_root_down(LevelTable lt, int k, double* __restrict__ rv) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = (int64_t)1 << (3 * k);
  if (g >= nb * 64) return;
  const int64_t b = g >> 6;
  const int i = (int)(g & 63);
  rv[(lt.off[k] + b) * 64 + i] += rv[(lt.off[k - 1] + (b >> 3)) * 64 + i];
}

// F(v) = L_{m^l}(v) for a unit probe at each particle: the finest box's dual
// vector against the particle's root weights, minus its gradient for the
// field; near field added; outputs scattered to input order.
template <int NS>
__global__ __launch_bounds__(256) void k_root_eval(FmmArgs a, const double* __restrict__ rv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const LevelTable& lt = a.lt;
  double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
  if (lt.L >= lt.kmin) {
    const double is = 5.0 / lt.side;
    double fx[4], dfx[4], fy[4], dfy[4], fz[4], dfz[4];
    lag1x4<NS>((a.xs[j] - (lt.origin[0] + 0.5 * lt.side)) * is, fx, dfx);
    lag1x4<NS>((a.ys[j] - (lt.origin[1] + 0.5 * lt.side)) * is, fy, dfy);
    lag1x4<NS>((a.zs[j] - (lt.origin[2] + 0.5 * lt.side)) * is, fz, dfz);
    const double* Lr = rv + (lt.off[lt.L] + a.keys[j]) * 64;
    double F = 0, Gx = 0, Gy = 0, Gz = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      double h = 0, hx = 0, hy = 0;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        double g = 0, gd = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double v = Lr[i + 4 * jj + 16 * l];
          g += fx[i] * v;
          gd += dfx[i] * v;
        }
        h += fy[jj] * g;
        hx += fy[jj] * gd;
        hy += dfy[jj] * g;
      }
      F += fz[l] * h;
      Gx += fz[l] * hx;
      Gy += fz[l] * hy;
      Gz += dfz[l] * h;
    }
    phi = F;
    ex = -Gx * is;
    ey = -Gy * is;
    ez = -Gz * is;
  }
  const int64_t o = a.perm[j];
  a.pot[o] = phi + a.near_pot[j];
  if (a.field) {
    a.field[3 * o] = ex + a.near_ex[j];
    a.field[3 * o + 1] = ey + a.near_ey[j];
    a.field[3 * o + 2] = ez + a.near_ez[j];
  }
}

template <int NS>
void upward(const FmmArgs& a, double* rv, hipStream_t st) {
  const LevelTable& lt = a.lt;
  const int64_t nleaf = (int64_t)1 << (3 * lt.L);
  hipLaunchKernelGGL(k_root_leaf<NS>, dim3((unsigned)nleaf), dim3(64), 0, st, a, rv);
  for (int k = lt.L - 1; k >= lt.kmin; --k) {
    const int64_t cnt = ((int64_t)1 << (3 * k)) * 64;
    hipLaunchKernelGGL(k_root_up, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, lt, k,
                       rv);
  }
  int64_t boxes = 0;
  for (int k = a.klo; k <= a.khi; ++k) boxes += (int64_t)1 << (3 * k);
  hipLaunchKernelGGL(k_root_to_box<NS>, dim3((unsigned)boxes), dim3(64), 0, st, a,
                     (const double*)rv);
}

template <int NS>
void downward(const FmmArgs& a, double* rv, hipStream_t st) {
  const LevelTable& lt = a.lt;
  int64_t boxes = 0;
  for (int k = a.klo; k <= a.khi; ++k) boxes += (int64_t)1 << (3 * k);
  hipLaunchKernelGGL(k_root_from_box<NS>, dim3((unsigned)boxes), dim3(64), 0, st, a, rv);
  for (int k = lt.kmin + 1; k <= lt.L; ++k) {
    const int64_t cnt = ((int64_t)1 << (3 * k)) * 64;
    hipLaunchKernelGGL(k_root_down, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, lt, k,
                       rv);
  }
}

}  // namespace

void launch_root_upward(const FmmArgs& a, double* rv, hipStream_t st) {
  if (a.n <= 0 || a.lt.L < a.lt.kmin) return;
  if (a.basis == 2)
    upward<2>(a, rv, st);
  else
    upward<1>(a, rv, st);
}

void launch_root_downward(const FmmArgs& a, double* rv, hipStream_t st) {
  if (a.n <= 0 || a.lt.L < a.lt.kmin) return;
  if (a.basis == 2)
    downward<2>(a, rv, st);
  else
    downward<1>(a, rv, st);
}

void launch_root_eval(const FmmArgs& a, const double* rv, hipStream_t st) {
  if (a.n <= 0) return;
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (a.basis == 2)
    hipLaunchKernelGGL(k_root_eval<2>, grid, dim3(256), 0, st, a, rv);
  else
    hipLaunchKernelGGL(k_root_eval<1>, grid, dim3(256), 0, st, a, rv);
}

}  // namespace sffmm
