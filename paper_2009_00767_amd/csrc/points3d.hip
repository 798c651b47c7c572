// points3d.hip -- particle passes of the 3D 1/r kernel with n x n x n fixed
// point charges per box, n in {2, 3, 5} (layout in points3d.h):
//   P2M (STEP2): a charge q at w = (r - c) / s adds q f_i(5 w_x) f_j(5 w_y)
//     f_l(5 w_z) to point i + n j + n^2 l (f the Lagrange weights of the node
//     set).  One thread range per z-plane l of the points: each thread holds
//     the n^2 charges of its plane, so the registers stay n^2 whatever n.
//   L2P: the potential at r is sum f_i f_j f_l L_{i+nj+n^2l} / s_k over the
//     levels, contracted one axis at a time, the field minus its gradient
//     (d/dx = (5 / s_k) d/du); then the near field is added and the outputs
//     go to input order.
// The contraction of the locals (STEP3) is the 3D matrix-core kernel with
// this layout's operators.
#include <cmath>

#include "device_common.h"
#include "points3d.h"

namespace sffmm {

M2lLayout points3d_layout_n(int n) {
  M2lLayout L = points3d_layout();
  L.p = n;
  if (n <= 4) return L;  // d <= 64: the n = 4 rows, the tail left zero
  L.kpad = 128;
  L.npad = 128;
  L.nr = 126;  // the degree-0 slot (index 125) inside the padding
  L.cs = 128;
  L.stride = L.npad * L.kpad + L.npad + L.kpad + 4;
  L.lstride = 64 * ((L.npad / 16) * (L.kpad / 4 + 1) + L.kpad / 4) + 4;
  return L;
}

void build_points3d_operators_n(const M2lLayout& L, int node_set, int n, double* out) {
  double a[kPointsMaxN];
  for (int i = 0; i < 343 * L.stride; ++i) out[i] = 0.0;
  if (!point_nodes(node_set, n, a)) return;
  for (int i = 0; i < n; ++i) a[i] /= 5.0;  // in units of the box side
  const int d = n * n * n;
  for (int dz = -3; dz <= 3; ++dz)
    for (int dy = -3; dy <= 3; ++dy)
      for (int dx = -3; dx <= 3; ++dx) {
        if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
        double* W = out + (size_t)((dx + 3) + 7 * (dy + 3) + 49 * (dz + 3)) * L.stride;
        for (int t = 0; t < d; ++t)
          for (int s = 0; s < d; ++s) {
            const double rx = dx + a[s % n] - a[t % n];
            const double ry = dy + a[(s / n) % n] - a[(t / n) % n];
            const double rz = dz + a[s / (n * n)] - a[t / (n * n)];
            W[(size_t)t * L.kpad + s] = 1.0 / std::sqrt(rx * rx + ry * ry + rz * rz);
          }
      }
}

namespace {

// P2M over the plan of device_common.h, repeated for each z-plane l of the
// points: thread tg = l thr + t (thr a multiple of 64, so l is uniform over a
// wave and the butterfly lanes of a group stay in one wave).
template <typename T, int N, bool LL>
__global__ __launch_bounds__(256) void k_p2m3d_pts(FmmArgs a, P2mPlan pl, PtsNodes nd,
                                                    int64_t thr) {
  constexpr int P = N * N;  // point charges of one plane
  const int64_t tg = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int l = (int)(tg / thr);
  if (l >= N) return;  // whole waves past the last plane
  const int64_t t = tg - (int64_t)l * thr;
  if ((t & ~(int64_t)63) >= pl.thr_off[pl.khi + 1]) return;
  const LevelTable& lt = a.lt;
  int k = pl.klo;
  while (k < pl.khi && t >= pl.thr_off[k + 1]) ++k;
  const int G = pl.G[k], S = pl.S[k];
  const int64_t local = t - pl.thr_off[k];
  const int64_t nb = (int64_t)1 << (3 * k);
  const int64_t b = local / (G * S);
  const bool valid = b < nb;
  const int rem = (int)(local - b * G * S);
  const int j = rem / G, r = rem - (rem / G) * G;
  const int sh = lt.L - k;
  // the weight of plane l: c_l prod_{m != l} (u - a_m)
  T al[N], cl = (T)0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    al[m] = (T)nd.a[m];
    if (m == l) cl = (T)nd.c[m];
  }
  T acc[P];
#pragma unroll
  for (int i = 0; i < P; ++i) acc[i] = (T)0;
  if (valid) {
    const int64_t s0 = a.leaf_start[b << (3 * sh)], s1 = a.leaf_start[(b + 1) << (3 * sh)];
    const int64_t len = s1 - s0;
    const int64_t lo = s0 + len * j / S, hi = s0 + len * (j + 1) / S;
    const T is = (T)lt.inv_s[k], sL = (T)lt.s[lt.L];
    T cx = 0, cy = 0, cz = 0;
    if (!LL) {
      const uint32_t ub = (uint32_t)b;
      cx = (T)(lt.origin[0] + lt.s[k] * ((double)compact3(ub) + 0.5));
      cy = (T)(lt.origin[1] + lt.s[k] * ((double)compact3(ub >> 1) + 0.5));
      cz = (T)(lt.origin[2] + lt.s[k] * ((double)compact3(ub >> 2) + 0.5));
    }
    for (int64_t i = lo + r; i < hi; i += G) {
      T q, wx, wy, wz;
      if (LL) {
        const float4 pt = a.pts[i];
        const uint32_t key = a.keys[i];
        q = (T)pt.w;
        wx = ((T)pt.x + leaf_to_box<T>(compact3(key), sh) * sL) * is;
        wy = ((T)pt.y + leaf_to_box<T>(compact3(key >> 1), sh) * sL) * is;
        wz = ((T)pt.z + leaf_to_box<T>(compact3(key >> 2), sh) * sL) * is;
      } else {
        q = (T)a.qs[i];
        wx = ((T)a.xs[i] - cx) * is;
        wy = ((T)a.ys[i] - cy) * is;
        wz = ((T)a.zs[i] - cz) * is;
      }
      const T uz = (T)5 * wz;
      T fzl = cl;
#pragma unroll
      for (int m = 0; m < N; ++m)
        if (m != l) fzl *= uz - al[m];
      T fx[N], fy[N];
      lagn<N>(nd, wx, fx);
      lagn<N>(nd, wy, fy);
      const T ql = q * fzl;
#pragma unroll
      for (int jj = 0; jj < N; ++jj) {
        const T qj = ql * fy[jj];
#pragma unroll
        for (int ii = 0; ii < N; ++ii) acc[ii + N * jj] += fx[ii] * qj;
      }
    }
  }
  for (int dd = 1; dd < G; dd <<= 1) {
#pragma unroll
    for (int i = 0; i < P; ++i) acc[i] += __shfl_xor(acc[i], dd, 64);
  }
  if (!valid || r != 0) return;
  const int cs = a.cs;
  T* out;
  if (S == 1)
    out = (sizeof(T) == 8 ? (T*)a.mom64 : (T*)a.mom32) + (lt.off[k] + b) * cs;
  else
    out = (sizeof(T) == 8 ? (T*)a.part64 : (T*)a.part32) + (pl.part_off[k] + b * S + j) * cs;
  out += P * l;
#pragma unroll
  for (int i = 0; i < P; ++i) out[i] = acc[i];
}

// the S slice rows of each level-k box added in slice order
template <typename T>
__global__ void k_p2m3d_pts_slices(FmmArgs a, P2mPlan pl, int k, int nc) {
  const int64_t nb = (int64_t)1 << (3 * k);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nb * nc) return;
  const int64_t b = g / nc;
  const int c = (int)(g - b * nc);
  const int S = pl.S[k];
  const T* src = (sizeof(T) == 8 ? (const T*)a.part64 : (const T*)a.part32) +
                 (pl.part_off[k] + b * S) * a.cs + c;
  T acc = 0;
  for (int s = 0; s < S; ++s) acc += src[(int64_t)s * a.cs];
  (sizeof(T) == 8 ? (T*)a.mom64 : (T*)a.mom32)[(a.lt.off[k] + b) * a.cs + c] = acc;
}

// (F, Fz, Gr, Gi) = (phi, dphi/dz, dphi/dx, dphi/dy) of the box's locals at w,
// in units of the box side (the 3D harmonic evaluation's outputs)
template <int N, typename T>
__device__ __forceinline__ void eval_pts3(const T* B, const PtsNodes& nd, T wx, T wy, T wz, T& F,
                                          T& Fz, T& Gr, T& Gi) {
  T fx[N], dfx[N], fy[N], dfy[N], fz[N], dfz[N];
  lagnd<N>(nd, wx, fx, dfx);
  lagnd<N>(nd, wy, fy, dfy);
  lagnd<N>(nd, wz, fz, dfz);
  F = Fz = Gr = Gi = (T)0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    T h = 0, hx = 0, hy = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T g = 0, gd = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const T v = B[i + N * j + N * N * l];
        g += fx[i] * v;
        gd += dfx[i] * v;
      }
      h += fy[j] * g;
      hx += fy[j] * gd;
      hy += dfy[j] * g;
    }
    F += fz[l] * h;
    Gr += fz[l] * hx;
    Gi += fz[l] * hy;
    Fz += dfz[l] * h;
  }
  Gr *= (T)5;
  Gi *= (T)5;
  Fz *= (T)5;
}

template <int N, bool LL>
__global__ __launch_bounds__(256) void k_l2p3d_pts(FmmArgs a, PtsNodes nd) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const LevelTable& lt = a.lt;
  const uint32_t key = a.keys[j];
  const uint32_t lx = compact3(key), ly = compact3(key >> 1), lz = compact3(key >> 2);
  const int cs = a.cs;
  float4 pt = make_float4(0.f, 0.f, 0.f, 0.f);
  double x = 0, y = 0, z = 0;
  if (LL)
    pt = a.pts[j];
  else {
    x = a.xs[j];
    y = a.ys[j];
    z = a.zs[j];
  }
  double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
  for (int k = lt.kmin; k <= lt.L; ++k) {
    const int sh = lt.L - k;
    const uint32_t box = key >> (3 * sh);
    if (k < lt.split) {
      double wx, wy, wz;
      if (LL) {
        const double sL = lt.s[lt.L], is = lt.inv_s[k];
        wx = ((double)pt.x + leaf_to_box<double>(lx, sh) * sL) * is;
        wy = ((double)pt.y + leaf_to_box<double>(ly, sh) * sL) * is;
        wz = ((double)pt.z + leaf_to_box<double>(lz, sh) * sL) * is;
      } else {
        wx = (x - (lt.origin[0] + lt.s[k] * ((double)(lx >> sh) + 0.5))) * lt.inv_s[k];
        wy = (y - (lt.origin[1] + lt.s[k] * ((double)(ly >> sh) + 0.5))) * lt.inv_s[k];
        wz = (z - (lt.origin[2] + lt.s[k] * ((double)(lz >> sh) + 0.5))) * lt.inv_s[k];
      }
      double F, Fz, Gr, Gi;
      eval_pts3<N, double>(a.loc64 + (lt.off[k] + box) * cs, nd, wx, wy, wz, F, Fz, Gr, Gi);
      const double is = lt.inv_s[k];
      phi += F * is;
      ex -= Gr * is * is;
      ey -= Gi * is * is;
      ez -= Fz * is * is;
    } else {
      const float sL = (float)lt.s[lt.L], is = (float)lt.inv_s[k];
      const float wx = (pt.x + leaf_to_box<float>(lx, sh) * sL) * is;
      const float wy = (pt.y + leaf_to_box<float>(ly, sh) * sL) * is;
      const float wz = (pt.z + leaf_to_box<float>(lz, sh) * sL) * is;
      float F, Fz, Gr, Gi;
      eval_pts3<N, float>(a.loc32 + (lt.off[k] + box) * cs, nd, wx, wy, wz, F, Fz, Gr, Gi);
      const double id = lt.inv_s[k];
      phi += (double)F * id;
      ex -= (double)Gr * id * id;
      ey -= (double)Gi * id * id;
      ez -= (double)Fz * id * id;
    }
  }
  const int64_t o = a.perm[j];
  a.pot[o] = phi + a.near_pot[j];
  if (a.field) {
    a.field[3 * o] = ex + a.near_ex[j];
    a.field[3 * o + 1] = ey + a.near_ey[j];
    a.field[3 * o + 2] = ez + a.near_ez[j];
  }
}

template <int N>
void p2m3_pts(const FmmArgs& a, bool ll, bool f64, hipStream_t st) {
  const PtsNodes nd = make_nodes(a.basis, N);
  const P2mPlan pl = make_p2m_plan(3, a.klo, a.khi, a.n);
  const int64_t thr = pl.thr_off[a.khi + 1];  // a multiple of 64
  const dim3 grid((unsigned)((N * thr + 255) / 256));
  if (f64) {
    if (ll)
      hipLaunchKernelGGL((k_p2m3d_pts<double, N, true>), grid, dim3(256), 0, st, a, pl, nd, thr);
    else
      hipLaunchKernelGGL((k_p2m3d_pts<double, N, false>), grid, dim3(256), 0, st, a, pl, nd, thr);
  } else {
    hipLaunchKernelGGL((k_p2m3d_pts<float, N, true>), grid, dim3(256), 0, st, a, pl, nd, thr);
  }
  for (int k = a.klo; k <= a.khi; ++k)
    if (pl.S[k] > 1) {
      const int64_t cnt = ((int64_t)1 << (3 * k)) * (N * N * N);
      const dim3 sg((unsigned)((cnt + 255) / 256));
      if (f64)
        hipLaunchKernelGGL(k_p2m3d_pts_slices<double>, sg, dim3(256), 0, st, a, pl, k, N * N * N);
      else
        hipLaunchKernelGGL(k_p2m3d_pts_slices<float>, sg, dim3(256), 0, st, a, pl, k, N * N * N);
    }
}

template <int N>
void l2p3_pts(const FmmArgs& a, bool ll, hipStream_t st) {
  const PtsNodes nd = make_nodes(a.basis, N);
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (ll)
    hipLaunchKernelGGL((k_l2p3d_pts<N, true>), grid, dim3(256), 0, st, a, nd);
  else
    hipLaunchKernelGGL((k_l2p3d_pts<N, false>), grid, dim3(256), 0, st, a, nd);
}

}  // namespace

void launch_p2m3d_points(const FmmArgs& a, bool leaf_local, bool fp64, hipStream_t st) {
  if (a.khi < a.klo || a.n <= 0) return;
  switch (a.p) {
    case 2: p2m3_pts<2>(a, leaf_local, fp64, st); break;
    case 3: p2m3_pts<3>(a, leaf_local, fp64, st); break;
    case 5: p2m3_pts<5>(a, leaf_local, fp64, st); break;
    default: break;  // n = 4 runs in the shared passes; the plan admits no other n
  }
}

void launch_l2p3d_points(const FmmArgs& a, bool leaf_local, hipStream_t st) {
  if (a.n <= 0) return;
  switch (a.p) {
    case 2: l2p3_pts<2>(a, leaf_local, st); break;
    case 3: l2p3_pts<3>(a, leaf_local, st); break;
    case 5: l2p3_pts<5>(a, leaf_local, st); break;
    default: break;
  }
}

}  // namespace sffmm
