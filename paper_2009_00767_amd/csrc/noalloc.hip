// noalloc.hip -- fmm_eval_noalloc: the 2D evaluation of fmm_eval for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// Every buffer the evaluation needs besides the caller's inputs and outputs
// (sort keys and their second buffers, radix counts, leaf offsets, status words,
// sorted particles, moments, locals, slice partials, operator packs, per-level
// orders, near-field sums) is carved out of one file-scope device array of
// kNoAllocScratchBytes, `scratch`.  Each device holds its own copy of it until
// the process ends; its address on a device is taken once, with that device
// current, by hipGetSymbolAddress, and only that address is handed to kernels.
// The operators are built into the array by a kernel on every call (a few
// microseconds), so a call needs no plan and no host-to-device copy.  Calls on
// one device share the array: calls that overlap in time on one device race.
// Everything runs in order on the caller's stream (no second stream, no event).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "device_common.h"

namespace sffmm {
namespace {

// The largest carve the limits below allow (FP64, n = 65536, level 6, order 20)
// is 12.7 MiB.
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
constexpr int64_t kNoAllocMaxN = 1 << 16;
constexpr int kNoAllocMaxLevels = 6;
constexpr int kNoAllocMaxOrder = 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device
bool g_gfx950[kMaxDevices] = {};

// The scratch address on the current device (taken once per device).
int scratch_on(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return FMM_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return FMM_ERR_DEVICE;
    g_gfx950[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (!g_gfx950[dev]) return FMM_ERR_DEVICE;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return FMM_ERR_DEVICE;
    }
    g_scratch[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return FMM_OK;
}

// Bump allocation of 256-byte aligned regions inside the scratch array.
struct Carve {
  unsigned char* base;
  size_t used = 0;
  bool over = false;
  template <class T>
  T* take(size_t count) {
    const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
    if (used + bytes > kNoAllocScratchBytes) {
      over = true;
      return nullptr;
    }
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

__device__ double binom_d(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double c = 1.0;
  for (int i = 1; i <= k; ++i) c *= double(n - k + i) / double(i);
  return c;
}

// u^-e for the Gaussian integer u = dx + i dy, by repeated multiplication with
// 1/u (the product order the host builder uses).
__device__ void uinv_pow(double dx, double dy, int e, double& re, double& im) {
  const double d = dx * dx + dy * dy;
  const double ir = dx / d, ii = -dy / d;
  re = 1.0;
  im = 0.0;
  for (int k = 0; k < e; ++k) {
    const double r = re * ir - im * ii;
    im = re * ii + im * ir;
    re = r;
  }
}

// Value `idx` of offset slot `slot` of the FP64 operator pack of order p in
// layout ly (the multipole-to-local lemma in box-side-scaled variables, the
// same entries as the host builder: Wb, c0, r0, t00; zero for adjacent slots
// and padding).
__device__ double pack_value(const M2lLayout& ly, int p, int slot, int idx) {
  const int dx = slot % 7 - 3, dy = slot / 7 - 3;
  if (abs(dx) <= 1 && abs(dy) <= 1) return 0.0;
  const int nk = ly.npad * ly.kpad;
  double re, im;
  if (idx < nk) {
    const int j = idx / ly.kpad, k = idx % ly.kpad;
    const int l = j / 2 + 1, m = k / 2 + 1;
    if (l > p || m > p) return 0.0;
    uinv_pow(dx, dy, l + m, re, im);
    const double c = (m & 1 ? -1.0 : 1.0) * binom_d(l + m - 1, m - 1);
    re *= c;
    im *= c;
    const int a = j & 1, b = k & 1;
    return a == b ? re : (a == 0 ? -im : im);
  }
  idx -= nk;
  if (idx < ly.npad) {  // c0: -1 / (l u^l)
    const int l = idx / 2 + 1;
    if (l > p) return 0.0;
    uinv_pow(dx, dy, l, re, im);
    return -(idx & 1 ? im : re) / double(l);
  }
  idx -= ly.npad;
  if (idx < ly.kpad) {  // r0: Re((-1)^m u^-m A_m)
    const int m = idx / 2 + 1;
    if (m > p) return 0.0;
    uinv_pow(dx, dy, m, re, im);
    const double s = m & 1 ? -1.0 : 1.0;
    return idx & 1 ? -s * im : s * re;
  }
  idx -= ly.kpad;
  if (idx == 0) return 0.5 * log(double(dx * dx + dy * dy));  // Re log(-u)
  return 0.0;
}

// One workgroup per offset slot: the FP64 pack and its FP32 rounding, then the
// lane-major FP64 / FP32 packs of the matrix-core kernel (the same mapping as
// the host builder).
__global__ __launch_bounds__(256) void k_build_ops2d(M2lLayout ly, int p, double* op64,
                                                     float* op32, double* opl64, float* opl32) {
  const int slot = blockIdx.x;
  for (int i = threadIdx.x; i < ly.stride; i += blockDim.x) {
    const double v = pack_value(ly, p, slot, i);
    op64[(size_t)slot * ly.stride + i] = v;
    op32[(size_t)slot * ly.stride + i] = (float)v;
  }
  const int ks = ly.kpad / 4, nbk = ly.npad / 16;
  const int nlane = nbk * (ks + 1) * 64, nr = ks * 64;
  for (int i = threadIdx.x; i < ly.lstride; i += blockDim.x) {
    int src = -1;
    if (i < nlane) {
      const int l = i & 63, q = i >> 6, st = q % (ks + 1), nb = q / (ks + 1);
      const int li = l & 15, g = l >> 4;
      if (st < ks)
        src = (16 * nb + li) * ly.kpad + 4 * st + g;
      else if (g == 0)
        src = ly.npad * ly.kpad + 16 * nb + li;
    } else if (i < nlane + nr) {
      const int r = i - nlane, st = r >> 6, g = (r & 63) >> 4;
      src = ly.npad * ly.kpad + ly.npad + 4 * st + g;
    } else if (i == nlane + nr) {
      src = ly.npad * ly.kpad + ly.npad + ly.kpad;  // t00
    }
    const double v = src >= 0 ? pack_value(ly, p, slot, src) : 0.0;
    opl64[(size_t)slot * ly.lstride + i] = v;
    opl32[(size_t)slot * ly.lstride + i] = (float)v;
  }
}

}  // namespace
}  // namespace sffmm

using namespace sffmm;

extern "C" int fmm_eval_noalloc(const fmm_options* opt, int64_t n, const double* pos,
                                const double* q, double* pot, double* field, void* stream) {
  if (!opt) return FMM_ERR_INVALID_ARG;
  const fmm_options& o = *opt;
  if (o.kernel != FMM_LOG2D || o.order_policy != FMM_ORDER_FIXED || o.max_systems > 1 ||
      o.adaptive_near != 0)
    return FMM_ERR_UNSUPPORTED;
  if (o.precision != FMM_FP64 && o.precision != FMM_FP32) return FMM_ERR_UNSUPPORTED;
  if (o.flags & ~(FMM_NO_FIELD | FMM_SYNC_CHECK)) return FMM_ERR_UNSUPPORTED;
  if (!(o.side > 0) || !std::isfinite(o.side) || !std::isfinite(o.origin[0]) ||
      !std::isfinite(o.origin[1]))
    return FMM_ERR_INVALID_ARG;
  if (o.levels < 0 || o.order_p < 1 || o.order_p > kMaxOrder2D) return FMM_ERR_INVALID_ARG;
  if (n < 0) return FMM_ERR_INVALID_ARG;
  // the fixed scratch's limits
  if (o.levels > kNoAllocMaxLevels || o.order_p > kNoAllocMaxOrder || n > kNoAllocMaxN)
    return FMM_ERR_SCRATCH;
  const bool want_field = !(o.flags & FMM_NO_FIELD);
  if (n > 0 && (!pos || !q || !pot || (want_field && !field))) return FMM_ERR_INVALID_ARG;
  if (!want_field) field = nullptr;
  if (n == 0) return FMM_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FMM_ERR_DEVICE;
  unsigned char* base = nullptr;
  int rc = scratch_on(dev, &base);
  if (rc != FMM_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);

  const bool f32 = o.precision == FMM_FP32;
  const int L = o.levels, p = o.order_p, pb = order_bucket(p);
  const M2lLayout ly = m2l2d_layout(pb);
  const int cs = ly.cs;
  int64_t nbox64 = 0, nbox32 = 0;
  const LevelTable lt = level_table(2, f32, o.side, o.origin, L, 1, &nbox64, &nbox32);
  const int64_t nleaf = (int64_t)1 << (2 * L);
  const int bits = 2 * L;
  const int hi64 = std::min(lt.L, lt.split - 1);

  Carve c{base};
  uint32_t* keys = c.take<uint32_t>(n);
  uint32_t* keys_alt = c.take<uint32_t>(n);
  int32_t* vals = c.take<int32_t>(n);
  int32_t* vals_alt = c.take<int32_t>(n);
  int32_t* hist = c.take<int32_t>(radix_hist_entries(n));
  int32_t* tot = c.take<int32_t>(256);
  const bool two_digit = bits > 8 && bits <= 16 && radix_two_digit(n, bits);
  int32_t* parts = two_digit ? c.take<int32_t>(radix_two_digit_parts()) : nullptr;
  int32_t* leaf_start = c.take<int32_t>(nleaf + 1);
  int32_t* flag = c.take<int32_t>(4);
  int32_t* ord = c.take<int32_t>(16);
  float4 *pts = nullptr, *pts_alt = nullptr;
  uint8_t* over = nullptr;
  double *xs = nullptr, *ys = nullptr, *qs = nullptr;
  if (f32) {
    pts = c.take<float4>(n);
    pts_alt = c.take<float4>(n);
    if (L >= 2) over = c.take<uint8_t>((size_t)1 << (2 * (L - 2)));
  } else {
    xs = c.take<double>(n);
    ys = c.take<double>(n);
    qs = c.take<double>(n);
  }
  double* mom64 = c.take<double>((size_t)(nbox64 * cs));
  double* loc64 = c.take<double>((size_t)(nbox64 * cs));
  float* mom32 = c.take<float>((size_t)(nbox32 * cs));
  float* loc32 = c.take<float>((size_t)(nbox32 * cs));
  double* part64 = c.take<double>(p2m2d_partial_entries(lt, lt.kmin, hi64, n, cs));
  float* part32 = c.take<float>(p2m2d_partial_entries(lt, lt.split, lt.L, n, cs));
  double* op64 = c.take<double>((size_t)49 * ly.stride);
  float* op32 = c.take<float>((size_t)49 * ly.stride);
  double* opl64 = c.take<double>((size_t)49 * ly.lstride);
  float* opl32 = c.take<float>((size_t)49 * ly.lstride);
  double* near_pot = c.take<double>(n);
  double* near_ex = c.take<double>(n);
  double* near_ey = c.take<double>(n);
  if (c.over) return FMM_ERR_SCRATCH;

  // status words, orders and the box vectors (whose padding values no kernel
  // writes, and which an earlier call may have left holding other data) start
  // fresh in every call: fill kernels, no memset
  launch_fill_i32(flag, 0, 4, st);
  launch_fill_i32(ord, p, 16, st);
  launch_fill_i32(reinterpret_cast<int32_t*>(mom64), 0, nbox64 * cs * 2, st);
  launch_fill_i32(reinterpret_cast<int32_t*>(loc64), 0, nbox64 * cs * 2, st);
  launch_fill_i32(reinterpret_cast<int32_t*>(mom32), 0, nbox32 * cs, st);
  launch_fill_i32(reinterpret_cast<int32_t*>(loc32), 0, nbox32 * cs, st);
  hipLaunchKernelGGL(k_build_ops2d, dim3(49), dim3(256), 0, st, ly, p, op64, op32, opl64, opl32);
  const int32_t tag = 1;
  launch_bin(2, pos, n, lt, keys, vals, flag, tag, hist, st, q, f32 ? pts : nullptr,
             two_digit ? 8 : 0);
  int which = 0;
  if (two_digit)
    radix_sort_two_digit(keys, vals, keys_alt, vals_alt, n, bits, hist, tot, leaf_start, nleaf,
                         parts, st, f32 ? pts : nullptr, f32 ? pts_alt : nullptr);
  else
    which = radix_sort(keys, vals, keys_alt, vals_alt, n, bits, hist, tot, st, true,
                       f32 ? pts : nullptr, f32 ? pts_alt : nullptr);
  const uint32_t* skeys = which ? keys_alt : keys;
  const int32_t* perm = which ? vals_alt : vals;
  if (!two_digit) launch_leaf_bounds(skeys, n, nleaf, leaf_start, st);
  if (!f32) launch_gather_f64(2, pos, q, perm, n, xs, ys, nullptr, qs, st);

  FmmArgs a{};
  a.lt = lt;
  a.p = p;
  a.ord = ord;
  a.ord_full = p == pb ? 1 : 0;
  a.m2l_mb = 1;
  a.m2l_remap = 1;
  a.cs = cs;
  a.n = n;
  a.keys = skeys;
  a.leaf_start = leaf_start;
  a.perm = perm;
  a.xs = xs;
  a.ys = ys;
  a.qs = qs;
  a.pts = f32 ? (which ? pts_alt : pts) : nullptr;
  a.mom64 = mom64;
  a.loc64 = loc64;
  a.mom32 = mom32;
  a.loc32 = loc32;
  a.part64 = part64;
  a.part32 = part32;
  a.op64 = op64;
  a.op32 = op32;
  a.opl64 = opl64;
  a.opl32 = opl32;
  a.near_pot = near_pot;
  a.near_ex = near_ex;
  a.near_ey = near_ey;
  a.p2p_over = over;
  a.pot = pot;
  a.field = field;
  FmmArgs a64 = a, a32 = a;
  a64.klo = lt.kmin;
  a64.khi = hi64;
  a32.klo = std::max(lt.split, lt.kmin);
  a32.khi = lt.L;
  // the same kernels as fmm_eval, in order on one stream
  launch_p2p2d(a, f32, st);
  if (f32) {
    if (a64.khi >= a64.klo) {
      launch_p2m2d(a64, true, true, st);
      launch_m2l2d(a64, true, st);
    }
    launch_p2m2d(a32, true, false, st);
    launch_m2l2d(a32, false, st);
  } else {
    launch_p2m2d(a64, false, true, st);
    launch_m2l2d(a64, true, st);
  }
  launch_l2p2d(a, f32, st);
  if (hipGetLastError() != hipSuccess) return FMM_ERR_DEVICE;
  if (o.flags & FMM_SYNC_CHECK) {
    int32_t f = 0;
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(&f, flag, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess)
      return FMM_ERR_DEVICE;
    if (f == tag) return FMM_ERR_DOMAIN;
  }
  return FMM_OK;
}
