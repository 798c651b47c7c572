// fmm_api.cpp -- the C ABI of include/fmm.h: plan construction (tables,
// operators, device buffers), the evaluation pipeline on the caller's stream,
// status, statistics and debug export.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "device_common.h"
#include "points2d.h"
#include "points3d.h"

using namespace sffmm;

namespace sffmm {

LevelTable level_table(int dim, bool f32, double side, const double* origin, int L, int nsys,
                       int64_t* nbox64, int64_t* nbox32) {
  LevelTable lt{};
  lt.L = L;
  lt.kmin = 2;
  lt.split = f32 ? 3 : L + 1;
  lt.nsys = nsys;
  lt.side = side;
  for (int d = 0; d < 3; ++d) lt.origin[d] = d < dim ? origin[d] : 0.0;
  int64_t off64 = 0, off32 = 0;
  for (int k = lt.kmin; k <= L; ++k) {
    const int64_t nb = (int64_t)nsys << (dim * k);
    if (k < lt.split) {
      lt.off[k] = off64;
      off64 += nb;
    } else {
      lt.off[k] = off32;
      off32 += nb;
    }
  }
  lt.off[L + 1] = L + 1 < lt.split ? off64 : off32;
  for (int k = 0; k <= L; ++k) {
    lt.s[k] = side / (double)((int64_t)1 << k);
    lt.inv_s[k] = (double)((int64_t)1 << k) / side;
    lt.log_s[k] = std::log(lt.s[k]);
  }
  lt.leaf_scale = (double)((int64_t)1 << L) / side;
  if (nbox64) *nbox64 = off64;
  if (nbox32) *nbox32 = off32;
  return lt;
}

}  // namespace sffmm

struct fmm_plan_s {
  fmm_options opt{};
  int dim = 2, L = 0, p = 0, pb = 0, cs = 0, prec = 0, device = 0;
  int basis = 0;  // 0 expansions, 1 fixed point charges (the paper's nodes), 2 on Chebyshev points
  bool root = false;          // FMM_ROOT_FRAME: the point-charge passes in the root frame
  double* rbuf = nullptr;     // its box vectors / linear forms [boxes][64]
  bool f32 = false;  // FP32 / BF16 modes: leaf-local FP32 particles, levels >= 3 in FP32
  LevelTable lt{};
  M2lLayout ly{};
  int64_t nbox64 = 0, nbox32 = 0, nleaf = 0, maxn = 0;
  std::vector<void*> allocs;
  uint32_t* keys = nullptr;
  uint32_t* keys_alt = nullptr;
  int32_t* vals = nullptr;
  int32_t* vals_alt = nullptr;
  int32_t* hist = nullptr;
  int32_t* radix_tot = nullptr;  // the 256 digit totals of a radix pass
  int32_t* radix_parts = nullptr;  // two-digit sort: digit counts of large buckets' parts
  int32_t* leaf_start = nullptr;
  // Status words: [0] a position outside the box or NaN, [1] the learned order
  // rejected by the judge.  Each holds the tag of the last evaluation that set
  // it, so nothing has to clear them before an evaluation: plain evaluations
  // count tag through 1 .. 2^30 - 1; a batched evaluation (one HIP graph,
  // whose kernel arguments are fixed) uses kGraphTag and clears the words
  // inside the graph.
  int32_t* flag = nullptr;
  int32_t tag = 0;
  static constexpr int32_t kGraphTag = 0x7FFFFFFF;
  double* xs = nullptr;
  double* ys = nullptr;
  double* zs = nullptr;
  double* qs = nullptr;
  float4* pts = nullptr;
  float4* pts_alt = nullptr;  // FP32 modes: the records' second radix buffer
  double* mom64 = nullptr;
  double* loc64 = nullptr;
  float* mom32 = nullptr;
  float* loc32 = nullptr;
  double* part64 = nullptr;
  float* part32 = nullptr;
  double* op64 = nullptr;
  float* op32 = nullptr;
  uint16_t* op16 = nullptr;  // BF16 bit patterns (2D lane-major)
  double* opl64 = nullptr;   // 2D lane-major packs
  float* opl32 = nullptr;
  double* near_pot = nullptr;
  double* near_ex = nullptr;
  double* near_ey = nullptr;
  double* near_ez = nullptr;
  double* m2l_part = nullptr;  // 3D: partial sums of the split small-level contraction
  uint8_t* p2p_over = nullptr;  // 2D FP32 near field: tiles whose halo exceeds the LDS stage
  // adaptive depth (2D, one system; adaptive_near > 0): every sorted particle's
  // depth and the per-level open flags of the boxes
  uint8_t* depth = nullptr;
  uint8_t* adapt_open = nullptr;
  // 2D per-level orders on the device: one row of kOrdCols per tree (the single
  // tree, or each depth group of a batched call), indexed by level
  static constexpr int kOrdRows = kMaxLevels2D + 2, kOrdCols = 16;
  int32_t* d_ord = nullptr;
  int32_t h_ord[16] = {};  // orders set on the host (fixed policy, or the fallback order)
  // 2D M2L tile variant (FMM_AUTOTUNE picks it by timing; default 1 / XCD remap on)
  int m2l_mb = 1, m2l_remap = 1;
  float m2l_tuned_ms = 0.f;
  // learned order (2D): network weights, per-system order-selection tables
  // (pinned staging and device copy), chunk partials, debug features, judge
  bool learned = false, have_model = false;
  int p_fb = 0;  // fixed fallback order
  float* d_mlp = nullptr;
  OrderSys* d_ordsys = nullptr;  // [max_systems + 1]: the batched table, then the single system's
  int64_t pblk_cap = 0;
  double* d_pq = nullptr;
  int32_t* d_pcnt = nullptr;
  float* d_feat = nullptr;
  int last_nsys = 0;
  fmm_plan_s* judge = nullptr;  // FP64 fixed-order plan of the same shape
  double* jpot = nullptr;
  double* jfield = nullptr;
  double* jerr = nullptr;
  // capacities (single system: exactly the plan's tree; batched: worst case)
  int lcap = 0;                 // deepest tree
  int64_t leaf_cap = 0;         // leaf_start entries
  size_t part64_cap = 0, part32_cap = 0;  // partial buffers (values)
  // batched evaluations: the shape of the last fmm_batch_prepare (host copy of
  // its tables, the device tables the graph reads), the record of the caller's
  // buffers, the graph stream and the captured graph
  hipStream_t gstream = nullptr;
  int64_t* d_sysoff = nullptr;
  int32_t* d_sysinfo = nullptr;
  BatchIo* d_io = nullptr;
  bool prepared = false;
  int prep_nsys = 0;
  int64_t prep_n = 0;
  std::vector<int64_t> prep_off;
  std::vector<int32_t> prep_depth;
  bool prep_model = false;  // the prepared graph runs the order selection
  int32_t graph_builds = 0; // graphs instantiated since the plan was made
  hipGraphExec_t graph_exec = nullptr;
  const uint32_t* graph_keys = nullptr;  // sorted keys / permutation the graph writes
  const int32_t* graph_perm = nullptr;
  bool last_batched = false;
  // state of the last evaluation
  int64_t last_n = 0;
  const uint32_t* sorted_keys = nullptr;
  const int32_t* perm = nullptr;
  hipStream_t last_stream = nullptr;
  // FMM_TIMING: a ring of per-evaluation phase events; fmm_get_stats averages
  // the evaluations recorded since its previous call (at most kRing).
  static constexpr int kRing = 64;
  // fork_ev forks the near-field stream (and the batched path's graph stream)
  // from the caller's stream; join_ev joins the graph stream back.
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // Near-field stream: P2P needs only the sort and overlaps the far field.
  hipStream_t near = nullptr;
  hipEvent_t near_ev = nullptr;
  bool have_events = false;
  unsigned ev_mask = 0;  // events recorded: FMM_TIMING all, FMM_TIMING_NEAR 6-7, FMM_TIMING_M2L 2-3
  int ring_next = 0, ring_count = 0;
  bool ring_batched[64] = {};  // slot timed a batched (graph) evaluation
  // events per evaluation: 0 start, 1 sorted, 2 moments, 3 main M2L kernel done,
  // 4 locals (after the join), 5 end (caller's stream); 6 / 7 near field start
  // / end (near-field stream)
  hipEvent_t ev[kRing][8]{};
};

namespace {

template <class T>
int dalloc(fmm_plan_s* pl, T** out, size_t count) {
  void* p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return FMM_ERR_NOMEM;
  }
  pl->allocs.push_back(p);
  *out = static_cast<T*>(p);
  return FMM_OK;
}

void free_plan(fmm_plan_s* pl) {
  if (!pl) return;
  (void)hipSetDevice(pl->device);
  (void)hipDeviceSynchronize();
  for (void* p : pl->allocs) (void)hipFree(p);
  if (pl->have_events)
    for (auto& r : pl->ev)
      for (auto& e : r) (void)hipEventDestroy(e);
  if (pl->fork_ev) (void)hipEventDestroy(pl->fork_ev);
  if (pl->join_ev) (void)hipEventDestroy(pl->join_ev);
  if (pl->graph_exec) (void)hipGraphExecDestroy(pl->graph_exec);
  if (pl->gstream) (void)hipStreamDestroy(pl->gstream);
  if (pl->near_ev) (void)hipEventDestroy(pl->near_ev);
  if (pl->near) (void)hipStreamDestroy(pl->near);
  fmm_plan_s* j = pl->judge;
  delete pl;
  if (j) free_plan(j);
}

LevelTable make_level_table(const fmm_plan_s* pl, int L, int nsys, int64_t* nbox64,
                            int64_t* nbox32);
int autotune_m2l(fmm_plan_s* pl);
bool orders_full(const fmm_plan_s* pl);

// Copies the host per-level orders into every row of the device table.
int upload_orders(fmm_plan_s* pl) {
  std::vector<int32_t> rows((size_t)fmm_plan_s::kOrdRows * fmm_plan_s::kOrdCols);
  for (int r = 0; r < fmm_plan_s::kOrdRows; ++r)
    for (int k = 0; k < fmm_plan_s::kOrdCols; ++k)
      rows[(size_t)r * fmm_plan_s::kOrdCols + k] = pl->h_ord[k];
  if (hipMemcpy(pl->d_ord, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
      hipSuccess)
    return FMM_ERR_DEVICE;
  return FMM_OK;
}

int check_device(int* dev) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return FMM_ERR_DEVICE;
  }
  if (hipGetDevice(dev) != hipSuccess) return FMM_ERR_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return FMM_ERR_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FMM_ERR_DEVICE;
  return FMM_OK;
}

}  // namespace

extern "C" {

const char* fmm_status_str(int s) {
  switch (s) {
    case FMM_OK:
      return "ok";
    case FMM_ERR_INVALID_ARG:
      return "invalid argument";
    case FMM_ERR_DOMAIN:
      return "a position lies outside the box or is NaN";
    case FMM_ERR_NOMEM:
      return "device allocation failed";
    case FMM_ERR_DEVICE:
      return "no usable gfx950 device or a HIP runtime error";
    case FMM_ERR_UNSUPPORTED:
      return "unsupported combination of options";
    case FMM_ERR_SCRATCH:
      return "input beyond the fixed scratch of fmm_eval_noalloc (n <= 65536, levels <= 6, "
             "order <= 20)";
    case FMM_WARN_FALLBACK:
      return "learned order rejected by its check; fixed order used";
    default:
      return "unknown status";
  }
}

static bool known_kernel(int32_t k) {
  return k == FMM_LOG2D || k == FMM_COULOMB3D || k == FMM_COULOMB3D_POINTS ||
         k == FMM_COULOMB3D_CHEBYSHEV || k == FMM_LOG2D_POINTS || k == FMM_LOG2D_CHEBYSHEV;
}
static int kernel_dim(int32_t k) {
  return k == FMM_LOG2D || k == FMM_LOG2D_POINTS || k == FMM_LOG2D_CHEBYSHEV ? 2 : 3;
}
// 0: expansions; 1: point charges at the paper's nodes; 2: at Chebyshev points
static int kernel_basis(int32_t k) {
  return k == FMM_COULOMB3D_POINTS || k == FMM_LOG2D_POINTS        ? 1
         : k == FMM_COULOMB3D_CHEBYSHEV || k == FMM_LOG2D_CHEBYSHEV ? 2
                                                                     : 0;
}

int fmm_default_options(int32_t kernel, fmm_options* out) {
  if (!out || !known_kernel(kernel)) return FMM_ERR_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  out->kernel = kernel;
  out->levels = kernel_dim(kernel) == 2 ? 4 : 3;
  out->order_p = kernel == FMM_LOG2D ? 12 : kernel == FMM_COULOMB3D ? 8 : 4;
  out->precision = FMM_FP64;
  out->order_policy = FMM_ORDER_FIXED;
  out->side = 5.0;
  out->tol = 1e-6;
  out->max_particles = 1 << 20;
  out->max_systems = 1;
  out->max_levels = out->levels;
  return FMM_OK;
}

int fmm_plan(const fmm_options* opt, fmm_plan_t* out) {
  if (!opt || !out) return FMM_ERR_INVALID_ARG;
  *out = nullptr;
  const fmm_options& o = *opt;
  if (!known_kernel(o.kernel)) return FMM_ERR_INVALID_ARG;
  const int dim = kernel_dim(o.kernel);
  const int basis = kernel_basis(o.kernel);
  const int maxL = dim == 2 ? kMaxLevels2D : kMaxLevels3D;
  const int maxp = dim == 2 ? kMaxOrder2D : kMaxOrder3D;
  if (o.levels < 0 || o.levels > maxL) return FMM_ERR_INVALID_ARG;
  if (o.order_p < 1 || o.order_p > maxp) return FMM_ERR_INVALID_ARG;
  // points per axis: 4 for the paper's set, 2..8 for the 2D Chebyshev points,
  // 2..5 for the 3D ones
  if (basis && !(basis == 2 ? o.order_p >= 2 &&
                                  o.order_p <= (dim == 2 ? kPoints2DMaxN : kPoints3DMaxN)
                            : o.order_p == 4))
    return FMM_ERR_UNSUPPORTED;
  if (o.precision < FMM_FP64 || o.precision > FMM_BF16_M2L) return FMM_ERR_INVALID_ARG;
  if (o.order_policy != FMM_ORDER_FIXED && o.order_policy != FMM_ORDER_LEARNED)
    return FMM_ERR_INVALID_ARG;
  if (!(o.side > 0) || !std::isfinite(o.side)) return FMM_ERR_INVALID_ARG;
  for (int d = 0; d < dim; ++d)
    if (!std::isfinite(o.origin[d])) return FMM_ERR_INVALID_ARG;
  if (o.max_particles < 0 || o.max_particles > 0x7FFFFFFFLL - 1) return FMM_ERR_INVALID_ARG;
  if (o.flags & ~(FMM_NO_FIELD | FMM_SYNC_CHECK | FMM_TIMING | FMM_TIMING_NEAR | FMM_TIMING_M2L |
                  FMM_JUDGE | FMM_AUTOTUNE | FMM_ROOT_FRAME))
    return FMM_ERR_INVALID_ARG;
  // the root frame needs the point charges and double precision (Discussion (3))
  if ((o.flags & FMM_ROOT_FRAME) &&
      (!basis || dim != 3 || o.order_p != 4 || o.precision != FMM_FP64))
    return FMM_ERR_UNSUPPORTED;
  const bool learned = o.order_policy == FMM_ORDER_LEARNED;
  if ((o.flags & FMM_JUDGE) && !learned) return FMM_ERR_INVALID_ARG;
  if (learned && (!(o.tol > 0) || !std::isfinite(o.tol))) return FMM_ERR_INVALID_ARG;
  // BF16 M2L and the learned order exist for the 2D kernel only.
  if ((o.precision == FMM_BF16_M2L || learned) && (dim != 2 || basis)) return FMM_ERR_UNSUPPORTED;
  const bool batched = o.max_systems > 1;
  if (o.max_systems < 0 || o.max_systems > (1 << 20)) return FMM_ERR_INVALID_ARG;
  // adaptive depth: 2D, one system, fixed order, levels >= 2
  if (o.adaptive_near < 0) return FMM_ERR_INVALID_ARG;
  if (o.adaptive_near > 0 && (dim != 2 || basis || batched || learned || o.levels < 2))
    return FMM_ERR_UNSUPPORTED;
  if (batched) {
    if (dim != 2 || basis) return FMM_ERR_UNSUPPORTED;
    if (o.max_levels < 0 || o.max_levels > kMaxLevels2D) return FMM_ERR_INVALID_ARG;
    int rbits = 0;
    while ((1 << rbits) < o.max_systems) ++rbits;
    if (rbits + 2 * std::max(o.levels, o.max_levels) > 32) return FMM_ERR_INVALID_ARG;
  }
  int dev = 0;
  int rc = check_device(&dev);
  if (rc) return rc;

  fmm_plan_s* pl = new (std::nothrow) fmm_plan_s();
  if (!pl) return FMM_ERR_NOMEM;
  pl->opt = o;
  pl->dim = dim;
  pl->L = o.levels;
  pl->learned = learned;
  pl->p_fb = o.order_p;
  // the learned order picks from 4..24: the layout holds the larger of that and
  // the fallback order
  pl->p = learned ? std::max(o.order_p, kLearnedMaxOrder) : o.order_p;
  pl->basis = basis;
  pl->pb = basis ? pl->p : dim == 2 ? order_bucket(pl->p) : order_bucket3(pl->p);
  pl->ly = dim == 2 ? (basis ? points2d_layout(pl->p, o.levels) : m2l2d_layout(pl->pb))
                    : basis ? points3d_layout_n(pl->p) : m2l3d_layout(pl->pb);
  pl->cs = pl->ly.cs;
  // the 2D matrix-core kernel stages box rows of 4 (kpad / 4 + 1) values
  if (dim == 2 && !basis && pl->ly.cs != pl->ly.kpad + 4) {
    free_plan(pl);
    return FMM_ERR_UNSUPPORTED;
  }
  pl->prec = o.precision;
  pl->f32 = o.precision != FMM_FP64;
  pl->device = dev;
  pl->maxn = o.max_particles;

  pl->lt = make_level_table(pl, pl->L, 1, &pl->nbox64, &pl->nbox32);
  const LevelTable& lt = pl->lt;
  pl->nleaf = (int64_t)1 << (dim * lt.L);
  pl->lcap = batched ? std::max(o.levels, o.max_levels) : o.levels;
  const int64_t nsysmax = batched ? o.max_systems : 1;
  if (batched) {
    // worst case over every grouping of at most max_systems systems of depth
    // at most lcap: all systems at depth lcap
    int64_t nb64 = 0, nb32 = 0;
    (void)make_level_table(pl, pl->lcap, 1, &nb64, &nb32);
    pl->nbox64 = std::max(pl->nbox64, nb64 * nsysmax);
    pl->nbox32 = std::max(pl->nbox32, nb32 * nsysmax);
    pl->leaf_cap = (nsysmax << (2 * pl->lcap)) + (pl->lcap + 2);
  } else {
    pl->leaf_cap = pl->nleaf + 1;
  }
  const int64_t N = pl->maxn > 0 ? pl->maxn : 1;
  const int hi64 = std::min(lt.L, lt.split - 1);
  rc = 0;
  rc |= dalloc(pl, &pl->keys, N);
  rc |= dalloc(pl, &pl->keys_alt, N);
  rc |= dalloc(pl, &pl->vals, N);
  rc |= dalloc(pl, &pl->vals_alt, N);
  rc |= dalloc(pl, &pl->hist, radix_hist_entries(N));
  rc |= dalloc(pl, &pl->radix_tot, (size_t)256);
  if (dim * lt.L > 8 && dim * lt.L <= 16)
    rc |= dalloc(pl, &pl->radix_parts, radix_two_digit_parts());
  rc |= dalloc(pl, &pl->leaf_start, (size_t)std::max(pl->leaf_cap, pl->nleaf + 1));
  rc |= dalloc(pl, &pl->flag, 4);
  if (!rc && hipMemset(pl->flag, 0, 4 * sizeof(int32_t)) != hipSuccess) rc |= FMM_ERR_DEVICE;
  if (pl->f32) {
    rc |= dalloc(pl, &pl->pts, N);
    rc |= dalloc(pl, &pl->pts_alt, N);
    // one flag per 4 x 4-leaf tile of the deepest tree (of every system)
    if (dim == 2 && pl->lcap >= 2)
      rc |= dalloc(pl, &pl->p2p_over, (size_t)nsysmax << (2 * (pl->lcap - 2)));
  } else {
    rc |= dalloc(pl, &pl->xs, N);
    rc |= dalloc(pl, &pl->ys, N);
    if (dim == 3) rc |= dalloc(pl, &pl->zs, N);
    rc |= dalloc(pl, &pl->qs, N);
  }
  rc |= dalloc(pl, &pl->mom64, (size_t)(pl->nbox64 * pl->cs));
  rc |= dalloc(pl, &pl->loc64, (size_t)(pl->nbox64 * pl->cs));
  rc |= dalloc(pl, &pl->mom32, (size_t)(pl->nbox32 * pl->cs));
  rc |= dalloc(pl, &pl->loc32, (size_t)(pl->nbox32 * pl->cs));
  const size_t slots = dim == 2 ? 49 : 343;
  if (dim == 2) {
    pl->part64_cap = p2m2d_partial_entries(lt, lt.kmin, hi64, N, pl->cs);
    pl->part32_cap = p2m2d_partial_entries(lt, lt.split, lt.L, N, pl->cs);
    if (batched) {
      // rows per level <= boxes + 2 n / 1024 (slices are powers of two)
      int64_t r64 = 0, r32 = 0;
      const int sp = pl->f32 ? 3 : pl->lcap + 1;
      for (int k = 2; k <= pl->lcap; ++k) {
        const int64_t rows = (nsysmax << (2 * k)) + 2 * N / 1024 + 1;
        (k < sp ? r64 : r32) += rows;
      }
      pl->part64_cap = std::max(pl->part64_cap, (size_t)(r64 * pl->cs + 1));
      pl->part32_cap = std::max(pl->part32_cap, (size_t)(r32 * pl->cs + 1));
    }
  } else {
    pl->part64_cap = p2m3d_partial_entries(lt.kmin, hi64, N, pl->cs);
    pl->part32_cap = p2m3d_partial_entries(lt.split, lt.L, N, pl->cs);
  }
  rc |= dalloc(pl, &pl->part64, pl->part64_cap);
  rc |= dalloc(pl, &pl->part32, pl->part32_cap);
  if (batched) {
    rc |= dalloc(pl, &pl->d_sysoff, (size_t)nsysmax + 1);
    rc |= dalloc(pl, &pl->d_sysinfo, 2 * (size_t)nsysmax);
    rc |= dalloc(pl, &pl->d_io, 1);
  }
  rc |= dalloc(pl, &pl->op64, slots * pl->ly.stride);
  rc |= dalloc(pl, &pl->op32, slots * pl->ly.stride);
  if (o.precision == FMM_BF16_M2L) rc |= dalloc(pl, &pl->op16, (size_t)49 * pl->ly.l16);
  rc |= dalloc(pl, &pl->opl64, (size_t)slots * pl->ly.lstride);
  rc |= dalloc(pl, &pl->opl32, (size_t)slots * pl->ly.lstride);
  rc |= dalloc(pl, &pl->d_ord, (size_t)fmm_plan_s::kOrdRows * fmm_plan_s::kOrdCols);
  if (learned) {
    pl->pblk_cap = N / order_chunk() + nsysmax + 1;
    rc |= dalloc(pl, &pl->d_mlp, (size_t)FMM_MLP_NPARAM);
    rc |= dalloc(pl, &pl->d_ordsys, (size_t)nsysmax + 1);
    rc |= dalloc(pl, &pl->d_pq, (size_t)pl->pblk_cap);
    rc |= dalloc(pl, &pl->d_pcnt, (size_t)pl->pblk_cap * (kMaxLevels2D + 1));
    rc |= dalloc(pl, &pl->d_feat, (size_t)nsysmax * (kMaxLevels2D + 1) * 3);
    if (o.flags & FMM_JUDGE) {
      rc |= dalloc(pl, &pl->jpot, (size_t)N);
      rc |= dalloc(pl, &pl->jfield, (size_t)N * dim);
      rc |= dalloc(pl, &pl->jerr, (size_t)nsysmax + 1);
    }
  }
  pl->root = (o.flags & FMM_ROOT_FRAME) != 0;
  if (pl->root) rc |= dalloc(pl, &pl->rbuf, (size_t)(pl->nbox64 * 64));
  if (o.adaptive_near > 0) {
    rc |= dalloc(pl, &pl->depth, N);
    rc |= dalloc(pl, &pl->adapt_open, (size_t)adapt_open_off(lt.L));
  }
  rc |= dalloc(pl, &pl->near_pot, N);
  rc |= dalloc(pl, &pl->near_ex, N);
  rc |= dalloc(pl, &pl->near_ey, N);
  if (dim == 3) rc |= dalloc(pl, &pl->near_ez, N);
  if (dim == 3) rc |= dalloc(pl, &pl->m2l_part, m2l3d_partial_entries(pl->cs));
  if (rc) {
    free_plan(pl);
    return FMM_ERR_NOMEM;
  }
  // Coefficient rows carry a few padding values that no kernel writes: clear
  // them once so that debug exports are fully defined.
  if (hipMemset(pl->mom64, 0, (size_t)(pl->nbox64 * pl->cs) * sizeof(double)) != hipSuccess ||
      hipMemset(pl->loc64, 0, (size_t)(pl->nbox64 * pl->cs) * sizeof(double)) != hipSuccess ||
      hipMemset(pl->mom32, 0, (size_t)(pl->nbox32 * pl->cs) * sizeof(float)) != hipSuccess ||
      hipMemset(pl->loc32, 0, (size_t)(pl->nbox32 * pl->cs) * sizeof(float)) != hipSuccess) {
    free_plan(pl);
    return FMM_ERR_DEVICE;
  }
  for (int k = 0; k < fmm_plan_s::kOrdCols; ++k) pl->h_ord[k] = k >= 2 ? pl->p_fb : 0;
  if (upload_orders(pl) != FMM_OK) {
    free_plan(pl);
    return FMM_ERR_DEVICE;
  }
  {
    std::vector<double> ops(slots * pl->ly.stride);
    if (dim == 2 && basis)
      build_points2d_operators(basis, pl->p, ops.data());
    else if (dim == 2)
      build_m2l2d_operators(pl->p, pl->ly, ops.data());
    else if (basis && pl->p == 4)
      build_points3d_operators(pl->ly, basis, ops.data());
    else if (basis)
      build_points3d_operators_n(pl->ly, basis, pl->p, ops.data());
    else
      build_m2l3d_operators(pl->p, pl->ly, ops.data());
    std::vector<float> ops32(ops.size());
    for (size_t i = 0; i < ops.size(); ++i) ops32[i] = (float)ops[i];  // rounded once
    {
      std::vector<double> lp((size_t)slots * pl->ly.lstride);
      if (dim == 2 && basis)
        build_points2d_lane_pack(basis, pl->p, pl->lt, lp.data());
      else if (dim == 2)
        build_m2l2d_lane_pack(pl->ly, ops.data(), lp.data());
      else
        build_m2l3d_lane_pack(pl->ly, ops.data(), lp.data());
      std::vector<float> lp32(lp.size());
      for (size_t i = 0; i < lp.size(); ++i) lp32[i] = (float)lp[i];  // rounded once
      if (hipMemcpy(pl->opl64, lp.data(), lp.size() * sizeof(double), hipMemcpyHostToDevice) !=
              hipSuccess ||
          hipMemcpy(pl->opl32, lp32.data(), lp32.size() * sizeof(float), hipMemcpyHostToDevice) !=
              hipSuccess) {
        free_plan(pl);
        return FMM_ERR_DEVICE;
      }
    }
    if (pl->op16) {
      std::vector<uint16_t> ops16((size_t)49 * pl->ly.l16);
      build_m2l2d_bf16(pl->ly, ops.data(), ops16.data());
      if (hipMemcpy(pl->op16, ops16.data(), ops16.size() * sizeof(uint16_t),
                    hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(pl);
        return FMM_ERR_DEVICE;
      }
    }
    if (hipMemcpy(pl->op64, ops.data(), ops.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(pl->op32, ops32.data(), ops32.size() * sizeof(float), hipMemcpyHostToDevice) !=
            hipSuccess) {
      free_plan(pl);
      return FMM_ERR_DEVICE;
    }
  }
  // Events that order work between the plan's streams on one device, and the
  // timing events, need only a device-scope release: the system-scope fence an
  // event records by default writes back the L2 at every record and stalls the
  // stream it is recorded on.
  constexpr unsigned kSyncEv = hipEventDisableTiming | hipEventDisableSystemFence;
  if (hipStreamCreateWithFlags(&pl->near, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&pl->near_ev, kSyncEv) != hipSuccess ||
      hipEventCreateWithFlags(&pl->fork_ev, kSyncEv) != hipSuccess ||
      hipEventCreateWithFlags(&pl->join_ev, kSyncEv) != hipSuccess ||
      hipStreamCreateWithFlags(&pl->gstream, hipStreamNonBlocking) != hipSuccess) {
    free_plan(pl);
    return FMM_ERR_DEVICE;
  }
  if (learned && (o.flags & FMM_JUDGE)) {
    fmm_options jo = o;
    jo.precision = FMM_FP64;
    jo.order_policy = FMM_ORDER_FIXED;
    jo.flags = o.flags & (FMM_NO_FIELD | FMM_AUTOTUNE);
    const int jr = fmm_plan(&jo, &pl->judge);
    if (jr != FMM_OK) {
      free_plan(pl);
      return jr;
    }
  }
  if ((o.flags & FMM_AUTOTUNE) && autotune_m2l(pl) != FMM_OK) {
    free_plan(pl);
    return FMM_ERR_DEVICE;
  }
  if (o.flags & (FMM_TIMING | FMM_TIMING_NEAR | FMM_TIMING_M2L)) {
    for (auto& r : pl->ev)
      for (auto& e : r)
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
          free_plan(pl);
          return FMM_ERR_DEVICE;
        }
    pl->have_events = true;
    pl->ev_mask = (o.flags & FMM_TIMING) ? 0xFFu
                  : ((o.flags & FMM_TIMING_NEAR) ? 0xC0u : 0u) | ((o.flags & FMM_TIMING_M2L) ? 0x0Cu : 0u);
  }
  *out = pl;
  return FMM_OK;
}

}  // extern "C"

namespace {

// Level table of a tree of depth L made of nsys stacked systems (offsets
// relative to the tree's own regions of the coefficient arrays).
LevelTable make_level_table(const fmm_plan_s* pl, int L, int nsys, int64_t* nbox64,
                            int64_t* nbox32) {
  return level_table(pl->dim, pl->f32, pl->opt.side, pl->opt.origin, L, nsys, nbox64, nbox32);
}

// One tree (or a stack of same-depth systems) over a sorted particle range.
struct TreeRun {
  LevelTable lt;
  int group = 0;                // row of the per-level order table
  int64_t p0 = 0, n = 0;        // sorted particle range
  int64_t leaf0 = 0;            // first leaf_start entry
  int64_t box64 = 0, box32 = 0; // first box in the FP64 / FP32 coefficient arrays
  int64_t part64 = 0, part32 = 0;
  bool leaves_done = false;     // the sort already wrote the leaf offsets
};

// Enqueues everything after the sort for one tree: leaf offsets, gather, then
// the near field on the near-field stream beside the moments and M2L on the
// caller's stream, the join, and local evaluation + unsort.
// io (batched graphs): the caller's buffers come from this device record,
// not from pos / q / pot / field.
void enqueue_tree(fmm_plan_s* pl, const TreeRun& t, const uint32_t* skeys, const int32_t* perm,
                  const double* pos, const double* q, double* pot, double* field, hipStream_t st,
                  hipEvent_t* ev, const float4* spts, const BatchIo* io = nullptr) {
  const LevelTable& lt = t.lt;
  const int64_t nleaf = (int64_t)lt.nsys << (pl->dim * lt.L);
  const uint32_t* keys = skeys + t.p0;
  const int32_t* pm = perm + t.p0;
  if (!t.leaves_done) launch_leaf_bounds(keys, t.n, nleaf, pl->leaf_start + t.leaf0, st);
  // FP32 modes: the sorted leaf-local records came with the sort (spts);
  // FP64 mode gathers the sorted coordinates and charges
  if (!pl->f32)
    launch_gather_f64(pl->dim, pos, q, pm, t.n, pl->xs + t.p0, pl->ys + t.p0,
                      pl->zs ? pl->zs + t.p0 : nullptr, pl->qs + t.p0, st, io);
  if (ev && (pl->ev_mask >> 1 & 1)) (void)hipEventRecord(ev[1], st);

  FmmArgs a{};
  a.lt = lt;
  a.p = pl->p;
  a.basis = pl->basis;
  a.m2l_mb = pl->m2l_mb;
  a.m2l_remap = pl->m2l_remap;
  a.ord_full = orders_full(pl) ? 1 : 0;
  a.ord = pl->d_ord + fmm_plan_s::kOrdCols * t.group;
  a.cs = pl->cs;
  a.n = t.n;
  a.keys = keys;
  a.leaf_start = pl->leaf_start + t.leaf0;
  a.perm = pm;
  if (!pl->f32) {
    a.xs = pl->xs + t.p0;
    a.ys = pl->ys + t.p0;
    a.zs = pl->zs ? pl->zs + t.p0 : nullptr;
    a.qs = pl->qs + t.p0;
  } else {
    a.pts = spts + t.p0;
  }
  a.mom64 = pl->mom64 + t.box64 * pl->cs;
  a.loc64 = pl->loc64 + t.box64 * pl->cs;
  a.mom32 = pl->mom32 + t.box32 * pl->cs;
  a.loc32 = pl->loc32 + t.box32 * pl->cs;
  a.part64 = pl->part64 + t.part64 * pl->cs;
  a.part32 = pl->part32 + t.part32 * pl->cs;
  a.op64 = pl->op64;
  a.op32 = pl->op32;
  a.opl64 = pl->opl64;
  a.opl32 = pl->opl32;
  a.op16 = reinterpret_cast<const __bf16*>(pl->op16);
  a.near_pot = pl->near_pot + t.p0;
  a.near_ex = pl->near_ex + t.p0;
  a.near_ey = pl->near_ey + t.p0;
  a.near_ez = pl->near_ez ? pl->near_ez + t.p0 : nullptr;
  a.m2l_part = pl->m2l_part;
  a.p2p_over = pl->p2p_over;
  a.pot = pot;
  a.field = field;
  a.io = io;
  if (pl->depth) {  // adaptive depth: every particle's leaf level first
    a.adapt_near = pl->opt.adaptive_near;
    launch_adapt_depth(a, pl->adapt_open, pl->depth, st);
    a.adapt_open = pl->adapt_open;
    a.depth = pl->depth;
  }
  const int hi64 = std::min(lt.L, lt.split - 1);
  FmmArgs a64 = a, a32 = a;
  a64.klo = lt.kmin;
  a64.khi = hi64;
  a32.klo = std::max(lt.split, lt.kmin);
  a32.khi = lt.L;
  // Two streams after the sort: the near-field stream runs the near field,
  // which needs only the sort and overlaps everything else; the caller's stream
  // runs the far field: in the FP32 modes first the small FP64 chain of level 2
  // (moments, then the contraction on the VALU, which leaves most of the chip to
  // the near field), then the main level range.  The local evaluation joins both.
  // (Measured slower, on a 1M-particle 2D FP32 evaluation at 0.34 ms: a third
  // stream for the level-2 chain (the extra overlap only adds contention with
  // the near field); forking after the moments, the near field beside the
  // contractions only (0.38 ms); the roles of the two streams swapped, the
  // near field on the caller's stream (0.36 ms: the moments chain then starts
  // late and finishes behind the near field); and shortening this chain by
  // appending the slice sums to later launches (0.36 ms: the main contraction
  // then starts beside the near field's last workgroups); both together, the
  // short moments chain forked and joined before the main contraction, came
  // out even on that workload and slower on the batched and clustered ones.)
  const bool lvl64 = pl->f32 && a64.khi >= a64.klo;
  (void)hipEventRecord(pl->fork_ev, st);
  (void)hipStreamWaitEvent(pl->near, pl->fork_ev, 0);
  if (ev && (pl->ev_mask >> 6 & 1)) (void)hipEventRecord(ev[6], pl->near);
  if (pl->dim == 2)
    launch_p2p2d(a, pl->f32, pl->near);
  else
    launch_p2p3d(a, pl->f32, pl->near);
  if (ev && (pl->ev_mask >> 7 & 1)) (void)hipEventRecord(ev[7], pl->near);
  (void)hipEventRecord(pl->near_ev, pl->near);
  FmmArgs& am = pl->f32 ? a32 : a64;  // the main level range
  if (pl->root) {
    // root frame (FP64): U-bar-1/U-bar-2 and the transfers into box frames,
    // the contraction, the transfers back and D-bar-2, then F(v)
    launch_root_upward(a64, pl->rbuf, st);
    if (ev && (pl->ev_mask >> 2 & 1)) (void)hipEventRecord(ev[2], st);
    launch_m2l3d(a64, true, st);
    if (ev && (pl->ev_mask >> 3 & 1)) (void)hipEventRecord(ev[3], st);
    launch_root_downward(a64, pl->rbuf, st);
    if (ev && (pl->ev_mask >> 4 & 1)) (void)hipEventRecord(ev[4], st);
    (void)hipStreamWaitEvent(st, pl->near_ev, 0);
    launch_root_eval(a, pl->rbuf, st);
    if (ev && (pl->ev_mask >> 5 & 1)) (void)hipEventRecord(ev[5], st);
    return;
  }
  if (pl->dim == 2 && pl->basis) {
    if (lvl64) launch_p2m2d_points(a64, true, true, st);
    launch_p2m2d_points(am, pl->f32, !pl->f32, st);
  } else if (pl->dim == 2) {
    if (lvl64) launch_p2m2d(a64, true, true, st);
    launch_p2m2d(am, pl->f32, !pl->f32, st);
  } else if (pl->basis && pl->p != 4) {
    if (lvl64) launch_p2m3d_points(a64, true, true, st);
    launch_p2m3d_points(am, pl->f32, !pl->f32, st);
  } else {
    if (lvl64) launch_p2m3d(a64, true, true, st);
    launch_p2m3d(am, pl->f32, !pl->f32, st);
  }
  if (lvl64) {
    if (pl->dim == 2 && pl->basis)
      launch_m2l2d_points(a64, true, st);
    else if (pl->dim == 2)
      launch_m2l2d(a64, true, st);
    else
      launch_m2l3d(a64, true, st);
  }
  if (ev && (pl->ev_mask >> 2 & 1)) (void)hipEventRecord(ev[2], st);
  // the main M2L launch (all levels in FP64 mode, levels >= 3 in FP32 modes)
  // is bracketed by events 2 and 3 on the caller's stream
  if (pl->dim == 2 && pl->basis)
    launch_m2l2d_points(am, !pl->f32, st);
  else if (pl->dim == 2)
    launch_m2l2d(am, !pl->f32, st, pl->prec == FMM_BF16_M2L);
  else
    launch_m2l3d(am, !pl->f32, st);
  if (ev && (pl->ev_mask >> 3 & 1)) (void)hipEventRecord(ev[3], st);
  if (ev && (pl->ev_mask >> 4 & 1)) (void)hipEventRecord(ev[4], st);
  (void)hipStreamWaitEvent(st, pl->near_ev, 0);
  if (pl->dim == 2 && pl->basis)
    launch_l2p2d_points(a, pl->f32, st);
  else if (pl->dim == 2)
    launch_l2p2d(a, pl->f32, st);
  else if (pl->basis && pl->p != 4)
    launch_l2p3d_points(a, pl->f32, st);
  else
    launch_l2p3d(a, pl->f32, st);
  if (ev && (pl->ev_mask >> 5 & 1)) (void)hipEventRecord(ev[5], st);
}

// ----- M2L autotuner (2D) -----
// Candidates: tile height MB in {1, 2, 3, 4, 8} (8 x 8 MB targets per workgroup,
// operator loads shared by MB blocks of 16 targets) x XCD-contiguous tile order
// on / off, where compiled and within the LDS.  Each candidate runs the plan's
// main M2L launch once to warm up and then five times, each between HIP events
// on a private stream; the candidate with the fastest launch is kept.  Results
// are cached per process, keyed by (dimension, order bucket and basis,
// precision, finest level, first and last level of the launch); when the
// environment variable FMM_AUTOTUNE_CACHE names a file, the cache is also read
// from and written to that file as JSON (one entry per tuned shape, with the
// device architecture), so later processes skip the timing.
std::mutex g_tune_mu;
std::map<std::array<int, 6>, std::array<float, 3>> g_tune;
std::string g_tune_loaded;  // the cache file already read into g_tune

std::string device_arch(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// Reads entries of this architecture from the JSON cache file (lock held).
void tune_cache_read(const std::string& path, const std::string& arch) {
  if (g_tune_loaded == path) return;
  g_tune_loaded = path;
  FILE* fh = std::fopen(path.c_str(), "r");
  if (!fh) return;
  char line[512];
  while (std::fgets(line, sizeof(line), fh)) {
    char a[64] = {0};
    int k[6], mb = 0, rm = 0;
    float ms = 0.f;
    if (std::sscanf(line,
                    " {\"arch\": \"%63[^\"]\", \"key\": [%d, %d, %d, %d, %d, %d], "
                    "\"tile_mb\": %d, \"xcd_remap\": %d, \"ms\": %f}",
                    a, &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &mb, &rm, &ms) == 10 &&
        arch == a)
      g_tune[{k[0], k[1], k[2], k[3], k[4], k[5]}] = {(float)mb, (float)rm, ms};
  }
  std::fclose(fh);
}

// Writes every cached entry (lock held); the file is replaced as a whole.
void tune_cache_write(const std::string& path, const std::string& arch) {
  const std::string tmp = path + ".tmp";
  FILE* fh = std::fopen(tmp.c_str(), "w");
  if (!fh) return;
  std::fprintf(fh, "{\"m2l_autotune\": [\n");
  size_t i = 0;
  for (const auto& e : g_tune) {
    const auto& k = e.first;
    std::fprintf(fh,
                 " {\"arch\": \"%s\", \"key\": [%d, %d, %d, %d, %d, %d], \"tile_mb\": %d, "
                 "\"xcd_remap\": %d, \"ms\": %.6f}%s\n",
                 arch.c_str(), k[0], k[1], k[2], k[3], k[4], k[5], (int)e.second[0],
                 (int)e.second[1], e.second[2], ++i < g_tune.size() ? "," : "");
  }
  std::fprintf(fh, "]}\n");
  std::fclose(fh);
  std::rename(tmp.c_str(), path.c_str());
}

int autotune_m2l(fmm_plan_s* pl) {
  if (pl->dim == 2 && pl->basis) return FMM_OK;  // one contraction kernel, nothing to choose
  const LevelTable& lt = pl->lt;
  const bool fp64 = !pl->f32;
  const int klo = fp64 ? lt.kmin : std::max(lt.split, lt.kmin), khi = lt.L;
  if (khi < klo) return FMM_OK;
  const std::array<int, 6> key = {pl->dim, pl->pb + 100 * pl->basis, pl->prec, lt.L, klo, khi};
  const char* cache_env = std::getenv("FMM_AUTOTUNE_CACHE");
  const std::string cache_path = cache_env ? cache_env : "";
  const std::string arch = device_arch(pl->device);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!cache_path.empty()) tune_cache_read(cache_path, arch);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      pl->m2l_mb = (int)it->second[0];
      pl->m2l_remap = (int)it->second[1];
      pl->m2l_tuned_ms = it->second[2];
      return FMM_OK;
    }
  }
  FmmArgs a{};
  a.lt = lt;
  a.p = pl->p;
  a.basis = pl->basis;
  a.cs = pl->cs;
  a.ord = pl->d_ord;
  a.ord_full = orders_full(pl) ? 1 : 0;
  a.klo = klo;
  a.khi = khi;
  a.mom64 = pl->mom64;
  a.loc64 = pl->loc64;
  a.mom32 = pl->mom32;
  a.loc32 = pl->loc32;
  a.op64 = pl->op64;
  a.op32 = pl->op32;
  a.opl64 = pl->opl64;
  a.opl32 = pl->opl32;
  a.op16 = reinterpret_cast<const __bf16*>(pl->op16);
  a.m2l_part = pl->m2l_part;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return FMM_ERR_DEVICE;
  float best = 1e30f;
  int bmb = 1, brm = 1;
  const bool bf16 = pl->prec == FMM_BF16_M2L;
  auto launch = [&](hipStream_t st) {
    if (pl->dim == 2)
      launch_m2l2d(a, fp64, st, bf16);
    else
      launch_m2l3d(a, fp64, st);
  };
  for (int mb : {1, 2, 3, 4, 8}) {
    if (pl->dim == 2 ? !m2l2d_variant_ok(mb, fp64, pl->pb, bf16) : !m2l3d_variant_ok(mb, fp64))
      continue;
    for (int rm : {1, 0}) {
      if (pl->dim == 3 && rm == 0) continue;  // 3D tiles are always dealt per XCD
      a.m2l_mb = mb;
      a.m2l_remap = rm;
      launch(s);
      float ms = 1e30f;
      for (int r = 0; r < 5; ++r) {  // the fastest of five single launches
        float t = 0.f;
        (void)hipEventRecord(e0, s);
        launch(s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
          break;
        ms = std::min(ms, t);
      }
      if (ms < best) {
        best = ms;
        bmb = mb;
        brm = rm;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (hipGetLastError() != hipSuccess) return FMM_ERR_DEVICE;
  pl->m2l_mb = bmb;
  pl->m2l_remap = brm;
  pl->m2l_tuned_ms = best;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = {(float)bmb, (float)brm, best};
  if (!cache_path.empty()) tune_cache_write(cache_path, arch);
  return FMM_OK;
}

// Whether every level runs at the layout bucket's order (fixed orders known on
// the host), which lets the 2D contraction drop its per-level guards.
bool orders_full(const fmm_plan_s* pl) {
  if (pl->learned && pl->have_model) return false;
  for (int k = 2; k <= pl->lcap && k < 16; ++k)
    if (pl->h_ord[k] != pl->pb) return false;
  return true;
}

// log10 of the truncation budget of the learned order (the whole tolerance in
// FP64 mode, half of it in the reduced-precision modes).
float order_budget_log10(const fmm_plan_s* pl) {
  return (float)std::log10(pl->f32 ? 0.5 * pl->opt.tol : pl->opt.tol);
}

void ring_advance(fmm_plan_s* pl) {
  pl->ring_next = (pl->ring_next + 1) % fmm_plan_s::kRing;
  if (pl->ring_count < fmm_plan_s::kRing) ++pl->ring_count;
}

}  // namespace

extern "C" {

int fmm_eval(fmm_plan_t pl, int64_t n, const double* pos, const double* q, double* pot,
             double* field, void* stream) {
  if (!pl) return FMM_ERR_INVALID_ARG;
  if (n < 0 || n > pl->maxn) return FMM_ERR_INVALID_ARG;
  const bool want_field = !(pl->opt.flags & FMM_NO_FIELD);
  if (n > 0 && (!pos || !q || !pot || (want_field && !field))) return FMM_ERR_INVALID_ARG;
  if (!want_field) field = nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipSetDevice(pl->device) != hipSuccess) return FMM_ERR_DEVICE;
  pl->last_stream = st;
  pl->last_n = n;
  pl->last_batched = false;
  pl->tag = pl->tag % 0x3FFFFFFF + 1;  // never 0 (the words' first value) nor kGraphTag
  if (n == 0) return FMM_OK;
  const bool timing = pl->have_events;
  hipEvent_t* ev = timing ? pl->ev[pl->ring_next] : nullptr;
  if (timing && (pl->ev_mask & 1)) (void)hipEventRecord(ev[0], st);

  const int bits = pl->dim * pl->L;
  const bool two_digit = pl->radix_parts && radix_two_digit(n, bits);
  launch_bin(pl->dim, pos, n, pl->lt, pl->keys, pl->vals, pl->flag, pl->tag, pl->hist, st, q,
             pl->f32 ? pl->pts : nullptr, two_digit ? 8 : 0);
  int which = 0;
  if (two_digit)
    radix_sort_two_digit(pl->keys, pl->vals, pl->keys_alt, pl->vals_alt, n, bits, pl->hist,
                         pl->radix_tot, pl->leaf_start, (int64_t)1 << bits, pl->radix_parts, st,
                         pl->f32 ? pl->pts : nullptr, pl->f32 ? pl->pts_alt : nullptr);
  else
    which = radix_sort(pl->keys, pl->vals, pl->keys_alt, pl->vals_alt, n, bits, pl->hist,
                       pl->radix_tot, st, true, pl->f32 ? pl->pts : nullptr,
                       pl->f32 ? pl->pts_alt : nullptr);
  const float4* spts = pl->f32 ? (which ? pl->pts_alt : pl->pts) : nullptr;
  const uint32_t* skeys = which ? pl->keys_alt : pl->keys;
  const int32_t* perm = which ? pl->vals_alt : pl->vals;
  pl->sorted_keys = skeys;
  pl->perm = perm;
  const bool use_model = pl->learned && pl->have_model;
  if (use_model) {
    // order selection: one system over the whole sorted range; its record
    // goes to the device as a kernel argument (slot max_systems, apart from
    // the batched table)
    const int nblk = (int)((n + order_chunk() - 1) / order_chunk());
    OrderSys* one = pl->d_ordsys + std::max(pl->opt.max_systems, 1);
    launch_set_ordsys(one, OrderSys{0, (int32_t)n, pl->L, 0, 0, nblk, 0, 0}, st);
    launch_fill_i32(pl->d_ord, 0, (int64_t)fmm_plan_s::kOrdRows * fmm_plan_s::kOrdCols, st);
    launch_order_select(one, 1, nblk, skeys, perm, q, pl->L, pl->d_mlp, pl->d_pq, pl->d_pcnt,
                        order_budget_log10(pl), pl->d_ord, fmm_plan_s::kOrdCols, pl->d_feat, st);
    pl->last_nsys = 1;
  }
  TreeRun t;
  t.lt = pl->lt;
  t.n = n;
  t.leaves_done = two_digit;
  enqueue_tree(pl, t, skeys, perm, pos, q, pot, field, st, ev, spts);
  if (timing) {
    pl->ring_batched[pl->ring_next] = false;
    ring_advance(pl);
  }
  if (use_model && pl->judge) {
    // the fixed-order FP64 result judges the learned one
    const int jr = fmm_eval(pl->judge, n, pos, q, pl->jpot, field ? pl->jfield : nullptr, stream);
    if (jr < 0) return jr;
    launch_judge(pot, field, pl->jpot, pl->jfield, n, pl->dim, nullptr, 1, pl->opt.tol, pl->flag,
                 pl->tag, pl->jerr, st);
  }
  if (hipGetLastError() != hipSuccess) return FMM_ERR_DEVICE;
  int ret = FMM_OK;
  if (pl->opt.flags & FMM_SYNC_CHECK) ret = fmm_last_status(pl);
  if (ret == FMM_OK && pl->learned && !pl->have_model) ret = FMM_WARN_FALLBACK;
  return ret;
}

}  // extern "C"

namespace {
// After a setting that the captured batched graph depends on (orders, tile
// variant, order model) has changed: capture the prepared shape again.
int reprepare(fmm_plan_s* pl) {
  if (!pl->prepared) return FMM_OK;
  pl->prepared = false;
  const std::vector<int64_t> off = pl->prep_off;
  const std::vector<int32_t> depth = pl->prep_depth;
  return fmm_batch_prepare(pl, pl->prep_nsys, off.data(), depth.data());
}
}  // namespace

extern "C" {

int fmm_batch_prepare(fmm_plan_t pl, int32_t nsys, const int64_t* sys_offsets,
                      const int32_t* sys_levels) {
  if (!pl || !sys_offsets) return FMM_ERR_INVALID_ARG;
  if (pl->dim != 2 || pl->opt.max_systems <= 1) return FMM_ERR_UNSUPPORTED;
  if (nsys < 0 || nsys > pl->opt.max_systems) return FMM_ERR_INVALID_ARG;
  if (nsys > 0 && sys_offsets[0] != 0) return FMM_ERR_INVALID_ARG;
  for (int s = 0; s < nsys; ++s)
    if (sys_offsets[s + 1] < sys_offsets[s]) return FMM_ERR_INVALID_ARG;
  const int64_t n = nsys > 0 ? sys_offsets[nsys] : 0;
  if (n > pl->maxn) return FMM_ERR_INVALID_ARG;
  const int lmax = pl->lcap;
  // depths: given, or clamp(round(log4(n_s / 16)), 2, lmax)
  std::vector<int32_t> depth(nsys);
  for (int s = 0; s < nsys; ++s) {
    int L;
    if (sys_levels) {
      L = sys_levels[s];
    } else {
      const double ns = (double)(sys_offsets[s + 1] - sys_offsets[s]);
      L = ns > 0 ? (int)std::lround(std::log(ns / 16.0) / std::log(4.0)) : 2;
      L = std::min(std::max(L, 2), lmax);
    }
    if (L < 0 || L > lmax) return FMM_ERR_INVALID_ARG;
    depth[s] = L;
  }
  const bool use_model = pl->learned && pl->have_model;
  std::vector<int64_t> off(sys_offsets, sys_offsets + nsys + 1);
  if (pl->prepared && pl->graph_exec && nsys == pl->prep_nsys && off == pl->prep_off &&
      depth == pl->prep_depth && use_model == pl->prep_model)
    return FMM_OK;  // this shape's graph is ready
  if (hipSetDevice(pl->device) != hipSuccess) return FMM_ERR_DEVICE;
  // the sort key scales every Morton code to the deepest system of the call
  // (fewer key bits: fewer radix passes than scaling to the plan's limit)
  int kl = 0;
  for (int s = 0; s < nsys; ++s) kl = std::max(kl, depth[s]);
  // order systems by (depth, index); groups of equal depth are stacked trees
  std::vector<int> order(nsys);
  for (int s = 0; s < nsys; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return depth[x] < depth[y]; });
  std::vector<int32_t> info(2 * (size_t)std::max(nsys, 1));
  for (int r = 0; r < nsys; ++r) {
    info[2 * order[r]] = r;
    info[2 * order[r] + 1] = depth[order[r]];
  }
  // order-selection table in sorted (rank) order: sorted start, size, depth,
  // depth-group row, chunk blocks, system index
  std::vector<OrderSys> osys;
  int total_blocks = 0;
  if (use_model) {
    int64_t acc = 0;
    for (int r = 0; r < nsys; ++r) {
      const int s = order[r];
      const int64_t ns = sys_offsets[s + 1] - sys_offsets[s];
      const int nb = (int)((ns + order_chunk() - 1) / order_chunk());
      osys.push_back(OrderSys{(int32_t)acc, (int32_t)ns, depth[s], depth[s], total_blocks, nb, s, 0});
      acc += ns;
      total_blocks += nb;
    }
  }
  std::vector<TreeRun> runs;
  std::vector<int> run_r0;
  int64_t p0 = 0, leaf0 = 0, box64 = 0, box32 = 0, part64 = 0, part32 = 0;
  for (int r = 0; r < nsys;) {
    const int L = depth[order[r]];
    int r1 = r;
    int64_t ng = 0;
    while (r1 < nsys && depth[order[r1]] == L) {
      ng += sys_offsets[order[r1] + 1] - sys_offsets[order[r1]];
      ++r1;
    }
    TreeRun t;
    int64_t nb64 = 0, nb32 = 0;
    t.lt = make_level_table(pl, L, r1 - r, &nb64, &nb32);
    t.group = L;  // one depth group per depth
    t.p0 = p0;
    t.n = ng;
    t.leaf0 = leaf0;
    t.box64 = box64;
    t.box32 = box32;
    t.part64 = part64;
    t.part32 = part32;
    p0 += ng;
    leaf0 += ((int64_t)(r1 - r) << (2 * L)) + 1;
    box64 += nb64;
    box32 += nb32;
    part64 += (int64_t)p2m_partial_rows(2, 2, std::min(L, t.lt.split - 1), ng, r1 - r);
    part32 += (int64_t)p2m_partial_rows(2, std::max(t.lt.split, 2), L, ng, r1 - r);
    if (ng > 0) {
      runs.push_back(t);
      run_r0.push_back(r);
    }
    r = r1;
  }
  if (leaf0 > pl->leaf_cap || box64 > pl->nbox64 || box32 > pl->nbox32 ||
      part64 * pl->cs >= (int64_t)pl->part64_cap || part32 * pl->cs >= (int64_t)pl->part32_cap)
    return FMM_ERR_INVALID_ARG;

  // plan-time work from here: wait for the plan's streams (an earlier replay
  // may still read the tables), upload the tables, capture and instantiate
  hipStream_t gs = pl->gstream;
  if (hipStreamSynchronize(gs) != hipSuccess) return FMM_ERR_DEVICE;
  if (pl->last_stream && hipStreamSynchronize(pl->last_stream) != hipSuccess)
    (void)hipGetLastError();  // the judge's reads; a stream the caller has since destroyed
  pl->prepared = false;
  if (pl->graph_exec) {
    (void)hipGraphExecDestroy(pl->graph_exec);
    pl->graph_exec = nullptr;
  }
  if (nsys > 0 &&
      (hipMemcpy(pl->d_sysoff, off.data(), sizeof(int64_t) * (size_t)(nsys + 1),
                 hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(pl->d_sysinfo, info.data(), sizeof(int32_t) * 2 * (size_t)nsys,
                 hipMemcpyHostToDevice) != hipSuccess ||
       (use_model && hipMemcpy(pl->d_ordsys, osys.data(), sizeof(OrderSys) * (size_t)nsys,
                               hipMemcpyHostToDevice) != hipSuccess)))
    return FMM_ERR_DEVICE;
  if (hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return FMM_ERR_DEVICE;
  // the graph clears the first two status words; the third is the argument
  // check of fmm_eval_batched, written before every replay
  launch_fill_i32(pl->flag, 0, 2, gs);
  const BatchIo* io = pl->d_io;
  if (n > 0) {
    launch_bin_batched(nullptr, n, pl->d_sysoff, nsys, pl->d_sysinfo, pl->lt, kl, pl->keys,
                       pl->vals, pl->flag, fmm_plan_s::kGraphTag, pl->hist, gs, nullptr,
                       pl->f32 ? pl->pts : nullptr, io);
    int rbits = 0;
    while ((1 << rbits) < nsys) ++rbits;
    const int which = radix_sort(pl->keys, pl->vals, pl->keys_alt, pl->vals_alt, n,
                                 rbits + 2 * kl, pl->hist, pl->radix_tot, gs, true,
                                 pl->f32 ? pl->pts : nullptr, pl->f32 ? pl->pts_alt : nullptr);
    const float4* spts = pl->f32 ? (which ? pl->pts_alt : pl->pts) : nullptr;
    uint32_t* skeys = which ? pl->keys_alt : pl->keys;
    const int32_t* perm = which ? pl->vals_alt : pl->vals;
    pl->graph_keys = skeys;
    pl->graph_perm = perm;
    if (use_model) {
      launch_fill_i32(pl->d_ord, 0, (int64_t)fmm_plan_s::kOrdRows * fmm_plan_s::kOrdCols, gs);
      launch_order_select(pl->d_ordsys, nsys, total_blocks, skeys, perm, nullptr, kl, pl->d_mlp,
                          pl->d_pq, pl->d_pcnt, order_budget_log10(pl), pl->d_ord,
                          fmm_plan_s::kOrdCols, pl->d_feat, gs, io);
    }
    for (size_t g = 0; g < runs.size(); ++g) {
      launch_rekey(skeys + runs[g].p0, runs[g].n, run_r0[g], runs[g].lt.L, kl, gs);
      enqueue_tree(pl, runs[g], skeys, perm, nullptr, nullptr, nullptr, nullptr, gs, nullptr,
                   spts, io);
    }
  }
  hipGraph_t graph = nullptr;
  if (hipStreamEndCapture(gs, &graph) != hipSuccess || !graph) return FMM_ERR_DEVICE;
  const hipError_t ie = hipGraphInstantiate(&pl->graph_exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    pl->graph_exec = nullptr;
    return FMM_ERR_DEVICE;
  }
  ++pl->graph_builds;
  if (pl->judge) {  // the judge's fixed-order plan runs the same shape
    const int jr = fmm_batch_prepare(pl->judge, nsys, sys_offsets, depth.data());
    if (jr != FMM_OK) return jr;
  }
  pl->prepared = true;
  pl->prep_nsys = nsys;
  pl->prep_n = n;
  pl->prep_off = off;
  pl->prep_depth = depth;
  pl->prep_model = use_model;
  if (use_model) pl->last_nsys = nsys;
  return FMM_OK;
}

int fmm_eval_batched(fmm_plan_t pl, int32_t nsys, const int64_t* sys_offsets,
                     const int32_t* sys_levels, const double* pos, const double* q, double* pot,
                     double* field, void* stream) {
  if (!pl || !sys_offsets) return FMM_ERR_INVALID_ARG;
  if (pl->dim != 2 || pl->opt.max_systems <= 1) return FMM_ERR_UNSUPPORTED;
  if (!pl->prepared || !pl->graph_exec || nsys != pl->prep_nsys) return FMM_ERR_INVALID_ARG;
  if ((pl->learned && pl->have_model) != pl->prep_model) return FMM_ERR_INVALID_ARG;
  const int64_t n = pl->prep_n;
  const bool want_field = !(pl->opt.flags & FMM_NO_FIELD);
  if (n > 0 && (!pos || !q || !pot || (want_field && !field))) return FMM_ERR_INVALID_ARG;
  if (!want_field) field = nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipSetDevice(pl->device) != hipSuccess) return FMM_ERR_DEVICE;
  pl->last_stream = st;
  pl->last_n = n;
  pl->last_batched = true;
  pl->tag = fmm_plan_s::kGraphTag;
  const bool timing = pl->have_events;
  hipEvent_t* ev = timing ? pl->ev[pl->ring_next] : nullptr;
  hipStream_t gs = pl->gstream;
  (void)hipEventRecord(pl->fork_ev, st);
  (void)hipStreamWaitEvent(gs, pl->fork_ev, 0);
  if (timing && (pl->ev_mask & 1)) (void)hipEventRecord(ev[0], gs);
  // the caller's buffers into the graph's record; the caller's device tables
  // checked against the prepared shape (status word 2)
  launch_batch_begin(pl->d_io, pos, q, pot, field, sys_offsets, sys_levels, pl->d_sysoff,
                     pl->d_sysinfo, nsys, pl->lcap, pl->flag, fmm_plan_s::kGraphTag, gs);
  if (hipGraphLaunch(pl->graph_exec, gs) != hipSuccess) return FMM_ERR_DEVICE;
  pl->sorted_keys = pl->graph_keys;
  pl->perm = pl->graph_perm;
  if (timing) {
    // the phases inside the graph are not separable: only the total is kept
    for (int i = 1; i < 8; ++i)
      if (pl->ev_mask >> i & 1) (void)hipEventRecord(ev[i], gs);
    pl->ring_batched[pl->ring_next] = true;
    ring_advance(pl);
  }
  (void)hipEventRecord(pl->join_ev, gs);
  (void)hipStreamWaitEvent(st, pl->join_ev, 0);
  if (pl->prep_model && pl->judge) {
    const int jr = fmm_eval_batched(pl->judge, nsys, sys_offsets, sys_levels, pos, q, pl->jpot,
                                    field ? pl->jfield : nullptr, stream);
    if (jr < 0) return jr;
    launch_judge(pot, field, pl->jpot, pl->jfield, n, 2, pl->d_sysoff, nsys, pl->opt.tol,
                 pl->flag, pl->tag, pl->jerr, st);
  }
  if (hipGetLastError() != hipSuccess) return FMM_ERR_DEVICE;
  int ret = FMM_OK;
  if (pl->opt.flags & FMM_SYNC_CHECK) ret = fmm_last_status(pl);
  if (ret == FMM_OK && pl->learned && !pl->have_model) ret = FMM_WARN_FALLBACK;
  return ret;
}

int fmm_set_level_orders(fmm_plan_t pl, const int32_t* orders, int32_t count) {
  if (!pl || !orders) return FMM_ERR_INVALID_ARG;
  if (pl->dim != 2 || pl->learned) return FMM_ERR_UNSUPPORTED;
  if (count != pl->lcap + 1) return FMM_ERR_INVALID_ARG;
  for (int k = 2; k < count; ++k)
    if (orders[k] < 1 || orders[k] > pl->p) return FMM_ERR_INVALID_ARG;
  if (hipSetDevice(pl->device) != hipSuccess) return FMM_ERR_DEVICE;
  // the previous evaluation may still read the table
  if (hipStreamSynchronize(pl->last_stream) != hipSuccess) return FMM_ERR_DEVICE;
  for (int k = 0; k < fmm_plan_s::kOrdCols; ++k) pl->h_ord[k] = (k >= 2 && k < count) ? orders[k] : 0;
  const int rc = upload_orders(pl);
  // the captured batched graph chose its kernels for the old orders: capture
  // the prepared shape again
  return rc == FMM_OK ? reprepare(pl) : rc;
}

int fmm_set_order_model(fmm_plan_t pl, const float* w, int64_t n) {
  if (!pl || !w) return FMM_ERR_INVALID_ARG;
  if (!pl->learned) return FMM_ERR_UNSUPPORTED;
  if (n != FMM_MLP_NPARAM) return FMM_ERR_INVALID_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(w[i])) return FMM_ERR_INVALID_ARG;
  if (hipSetDevice(pl->device) != hipSuccess) return FMM_ERR_DEVICE;
  if (hipStreamSynchronize(pl->last_stream) != hipSuccess) return FMM_ERR_DEVICE;
  if (hipMemcpy(pl->d_mlp, w, sizeof(float) * (size_t)n, hipMemcpyHostToDevice) != hipSuccess)
    return FMM_ERR_DEVICE;
  pl->have_model = true;
  // a prepared batched graph without the order selection: capture it again
  return reprepare(pl);
}

int fmm_mlp_forward(const float* w, const float* x, int64_t m, float* y, void* stream) {
  if (m < 0 || (m > 0 && (!w || !x || !y))) return FMM_ERR_INVALID_ARG;
  launch_mlp_forward(w, x, m, y, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FMM_OK : FMM_ERR_DEVICE;
}

namespace {
struct MlpScratch {
  float* part = nullptr;
  double* part_loss = nullptr;
  int alloc(int64_t m) {
    const int64_t nw = (mlp_grad_waves(m) + 3) / 4 * 4 + 4;
    if (hipMalloc(&part, sizeof(float) * (size_t)nw * FMM_MLP_NPARAM) != hipSuccess ||
        hipMalloc(&part_loss, sizeof(double) * (size_t)nw) != hipSuccess) {
      (void)hipGetLastError();
      return FMM_ERR_NOMEM;
    }
    return FMM_OK;
  }
  ~MlpScratch() {
    if (part || part_loss) (void)hipDeviceSynchronize();
    if (part) (void)hipFree(part);
    if (part_loss) (void)hipFree(part_loss);
  }
};
}  // namespace

int fmm_mlp_loss_grad(const float* w, const float* x, const float* t, int64_t m, float* grad,
                      float* loss, void* stream) {
  if (m < 0 || !w || !grad || (m > 0 && (!x || !t))) return FMM_ERR_INVALID_ARG;
  MlpScratch sc;
  if (sc.alloc(m) != FMM_OK) return FMM_ERR_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  launch_mlp_grad(w, x, t, m, sc.part, sc.part_loss, grad, loss, st);
  if (hipGetLastError() != hipSuccess) return FMM_ERR_DEVICE;
  return hipStreamSynchronize(st) == hipSuccess ? FMM_OK : FMM_ERR_DEVICE;
}

int fmm_mlp_adam_step(float* w, const float* grad, float* m1, float* m2, int32_t step, float lr,
                      void* stream) {
  if (!w || !grad || !m1 || !m2 || step < 1 || !(lr > 0)) return FMM_ERR_INVALID_ARG;
  launch_mlp_adam(w, grad, m1, m2, step, lr, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FMM_OK : FMM_ERR_DEVICE;
}

int fmm_mlp_train(float* w, const float* x, const float* t, int64_t m, int32_t steps, float lr,
                  float* loss_history, void* stream) {
  if (!w || m <= 0 || !x || !t || steps < 0 || !(lr > 0)) return FMM_ERR_INVALID_ARG;
  MlpScratch sc;
  if (sc.alloc(m) != FMM_OK) return FMM_ERR_NOMEM;
  float *grad = nullptr, *m1 = nullptr, *m2 = nullptr, *losses = nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = FMM_OK;
  if (hipMalloc(&grad, sizeof(float) * FMM_MLP_NPARAM) != hipSuccess ||
      hipMalloc(&m1, sizeof(float) * FMM_MLP_NPARAM) != hipSuccess ||
      hipMalloc(&m2, sizeof(float) * FMM_MLP_NPARAM) != hipSuccess ||
      hipMalloc(&losses, sizeof(float) * (size_t)(steps > 0 ? steps : 1)) != hipSuccess) {
    (void)hipGetLastError();
    rc = FMM_ERR_NOMEM;
  }
  if (rc == FMM_OK) {
    launch_fill_i32(reinterpret_cast<int32_t*>(m1), 0, FMM_MLP_NPARAM, st);  // +0.0f
    launch_fill_i32(reinterpret_cast<int32_t*>(m2), 0, FMM_MLP_NPARAM, st);
    for (int s = 1; s <= steps; ++s) {
      launch_mlp_grad(w, x, t, m, sc.part, sc.part_loss, grad, losses + (s - 1), st);
      launch_mlp_adam(w, grad, m1, m2, s, lr, st);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      rc = FMM_ERR_DEVICE;
    else if (loss_history && steps > 0 &&
             hipMemcpy(loss_history, losses, sizeof(float) * (size_t)steps,
                       hipMemcpyDeviceToHost) != hipSuccess)
      rc = FMM_ERR_DEVICE;
  }
  (void)hipStreamSynchronize(st);
  if (grad) (void)hipFree(grad);
  if (m1) (void)hipFree(m1);
  if (m2) (void)hipFree(m2);
  if (losses) (void)hipFree(losses);
  return rc;
}

int fmm_set_m2l_variant(fmm_plan_t pl, int32_t tile_mb, int32_t xcd_remap) {
  if (!pl || (xcd_remap != 0 && xcd_remap != 1)) return FMM_ERR_INVALID_ARG;
  if (pl->dim == 2 && pl->basis) return FMM_ERR_UNSUPPORTED;  // one contraction kernel
  if (pl->dim == 2 ? !m2l2d_variant_ok(tile_mb, !pl->f32, pl->pb, pl->prec == FMM_BF16_M2L)
                   : (!m2l3d_variant_ok(tile_mb, !pl->f32) || xcd_remap != 1))
    return FMM_ERR_INVALID_ARG;
  pl->m2l_mb = tile_mb;
  pl->m2l_remap = xcd_remap;
  // the captured batched graph holds the old variant: capture the prepared
  // shape again
  return reprepare(pl);
}

int fmm_last_status(fmm_plan_t pl) {
  if (!pl) return FMM_ERR_INVALID_ARG;
  if (hipSetDevice(pl->device) != hipSuccess) return FMM_ERR_DEVICE;
  int32_t f[3] = {0, 0, 0};
  if (hipStreamSynchronize(pl->last_stream) != hipSuccess) return FMM_ERR_DEVICE;
  if (hipMemcpy(f, pl->flag, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess)
    return FMM_ERR_DEVICE;
  // word 2: a batched call's device tables differed from the prepared shape
  if (pl->last_batched && f[2] == pl->tag) return FMM_ERR_INVALID_ARG;
  return f[0] == pl->tag ? FMM_ERR_DOMAIN : f[1] == pl->tag ? FMM_WARN_FALLBACK : FMM_OK;
}

int fmm_get_stats(fmm_plan_t pl, fmm_stats* out) {
  if (!pl || !out) return FMM_ERR_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  for (int k = 0; k <= pl->lcap && k < 16; ++k) out->order_per_level[k] = pl->h_ord[k];
  out->m2l_launches = (pl->nbox64 > 0 ? 1 : 0) + (pl->nbox32 > 0 ? 1 : 0);
  out->m2l_tile_mb = pl->m2l_mb;
  out->m2l_xcd_remap = pl->dim == 2 ? pl->m2l_remap : 1;
  out->m2l_tuned_ms = pl->m2l_tuned_ms;
  out->graph_builds = pl->graph_builds;
  if (pl->learned) {
    if (hipSetDevice(pl->device) != hipSuccess) return FMM_ERR_DEVICE;
    if (hipStreamSynchronize(pl->last_stream) != hipSuccess) return FMM_ERR_DEVICE;
    int32_t f[2] = {0, 0};
    if (hipMemcpy(f, pl->flag, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess)
      return FMM_ERR_DEVICE;
    out->fallback = (!pl->have_model || f[1] == pl->tag) ? 1 : 0;
    if (pl->have_model) {
      // the orders used: largest over the depth groups per level
      std::vector<int32_t> rows((size_t)fmm_plan_s::kOrdRows * fmm_plan_s::kOrdCols);
      if (hipMemcpy(rows.data(), pl->d_ord, rows.size() * sizeof(int32_t),
                    hipMemcpyDeviceToHost) != hipSuccess)
        return FMM_ERR_DEVICE;
      for (int k = 0; k < 16; ++k) {
        int32_t m = 0;
        for (int r = 0; r < fmm_plan_s::kOrdRows; ++r)
          m = std::max(m, rows[(size_t)r * fmm_plan_s::kOrdCols + k]);
        out->order_per_level[k] = m;
      }
    }
    if (pl->jerr &&
        hipMemcpy(&out->judge_rel_err, pl->jerr, sizeof(double), hipMemcpyDeviceToHost) !=
            hipSuccess)
      return FMM_ERR_DEVICE;
  }
  if (!pl->have_events || pl->ring_count == 0) return FMM_OK;
  const int cnt = pl->ring_count;
  const int last = (pl->ring_next + fmm_plan_s::kRing - 1) % fmm_plan_s::kRing;
  for (int e = 0; e < 8; ++e)
    if ((pl->ev_mask >> e & 1) && hipEventSynchronize(pl->ev[last][e]) != hipSuccess)
      return FMM_ERR_DEVICE;
  // phase: (from, to) event pairs; the near field runs on its own stream and
  // overlaps the far-field phases, so the phases do not add up to the total.
  static const int from[7] = {0, 1, 2, 4, 6, 0, 2}, to[7] = {1, 2, 4, 5, 7, 5, 3};
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int r = 0; r < cnt; ++r) {
    const int slot = (last + fmm_plan_s::kRing - r) % fmm_plan_s::kRing;
    for (int i = 0; i < 7; ++i) {
      // a batched evaluation is one graph: its total is timed, its phases are not
      if (pl->ring_batched[slot] && i != 5) continue;
      // only the pairs whose events the plan records
      if (!(pl->ev_mask >> from[i] & 1) || !(pl->ev_mask >> to[i] & 1)) continue;
      float t = 0;
      if (hipEventElapsedTime(&t, pl->ev[slot][from[i]], pl->ev[slot][to[i]]) != hipSuccess)
        return FMM_ERR_DEVICE;
      acc[i] += t;
    }
  }
  out->t_sort_ms = (float)(acc[0] / cnt);
  out->t_p2m_ms = (float)(acc[1] / cnt);
  out->t_m2l_ms = (float)(acc[2] / cnt);
  out->t_l2p_ms = (float)(acc[3] / cnt);
  out->t_p2p_ms = (float)(acc[4] / cnt);
  out->t_total_ms = (float)(acc[5] / cnt);
  out->t_m2l_kernel_ms = (float)(acc[6] / cnt);
  out->m2l_kernel_level_lo = pl->f32 ? std::max(pl->lt.split, pl->lt.kmin) : pl->lt.kmin;
  out->n_timed = cnt;
  pl->ring_count = 0;
  return FMM_OK;
}

int32_t fmm_coef_stride(fmm_plan_t pl) { return pl ? pl->cs : FMM_ERR_INVALID_ARG; }

int32_t fmm_coef_order(fmm_plan_t pl) { return pl ? pl->pb : FMM_ERR_INVALID_ARG; }

int64_t fmm_debug_level_data(fmm_plan_t pl, int32_t level, int32_t which, void* dst,
                             int64_t dst_bytes) {
  if (!pl || !dst || dst_bytes < 0) return FMM_ERR_INVALID_ARG;
  if (hipSetDevice(pl->device) != hipSuccess) return FMM_ERR_DEVICE;
  if (hipStreamSynchronize(pl->last_stream) != hipSuccess) return FMM_ERR_DEVICE;
  const void* src = nullptr;
  int64_t bytes = 0;
  switch (which) {
    case FMM_DBG_MOMENTS:
    case FMM_DBG_LOCALS: {
      if (pl->last_batched) return FMM_ERR_UNSUPPORTED;
      if (level < pl->lt.kmin || level > pl->L) return FMM_ERR_INVALID_ARG;
      const int64_t nb = (int64_t)1 << (pl->dim * level);
      const int64_t cnt = nb * pl->cs;
      bytes = cnt * (int64_t)sizeof(double);
      if (bytes > dst_bytes) return FMM_ERR_INVALID_ARG;
      if (level < pl->lt.split) {
        const double* base = which == FMM_DBG_MOMENTS ? pl->mom64 : pl->loc64;
        src = base + pl->lt.off[level] * pl->cs;
        break;
      }
      const float* base = which == FMM_DBG_MOMENTS ? pl->mom32 : pl->loc32;
      std::vector<float> tmp((size_t)cnt);
      if (hipMemcpy(tmp.data(), base + pl->lt.off[level] * pl->cs, (size_t)cnt * sizeof(float),
                    hipMemcpyDeviceToHost) != hipSuccess)
        return FMM_ERR_DEVICE;
      double* d = static_cast<double*>(dst);
      for (int64_t i = 0; i < cnt; ++i) d[i] = tmp[(size_t)i];
      return bytes;
    }
    case FMM_DBG_PERM:
      src = pl->perm;
      bytes = pl->last_n * (int64_t)sizeof(int32_t);
      break;
    case FMM_DBG_LEAF_START:
      if (pl->last_batched) return FMM_ERR_UNSUPPORTED;
      src = pl->leaf_start;
      bytes = (pl->nleaf + 1) * (int64_t)sizeof(int32_t);
      break;
    case FMM_DBG_SORTED_KEYS:
      src = pl->sorted_keys;
      bytes = pl->last_n * (int64_t)sizeof(uint32_t);
      break;
    case FMM_DBG_FEATURES:
      if (!pl->learned || !pl->have_model) return FMM_ERR_UNSUPPORTED;
      src = pl->d_feat;
      bytes = (int64_t)pl->last_nsys * (kMaxLevels2D + 1) * 3 * (int64_t)sizeof(float);
      break;
    default:
      return FMM_ERR_INVALID_ARG;
  }
  if (bytes > dst_bytes) return FMM_ERR_INVALID_ARG;
  if (bytes == 0) return 0;
  if (!src) return FMM_ERR_INVALID_ARG;
  if (hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return FMM_ERR_DEVICE;
  return bytes;
}

int fmm_destroy(fmm_plan_t pl) {
  free_plan(pl);
  return FMM_OK;
}

}  // extern "C"
