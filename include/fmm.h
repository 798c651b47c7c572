/*
 * fmm.h -- C ABI of the shift-free fast multipole method on one MI355X (gfx950).
 *
 * Problem (Kajima, arXiv:2009.00767, Section 2.1 items 1-5 and the evaluation
 * steps E-1/E-2): N charged particles in a square (2D) or cube (3D) of side S
 * (S = 5 in the paper), subdivided uniformly to level L.  For every particle i
 * the library returns the potential due to all other particles and the field
 * (minus its gradient):
 *     2D:  phi_i = sum_{j != i, r_ij > 0} q_j log r_ij,
 *     3D:  phi_i = sum_{j != i, r_ij > 0} q_j / r_ij,      field_i = -grad_i phi_i.
 * Far interactions are summed with the shift-free passes of Section 2.2.1:
 * box vectors (truncated multipole expansions of order p, scaled by box side)
 * formed directly from the particles at every level (U-bar-1/U-bar-2 without
 * the M2M shift, which the level-independent particle map of the Note closing
 * Section 2.2.2 makes unnecessary), bilinear forms summed over each box's
 * interaction list at every level (D-bar-1, the multipole-to-local operator),
 * and each level's linear form evaluated directly at the particles and summed
 * over levels (D-bar-2 and F(v) = L_{m^l}(v) without the L2L shift).  Near
 * pairs (same or adjacent leaf) are summed directly (E-2 of Section 2.1).
 *
 * Conventions common to every entry point
 *  - Every array argument is a DEVICE pointer to caller-owned, contiguous
 *    memory; the library never frees or retains it.  Inputs are FP64.
 *  - Work is enqueued asynchronously on the caller's HIP stream (`stream`,
 *    a hipStream_t; NULL = the null stream).  Argument errors are detected on
 *    the host and returned synchronously before anything is enqueued.
 *  - Positions outside [origin, origin + side] or NaN are detected on the
 *    device; they set a plan-owned flag that fmm_last_status() reads after
 *    the caller has synchronised (or fmm_eval returns it directly when the
 *    plan was made with FMM_SYNC_CHECK).  Results are then unspecified.
 *  - A plan serves one stream at a time; calls on one plan must not overlap.
 *    Separate plans are independent.  There is no global mutable state.
 *  - fmm_plan allocates every buffer the evaluation needs (sized by
 *    max_particles); fmm_eval allocates nothing.
 *  - Status codes: 0 success, < 0 error, > 0 warning (see fmm_status).
 */
#ifndef PAPER_2009_00767_FMM_H
#define PAPER_2009_00767_FMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan_s* fmm_plan_t;

/* Interaction kernel G. */
enum fmm_kernel {
  FMM_LOG2D = 1,     /* G = log r in the plane, complex Laurent/Taylor expansions */
  FMM_COULOMB3D = 2, /* G = 1/r in space, solid-harmonic expansions */
  /* G = 1/r in space with the paper's own box vectors (Appendix STEP1-STEP5):
   * 4 x 4 x 4 fixed point charges per box at (-2, -1, 1, 2) s / 5 from its
   * centre; a charge maps to them by cubic Lagrange weights and two boxes
   * interact through the pair sum of their point charges.  order_p must be 4
   * (points per axis); FMM_FP64 or FMM_FP32 (point charges, operators and the
   * contraction in FP32, sums over levels in FP64).  Same outputs, limits and
   * errors as FMM_COULOMB3D. */
  FMM_COULOMB3D_POINTS = 3,
  /* As FMM_COULOMB3D_POINTS with n = order_p points per axis (2 <= n <= 5,
   * d = n^3 point charges per box; Discussion (4): d is a free parameter) at
   * the Chebyshev points of the first kind of the box, (s / 2) cos((2i + 1) pi
   * / (2n)) from its centre (Discussion (1): Chebyshev interpolation as the
   * alternative to the paper's set).  FMM_ROOT_FRAME takes n = 4 only. */
  FMM_COULOMB3D_CHEBYSHEV = 4,
  /* G = log r in the plane with the paper's own box vectors in the square box
   * (Appendix STEP1-STEP3, Fig. 3): 4 x 4 fixed point charges per box at
   * (-2, -1, 1, 2) s / 5 from its centre; a charge maps to them by the cubic
   * Lagrange weights of STEP2, and two boxes interact through the pair sum of
   * their point charges (STEP3), q_a q_b log |y_a - y_b|.  order_p must be 4
   * (points per axis); FMM_FP64 or FMM_FP32 (point charges, operators and the
   * contraction in FP32, level 2 and the sums over levels in FP64); one
   * system, fixed order.  Same outputs, limits and errors as FMM_LOG2D. */
  FMM_LOG2D_POINTS = 5,
  /* As FMM_LOG2D_POINTS with n = order_p points per axis (2 <= n <= 8, d = n^2
   * point charges per box; Discussion (4): d is a free parameter) at the
   * Chebyshev points of the first kind of the box, (s / 2) cos((2i + 1) pi /
   * (2n)) from its centre (Discussion (1)). */
  FMM_LOG2D_CHEBYSHEV = 6
};

/* Internal arithmetic.  Inputs and outputs are FP64 in every mode.
 *  FMM_FP64     : every step in FP64.
 *  FMM_FP32     : moments, locals and the multipole-to-local operator in FP32
 *                 (operators built in FP64 and rounded once, Discussion (3));
 *                 positions stored as FP32 offsets from their leaf centre; the
 *                 near field in FP32; per-particle accumulation over levels and
 *                 the final near + far sum in FP64; the coarsest level that has
 *                 an interaction list (level 2) kept in FP64.
 *  FMM_BF16_M2L : as FMM_FP32, but the multipole-to-local contraction runs as
 *                 BF16 matrix-core products with FP32 accumulation: the A_0
 *                 terms through three-part BF16 splits, the leading (at least
 *                 four) coefficients through two-term splits, the rest rounded
 *                 to BF16 once (2D only; error measured, not bounded: about
 *                 2e-7 relative L2 of the potentials against FP64). */
enum fmm_precision { FMM_FP64 = 0, FMM_FP32 = 1, FMM_BF16_M2L = 2 };

/* Expansion order policy. */
/* FMM_ORDER_LEARNED (2D only): before the far field of every evaluation an
 * order-prediction network (see fmm_set_order_model) picks, per system and
 * level k >= 2, the smallest order p_k in 4..24 whose predicted truncation
 * error fits tol / (number of levels with an interaction list) (tol / 2 of
 * that in the FP32 and BF16 modes, the other half being left to rounding),
 * with a margin of a factor 2 (0.3 in log10) for the network's error of fit;
 * systems of one depth group take the largest choice per level.  order_p is
 * the fixed fallback order (20 in the batched configuration), used when no
 * model is loaded or when the judge (FMM_JUDGE) rejects the learned result. */
enum fmm_order_policy {
  FMM_ORDER_FIXED = 0,  /* order_p at every level (or fmm_set_level_orders) */
  FMM_ORDER_LEARNED = 1 /* per-level order chosen by the loaded order model */
};

/* Plan flags (bit mask). */
enum fmm_flags {
  FMM_NO_FIELD = 1,   /* fields are not computed; `field` may be NULL */
  FMM_SYNC_CHECK = 2, /* fmm_eval synchronises and returns device-detected errors */
  FMM_TIMING = 4,     /* record per-phase HIP events (read by fmm_get_stats) */
  FMM_TIMING_NEAR = 32, /* record HIP events only around the near-field launches (their
                           stream): t_p2p_ms; the other times read as zero.  Fewer events
                           in the streams, whose records cost a few microseconds each */
  FMM_TIMING_M2L = 64,  /* likewise around the main multipole-to-local launch only:
                           t_m2l_kernel_ms */
  FMM_AUTOTUNE = 16,  /* at plan time, time the multipole-to-local tile variants on
                         the plan's own level sizes and keep the fastest (cached per
                         process by dimension, order bucket, precision and levels;
                         with the environment variable FMM_AUTOTUNE_CACHE set to a
                         file path, also read from and written to that JSON file) */
  FMM_ROOT_FRAME = 128, /* point-charge kernels, FMM_FP64 only: the passes of Section
                           2.2.1 as written, in the root box's frame (Appendix STEP4-
                           STEP5): box vectors as sums of their children (U-bar-2),
                           bilinear forms M_mi^T M_b M_m, linear forms passed from parent
                           to child by addition (D-bar-2), F(v) = L_{m^l}(v).  The same
                           results as the box-local form up to rounding that the transfers
                           M_m amplify with the depth (about 1e-10 relative at level 2,
                           1e-7 at level 3, 1e-4 at level 4: Discussion (3)).  Other
                           kernels or precisions: FMM_ERR_UNSUPPORTED */
  FMM_JUDGE = 8       /* learned order: every evaluation is also made at the fixed
                         order order_p in FP64; if the relative L2 difference of the
                         potentials over the particles of any one system exceeds tol,
                         the outputs are replaced by the fixed-order result and the
                         status becomes FMM_WARN_FALLBACK (judge_rel_err: the largest
                         per-system difference) */
};

enum fmm_status {
  FMM_OK = 0,
  FMM_ERR_INVALID_ARG = -1, /* bad argument (null pointer, size above the plan's maximum, ...) */
  FMM_ERR_DOMAIN = -2,      /* a position outside the box or NaN (device-detected) */
  FMM_ERR_NOMEM = -3,       /* device allocation failed at plan time */
  FMM_ERR_DEVICE = -4,      /* no usable gfx950 device, or a HIP runtime error */
  FMM_ERR_UNSUPPORTED = -5, /* a valid but unimplemented combination of options */
  FMM_ERR_SCRATCH = -6,     /* fmm_eval_noalloc: the input exceeds its fixed scratch */
  FMM_WARN_FALLBACK = 1     /* learned order rejected by its check; fixed order used */
};

typedef struct {
  int32_t kernel;        /* enum fmm_kernel */
  int32_t levels;        /* finest level L: 2D 0..12, 3D 0..8 */
  int32_t order_p;       /* expansion order p: 2D 1..30, 3D 1..8 */
  int32_t precision;     /* enum fmm_precision */
  int32_t order_policy;  /* enum fmm_order_policy */
  int32_t flags;         /* enum fmm_flags */
  double side;           /* box side S (> 0); the paper uses 5 */
  double origin[3];      /* lower corner of the box (unused components ignored) */
  double tol;            /* target relative error for FMM_ORDER_LEARNED */
  int64_t max_particles; /* largest n passed to fmm_eval (or total, batched) */
  int32_t max_systems;   /* batched: largest number of systems (> 1 enables fmm_eval_batched) */
  int32_t max_levels;    /* batched: deepest per-system tree */
  int64_t adaptive_near; /* 0: the uniform tree of depth `levels` (Section 2.1).  T > 0
                            (2D, one system, fixed order, levels >= 2): adaptive depth
                            for clustered inputs: a particle's tree stops at the first
                            level k >= 2 whose 3 x 3 boxes around its level-k box hold
                            at most T particles (at `levels` if none), and the particle
                            runs the shift-free passes of the tree of that depth d:
                            the interaction-list forms of its ancestors at levels
                            2..d and the near field over the 3 x 3 boxes around its
                            level-d box (at most T sources above level `levels`).
                            Negative: FMM_ERR_INVALID_ARG; other combinations:
                            FMM_ERR_UNSUPPORTED */
} fmm_options;

/* Per-phase times (milliseconds, HIP events recorded on the caller's stream
 * around each phase; zero unless the plan has FMM_TIMING, or for t_p2p_ms
 * FMM_TIMING_NEAR, for t_m2l_kernel_ms FMM_TIMING_M2L), averaged over the
 * evaluations made since the previous fmm_get_stats call (at most the last 64).
 * A batched evaluation runs as one HIP graph: it contributes its total only
 * (its phase times read as zero). */
typedef struct {
  float t_sort_ms;  /* binning, stable counting sort, gather */
  float t_p2m_ms;   /* moments at every level (U-bar) */
  float t_m2l_ms;   /* interaction-list contraction at every level (D-bar-1) */
  float t_l2p_ms;   /* local evaluation at every level (D-bar-2, F(v)), near + far, unsort */
  float t_p2p_ms;   /* near field; it runs on a second stream concurrently with the
                       far-field phases, so the phases need not add up to the total */
  float t_total_ms; /* whole evaluation on the caller's stream */
  int32_t m2l_launches; /* launches of the multipole-to-local kernel per evaluation */
  int32_t order_per_level[16];
  int32_t fallback;     /* 1 if the learned order was rejected */
  int32_t n_timed;      /* evaluations averaged */
  float t_m2l_kernel_ms;        /* the main M2L launch alone (levels m2l_kernel_level_lo..L) */
  int32_t m2l_kernel_level_lo;  /* 2 in FP64 mode; 3 in FP32 modes (level 2 runs apart in FP64) */
  double judge_rel_err;         /* FMM_JUDGE: the last judged difference (else 0) */
  int32_t m2l_tile_mb;          /* M2L tile: 2D 8 x (8 m2l_tile_mb) targets per workgroup,
                                   3D 4 m2l_tile_mb layers of 16 targets per workgroup */
  int32_t m2l_xcd_remap;        /* M2L tiles dealt to the XCDs in contiguous ranges */
  float m2l_tuned_ms;           /* FMM_AUTOTUNE: the chosen variant's time (else 0) */
  int32_t graph_builds;         /* batched graphs instantiated since the plan was made */
} fmm_stats;

/* Fills *out with defaults for `kernel` (side 5, origin 0, FP64, fixed order). */
int fmm_default_options(int32_t kernel, fmm_options* out);

/* Validates the options, builds the interaction-list tables and the
 * multipole-to-local operators in FP64 (Discussion (2): they do not depend on
 * the particles, so they are built once and excluded from evaluation time;
 * Discussion (3): built in double precision), and allocates every device buffer
 * on the current device.  *out receives the plan (NULL on error). */
int fmm_plan(const fmm_options* opt, fmm_plan_t* out);

/* Potentials and fields of n particles.
 *   pos   : device, FP64 [n][D] row-major (x, y[, z] per particle)
 *   q     : device, FP64 [n] charges
 *   pot   : device, FP64 [n] output, input order
 *   field : device, FP64 [n][D] output (may be NULL with FMM_NO_FIELD)
 *   stream: hipStream_t or NULL
 * n = 0 is valid and enqueues nothing.  n > max_particles -> FMM_ERR_INVALID_ARG. */
int fmm_eval(fmm_plan_t plan, int64_t n, const double* pos, const double* q, double* pot,
             double* field, void* stream);

/* Prepares batched evaluation of nsys independent 2D systems of a fixed
 * shape (host tables; plan-time work).  The plan must have been made with
 * max_systems > 1 (buffers are sized for up to max_systems systems of depth up
 * to max(levels, max_levels) and max_particles particles in total).  Every
 * system lives in the plan's box [origin, origin + side]^2 and interacts only
 * with itself.
 *   sys_offsets : HOST int64 [nsys + 1], sys_offsets[0] = 0, non-decreasing;
 *                 system s owns particles [sys_offsets[s], sys_offsets[s+1]) of
 *                 the concatenated pos / q / pot / field arrays
 *   sys_levels  : HOST int32 [nsys], the tree depth of each system (0 .. the
 *                 plan's maximum), or NULL for clamp(round(log4(n_s / 16)), 2,
 *                 maximum) (about 16 particles per leaf)
 * Systems of equal depth are evaluated together as one stacked tree; one
 * stable sort orders all particles by (depth, system, leaf).  This call
 * uploads the system tables and captures the whole evaluation once as a HIP
 * graph (synchronising with the plan's streams); calling it again with the
 * same shape returns at once.  Settings the graph depends on (fmm_set_level_orders,
 * fmm_set_m2l_variant, fmm_set_order_model) capture the prepared shape again.
 * A shape beyond the plan's capacities returns FMM_ERR_INVALID_ARG;
 * FMM_ERR_UNSUPPORTED for 3D plans or plans without max_systems > 1. */
int fmm_batch_prepare(fmm_plan_t plan, int32_t nsys, const int64_t* sys_offsets,
                      const int32_t* sys_levels);

/* Potentials and fields of the prepared batch: one replay of its graph on the
 * caller's stream.  Allocates nothing, instantiates nothing and does not
 * synchronise (the caller's buffer addresses reach the graph through a device
 * record written by a one-thread kernel before the replay).
 *   nsys        : must equal the prepared count, else FMM_ERR_INVALID_ARG
 *   sys_offsets : DEVICE int64 [nsys + 1], the prepared offsets
 *   sys_levels  : DEVICE int32 [nsys], the prepared depths, or NULL if the
 *                 prepared depths follow the default rule
 *   pos, q, pot, field, stream : as in fmm_eval (device, concatenated; any
 *                 buffers, they may change from call to call)
 * The kernels run the prepared tables; device tables that differ from them are
 * detected on the device and reported by fmm_last_status as
 * FMM_ERR_INVALID_ARG (the outputs are then unspecified).  Other errors as in
 * fmm_eval; FMM_ERR_INVALID_ARG without a prepared shape. */
int fmm_eval_batched(fmm_plan_t plan, int32_t nsys, const int64_t* sys_offsets,
                     const int32_t* sys_levels, const double* pos, const double* q, double* pot,
                     double* field, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fmm_eval of
 * one 2D system without a plan.  It runs the kernels of fmm_eval, with every
 * buffer beyond the caller's inputs and outputs (sort keys, counts, leaf
 * offsets, sorted particles, moments, locals, operators built by a kernel in
 * each call, near-field sums, status words) in a fixed 16 MiB device array of
 * the library, one per device, which the device holds until the process ends.
 * It calls no allocation routine and records no memset.
 *   opt   : HOST options as for fmm_plan; kernel FMM_LOG2D, order_policy
 *           FMM_ORDER_FIXED, precision FMM_FP64 or FMM_FP32, flags among
 *           FMM_NO_FIELD and FMM_SYNC_CHECK, max_systems <= 1, adaptive_near 0
 *           (max_particles, tol and max_levels are ignored); otherwise
 *           FMM_ERR_UNSUPPORTED
 *   n, pos, q, pot, field, stream : as in fmm_eval (device, input order)
 * Limits of the fixed array: n <= 65536, levels <= 6, order_p <= 20; beyond
 * them FMM_ERR_SCRATCH, before anything is enqueued.  Results equal fmm_eval's
 * for the same options up to rounding (the same kernels, run one after another
 * on the caller's stream, with the M2L tile variant at its default).  Every
 * call on a device shares that device's array and leaves its contents there:
 * calls that overlap in time on one device (several streams or threads) race
 * and must be serialised by the caller.  Device-detected errors (positions
 * outside the box, NaN) are returned only with FMM_SYNC_CHECK, which
 * synchronises the stream; otherwise the call is asynchronous. */
int fmm_eval_noalloc(const fmm_options* opt, int64_t n, const double* pos, const double* q,
                     double* pot, double* field, void* stream);

/* Per-level expansion orders (2D plans).  orders: HOST int32 [count], count =
 * the plan's deepest level + 1 (levels, or max(levels, max_levels) for batched
 * plans); orders[k] for k >= 2 is the order p_k of level k, 1 <= p_k <=
 * order_p (entries 0 and 1 are ignored).  Level k's moments, interaction-list
 * contraction and local evaluation all truncate at p_k (the levels of the
 * shift-free method exchange no coefficients, Section 2.2.1, so each level is
 * the fixed-order method at its own order).  Applies to every later
 * evaluation until changed; the plan starts with p_k = order_p.  Synchronises
 * with the plan's last stream.  FMM_ERR_UNSUPPORTED for 3D plans. */
int fmm_set_level_orders(fmm_plan_t plan, const int32_t* orders, int32_t count);

/* ----- learned order (2D) ------------------------------------------------
 * Order-prediction network: 3 inputs -> 64 ReLU -> 64 ReLU -> 21 outputs, FP32.
 * Inputs of a (system, level k): k / 10, log2(number of non-empty level-k
 * boxes) / 20, log10 of the 2-norm of the system's charges.  Output o is the
 * predicted log10 of the level's truncation error at order 4 + o, relative to
 * the norm of the potentials.  Parameters, one array, row-major with the output
 * index major: W1[64][3], b1[64], W2[64][64], b2[64], W3[21][64], b3[21]. */
#define FMM_MLP_NPARAM 5781

/* Loads the network into a FMM_ORDER_LEARNED plan.  weights: HOST float
 * [FMM_MLP_NPARAM] (copied; every value must be finite, else
 * FMM_ERR_INVALID_ARG).  Synchronises with the plan's last stream. */
int fmm_set_order_model(fmm_plan_t plan, const float* weights, int64_t n_floats);

/* Network outputs y [m][21] for inputs x [m][3] (device arrays, FP32). */
int fmm_mlp_forward(const float* w, const float* x, int64_t m, float* y, void* stream);

/* Mean squared error over all outputs, loss = sum (y - t)^2 / (21 m), and its
 * gradient with respect to the parameters (backpropagation).  Device arrays:
 * w, grad [FMM_MLP_NPARAM], x [m][3], t [m][21], loss [1].  Deterministic (the
 * per-wave partial gradients are summed in a fixed order in FP64).  Allocates
 * and frees its partial-sum scratch (synchronises). */
int fmm_mlp_loss_grad(const float* w, const float* x, const float* t, int64_t m, float* grad,
                      float* loss, void* stream);

/* One Adam step (Kingma and Ba 2015, Algorithm 1; beta1 0.9, beta2 0.999,
 * eps 1e-8; step counts from 1): m1, m2 are the moment estimates, updated in
 * place with w.  Device arrays of FMM_MLP_NPARAM floats. */
int fmm_mlp_adam_step(float* w, const float* grad, float* m1, float* m2, int32_t step, float lr,
                      void* stream);

/* Full-batch training on the device: `steps` Adam steps (moments start at
 * zero) of the loss above on x [m][3], t [m][21]; w (device) holds the initial
 * parameters and receives the trained ones.  loss_history: HOST float [steps]
 * (the loss before each step) or NULL.  Allocates its scratch; synchronises. */
int fmm_mlp_train(float* w, const float* x, const float* t, int64_t m, int32_t steps, float lr,
                  float* loss_history, void* stream);

/* Selects the multipole-to-local tile variant (what FMM_AUTOTUNE chooses by
 * timing; fmm_get_stats reports the current one).  2D: workgroups of 8 x
 * (8 tile_mb) target boxes, tile_mb in {1, 2, 3, 4, 8} where compiled for the
 * plan's precision and order and within the LDS, tiles dealt to the XCDs in
 * contiguous ranges if xcd_remap = 1.  3D: 4 tile_mb layers of 16 targets per
 * workgroup, tile_mb in {1, 2} (four waves of tile_mb layers) or, FP32 only, 4
 * (eight waves of two layers); each operator value read from LDS serves the
 * products of a wave's layers; xcd_remap = 1 only.  Anything else: FMM_ERR_INVALID_ARG.  Every
 * variant forms the same sums in the same order: results are bit-identical. */
int fmm_set_m2l_variant(fmm_plan_t plan, int32_t tile_mb, int32_t xcd_remap);

/* Device-detected status of the last fmm_eval on this plan.  Synchronises with
 * the plan's last stream. */
int fmm_last_status(fmm_plan_t plan);

/* Phase times and the per-level order of the last evaluation (synchronises). */
int fmm_get_stats(fmm_plan_t plan, fmm_stats* out);

/* Debug export of the last evaluation's intermediate data, copied to host
 * memory dst (dst_bytes available).  Synchronises.  `which`:
 *   FMM_DBG_MOMENTS    level `level`'s box vectors: boxes in Morton order,
 *                      per box fmm_coef_stride() FP64 values laid out as
 *                      described at fmm_coef_order() (FP32 levels widened)
 *   FMM_DBG_LOCALS     level `level`'s local coefficients, same layout
 *   FMM_DBG_PERM       int32 [n]: sorted position -> input index
 *   FMM_DBG_LEAF_START int32 [leaves + 1]: first sorted position of each leaf
 *                      (Morton order)
 *   FMM_DBG_SORTED_KEYS uint32 [n]: Morton leaf key of each sorted position
 * After fmm_eval_batched only FMM_DBG_PERM (over the concatenated particles,
 * ordered by (depth, system, leaf)) and FMM_DBG_SORTED_KEYS ((rank of the
 * system within its depth group << 2 L) | Morton key, L the system's depth) are
 * available; the others return FMM_ERR_UNSUPPORTED.
 * Returns the number of bytes written (>= 0) or an error status. */
enum fmm_debug_which {
  FMM_DBG_MOMENTS = 0,
  FMM_DBG_LOCALS = 1,
  FMM_DBG_PERM = 2,
  FMM_DBG_LEAF_START = 3,
  FMM_DBG_SORTED_KEYS = 4,
  FMM_DBG_FEATURES = 5 /* learned order: float [systems][13][3], the network inputs of
                          every (system, level) of the last evaluation (levels 2..L_s) */
};
int64_t fmm_debug_level_data(fmm_plan_t plan, int32_t level, int32_t which, void* dst,
                             int64_t dst_bytes);

/* Number of FP64 values per box in the debug export of moments/locals. */
int32_t fmm_coef_stride(fmm_plan_t plan);

/* Layout order PB of the debug export.  2D: values 2(m-1), 2(m-1)+1 hold the
 * real and imaginary parts of coefficient m = 1..PB, values 2 PB, 2 PB + 1 those
 * of coefficient 0; the imaginary part of local coefficient 0 is not formed (it
 * enters neither the potential nor the field) and reads as zero.  3D (solid
 * harmonics, orders m >= 0 stored): degree n >= 1 at n^2 - 1 (m = 0), then
 * n^2 - 1 + 2m - 1 and n^2 - 1 + 2m (re, im of order m = 1..n); degree 0 at
 * (PB+1)^2 - 1.  Coefficients above the plan's order are zero.
 * FMM_COULOMB3D_POINTS (PB = 4): values 0..63 hold the charges of point
 * i + 4 j + 16 l of the box (x offset index i, y j, z l; offsets (-2, -1, 1, 2)
 * s / 5 in that order); the locals are the potentials at those points times the
 * box side s (an operator of unit box side); values 64..67 are zero.
 * FMM_COULOMB3D_CHEBYSHEV (PB = n): values 0..n^3 - 1 hold point i + n j +
 * n^2 l (nodes ascending), the same units; the row is padded with zeros to 68
 * values for n <= 4 and to 128 for n = 5.
 * FMM_LOG2D_POINTS and FMM_LOG2D_CHEBYSHEV (PB = n, the points per axis):
 * values 0..n^2 - 1 hold the charges of point i + n j of the box (x offset
 * index i, y j, nodes ascending), the locals the potentials at those points
 * (in the units of the inputs); the row is padded with zeros to a multiple of
 * 16 values. */
int32_t fmm_coef_order(fmm_plan_t plan);

/* Releases every device buffer of the plan (synchronises first).  NULL is a no-op. */
int fmm_destroy(fmm_plan_t plan);

/* Static, human-readable text for a status code. */
const char* fmm_status_str(int status);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_2009_00767_FMM_H */
