"""Shift-free fast multipole method on one MI355X (gfx950).

Python binding of ``libfmm.so`` (the C ABI declared in ``include/fmm.h``).
This module only marshals arguments: every step of the evaluation runs in the
library's HIP kernels.  PyTorch is used for device memory (tensor data
pointers) and streams (``torch.cuda.current_stream().cuda_stream``).

If ``libfmm.so`` is missing the first call raises ``RuntimeError``; there is no
fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm.so")

FMM_LOG2D = 1
FMM_COULOMB3D = 2
FMM_COULOMB3D_POINTS = 3
FMM_COULOMB3D_CHEBYSHEV = 4
FMM_LOG2D_POINTS = 5
FMM_LOG2D_CHEBYSHEV = 6
FMM_FP64 = 0
FMM_FP32 = 1
FMM_BF16_M2L = 2
FMM_ORDER_FIXED = 0
FMM_ORDER_LEARNED = 1
FMM_NO_FIELD = 1
FMM_SYNC_CHECK = 2
FMM_TIMING = 4
FMM_TIMING_NEAR = 32
FMM_TIMING_M2L = 64
FMM_JUDGE = 8
FMM_ROOT_FRAME = 128
FMM_AUTOTUNE = 16
FMM_MLP_NPARAM = 5781
FMM_OK = 0
FMM_ERR_INVALID_ARG = -1
FMM_ERR_DOMAIN = -2
FMM_ERR_NOMEM = -3
FMM_ERR_DEVICE = -4
FMM_ERR_UNSUPPORTED = -5
FMM_ERR_SCRATCH = -6
FMM_WARN_FALLBACK = 1
FMM_DBG_MOMENTS = 0
FMM_DBG_LOCALS = 1
FMM_DBG_PERM = 2
FMM_DBG_LEAF_START = 3
FMM_DBG_SORTED_KEYS = 4
FMM_DBG_FEATURES = 5

# Every symbol include/fmm.h declares (checked by the ABI tests).
EXPORTED = [
    "fmm_default_options", "fmm_plan", "fmm_eval", "fmm_batch_prepare", "fmm_eval_batched",
    "fmm_set_level_orders",
    "fmm_set_order_model", "fmm_mlp_forward", "fmm_mlp_loss_grad", "fmm_mlp_adam_step",
    "fmm_mlp_train", "fmm_set_m2l_variant", "fmm_last_status", "fmm_get_stats", "fmm_debug_level_data",
    "fmm_coef_stride", "fmm_coef_order", "fmm_destroy", "fmm_status_str", "fmm_eval_noalloc",
]


class FmmOptions(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32), ("levels", ctypes.c_int32), ("order_p", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("order_policy", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("side", ctypes.c_double), ("origin", ctypes.c_double * 3),
        ("tol", ctypes.c_double), ("max_particles", ctypes.c_int64),
        ("max_systems", ctypes.c_int32), ("max_levels", ctypes.c_int32),
        ("adaptive_near", ctypes.c_int64),
    ]


class FmmStats(ctypes.Structure):
    _fields_ = [
        ("t_sort_ms", ctypes.c_float), ("t_p2m_ms", ctypes.c_float),
        ("t_m2l_ms", ctypes.c_float), ("t_l2p_ms", ctypes.c_float),
        ("t_p2p_ms", ctypes.c_float), ("t_total_ms", ctypes.c_float),
        ("m2l_launches", ctypes.c_int32), ("order_per_level", ctypes.c_int32 * 16),
        ("fallback", ctypes.c_int32), ("n_timed", ctypes.c_int32),
        ("t_m2l_kernel_ms", ctypes.c_float), ("m2l_kernel_level_lo", ctypes.c_int32),
        ("judge_rel_err", ctypes.c_double),
        ("m2l_tile_mb", ctypes.c_int32), ("m2l_xcd_remap", ctypes.c_int32),
        ("m2l_tuned_ms", ctypes.c_float), ("graph_builds", ctypes.c_int32),
    ]


class FmmError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {fmm_status_str(status)} (status {status})")
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_2009_00767_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.fmm_default_options.argtypes = [i32, ctypes.POINTER(FmmOptions)]
        L.fmm_plan.argtypes = [ctypes.POINTER(FmmOptions), ctypes.POINTER(vp)]
        L.fmm_eval.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.fmm_batch_prepare.argtypes = [vp, i32, vp, vp]
        L.fmm_eval_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.fmm_eval_noalloc.argtypes = [ctypes.POINTER(FmmOptions), i64, vp, vp, vp, vp, vp]
        L.fmm_set_level_orders.argtypes = [vp, vp, i32]
        L.fmm_set_order_model.argtypes = [vp, vp, i64]
        L.fmm_set_m2l_variant.argtypes = [vp, i32, i32]
        L.fmm_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.fmm_mlp_loss_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.fmm_mlp_adam_step.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp]
        L.fmm_mlp_train.argtypes = [vp, vp, vp, i64, i32, ctypes.c_float, vp, vp]
        L.fmm_last_status.argtypes = [vp]
        L.fmm_get_stats.argtypes = [vp, ctypes.POINTER(FmmStats)]
        L.fmm_debug_level_data.argtypes = [vp, i32, i32, vp, i64]
        L.fmm_debug_level_data.restype = i64
        L.fmm_coef_stride.argtypes = [vp]
        L.fmm_coef_order.argtypes = [vp]
        L.fmm_destroy.argtypes = [vp]
        L.fmm_status_str.argtypes = [ctypes.c_int]
        L.fmm_status_str.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _ptr(x):
    """Device address of a tensor (or an int / None passed through)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def fmm_status_str(status):
    return lib().fmm_status_str(int(status)).decode()


def fmm_default_options(kernel=FMM_LOG2D):
    o = FmmOptions()
    rc = lib().fmm_default_options(kernel, ctypes.byref(o))
    if rc != FMM_OK:
        raise FmmError(rc, "fmm_default_options")
    return o


def fmm_plan(opts):
    h = ctypes.c_void_p()
    rc = lib().fmm_plan(ctypes.byref(opts), ctypes.byref(h))
    if rc != FMM_OK:
        raise FmmError(rc, "fmm_plan")
    return h


def fmm_eval(plan, n, pos, q, pot, field=None, stream=None):
    rc = lib().fmm_eval(plan, int(n), _ptr(pos), _ptr(q), _ptr(pot), _ptr(field), _stream(stream))
    if rc < 0:
        raise FmmError(rc, "fmm_eval")
    return rc


def fmm_eval_noalloc(opts, n, pos, q, pot, field=None, stream=None):
    """fmm_eval without a plan, every scratch buffer in the library's fixed
    device array (see include/fmm.h); opts: FmmOptions (host)."""
    rc = lib().fmm_eval_noalloc(ctypes.byref(opts), int(n), _ptr(pos), _ptr(q), _ptr(pot),
                                _ptr(field), _stream(stream))
    if rc < 0:
        raise FmmError(rc, "fmm_eval_noalloc")
    return rc


def fmm_batch_prepare(plan, sys_offsets, sys_levels=None):
    """sys_offsets / sys_levels: host arrays (int64 [nsys+1], int32 [nsys] or None)."""
    import numpy as np
    off = np.ascontiguousarray(sys_offsets, dtype=np.int64)
    lev = None if sys_levels is None else np.ascontiguousarray(sys_levels, dtype=np.int32)
    rc = lib().fmm_batch_prepare(plan, len(off) - 1, off.ctypes.data,
                                 None if lev is None else lev.ctypes.data)
    if rc < 0:
        raise FmmError(rc, "fmm_batch_prepare")
    return rc


def fmm_eval_batched(plan, nsys, sys_offsets, sys_levels, pos, q, pot, field=None, stream=None):
    """sys_offsets / sys_levels: device tensors (int64 [nsys+1], int32 [nsys] or None)
    describing the shape given to fmm_batch_prepare."""
    rc = lib().fmm_eval_batched(plan, int(nsys), _ptr(sys_offsets), _ptr(sys_levels), _ptr(pos),
                                _ptr(q), _ptr(pot), _ptr(field), _stream(stream))
    if rc < 0:
        raise FmmError(rc, "fmm_eval_batched")
    return rc


def fmm_set_level_orders(plan, orders):
    import numpy as np
    o = np.ascontiguousarray(orders, dtype=np.int32)
    rc = lib().fmm_set_level_orders(plan, o.ctypes.data, len(o))
    if rc < 0:
        raise FmmError(rc, "fmm_set_level_orders")
    return rc


def fmm_set_order_model(plan, weights):
    """weights: host array of FMM_MLP_NPARAM floats (see include/fmm.h)."""
    import numpy as np
    w = np.ascontiguousarray(weights, dtype=np.float32)
    rc = lib().fmm_set_order_model(plan, w.ctypes.data, w.size)
    if rc < 0:
        raise FmmError(rc, "fmm_set_order_model")
    return rc


def _check(rc, what):
    if rc < 0:
        raise FmmError(rc, what)
    return rc


def fmm_mlp_forward(w, x, y, stream=None):
    """Device FP32 tensors: w [5781], x [m, 3] -> y [m, 21]."""
    return _check(lib().fmm_mlp_forward(_ptr(w), _ptr(x), x.shape[0], _ptr(y), _stream(stream)),
                  "fmm_mlp_forward")


def fmm_mlp_loss_grad(w, x, t, grad, loss, stream=None):
    return _check(lib().fmm_mlp_loss_grad(_ptr(w), _ptr(x), _ptr(t), x.shape[0], _ptr(grad),
                                          _ptr(loss), _stream(stream)), "fmm_mlp_loss_grad")


def fmm_mlp_adam_step(w, grad, m1, m2, step, lr, stream=None):
    return _check(lib().fmm_mlp_adam_step(_ptr(w), _ptr(grad), _ptr(m1), _ptr(m2), step, lr,
                                          _stream(stream)), "fmm_mlp_adam_step")


def fmm_mlp_train(w, x, t, steps, lr, stream=None):
    """Trains w (device FP32 [5781], in place); returns the loss before each step."""
    import numpy as np
    hist = np.zeros(max(steps, 1), np.float32)
    _check(lib().fmm_mlp_train(_ptr(w), _ptr(x), _ptr(t), x.shape[0], steps, lr,
                               hist.ctypes.data, _stream(stream)), "fmm_mlp_train")
    return hist[:steps]


def fmm_last_status(plan):
    return lib().fmm_last_status(plan)


def fmm_get_stats(plan):
    s = FmmStats()
    rc = lib().fmm_get_stats(plan, ctypes.byref(s))
    if rc != FMM_OK:
        raise FmmError(rc, "fmm_get_stats")
    return s


def fmm_coef_stride(plan):
    return lib().fmm_coef_stride(plan)


def fmm_coef_order(plan):
    return lib().fmm_coef_order(plan)


def fmm_debug_level_data(plan, level, which, nbytes):
    buf = (ctypes.c_char * max(int(nbytes), 1))()
    got = lib().fmm_debug_level_data(plan, int(level), int(which), buf, int(nbytes))
    if got < 0:
        raise FmmError(int(got), "fmm_debug_level_data")
    return bytes(buf)[:got]


def fmm_destroy(plan):
    if plan:
        lib().fmm_destroy(plan)


class FMM:
    """Owns one plan.  ``evaluate(pos, q)`` takes FP64 CUDA tensors [n, D] and
    [n] and returns (pot [n], field [n, D] or None) as new FP64 tensors."""

    def __init__(self, kernel=FMM_LOG2D, levels=4, order=12, precision=FMM_FP64,
                 max_particles=1 << 20, side=5.0, origin=(0.0, 0.0, 0.0), flags=0,
                 order_policy=FMM_ORDER_FIXED, tol=1e-6, max_systems=1, max_levels=None,
                 adaptive_near=0):
        o = fmm_default_options(kernel)
        o.adaptive_near = adaptive_near
        o.levels, o.order_p, o.precision = levels, order, precision
        o.max_particles, o.side, o.flags = max_particles, side, flags
        o.order_policy, o.tol, o.max_systems = order_policy, tol, max_systems
        o.max_levels = levels if max_levels is None else max_levels
        for d in range(3):
            o.origin[d] = origin[d] if d < len(origin) else 0.0
        self.opts = o
        self.dim = 2 if kernel in (FMM_LOG2D, FMM_LOG2D_POINTS, FMM_LOG2D_CHEBYSHEV) else 3
        self.plan = fmm_plan(o)

    def evaluate(self, pos, q, stream=None, pot=None, field=None):
        import torch
        n = q.shape[0]
        if pot is None:
            pot = torch.empty(n, dtype=torch.float64, device=q.device)
        want_field = not (self.opts.flags & FMM_NO_FIELD)
        if want_field and field is None:
            field = torch.empty((n, self.dim), dtype=torch.float64, device=q.device)
        fmm_eval(self.plan, n, pos, q, pot, field if want_field else None, stream)
        return pot, (field if want_field else None)

    def evaluate_batched(self, sys_offsets, pos, q, sys_levels=None, stream=None, pot=None,
                         field=None):
        """sys_offsets / sys_levels: host arrays.  A new shape is prepared (and
        its tables copied to device tensors) once; repeated shapes only replay."""
        import numpy as np
        import torch
        off = np.ascontiguousarray(sys_offsets, dtype=np.int64)
        lev = None if sys_levels is None else np.ascontiguousarray(sys_levels, dtype=np.int32)
        key = (off.tobytes(), None if lev is None else lev.tobytes())
        if getattr(self, "_prep_key", None) != key:
            self._prep_key = None
            fmm_batch_prepare(self.plan, off, lev)
            self._d_off = torch.from_numpy(off).to(q.device)
            self._d_lev = None if lev is None else torch.from_numpy(lev).to(q.device)
            self._prep_key = key
        n = q.shape[0]
        if pot is None:
            pot = torch.empty(n, dtype=torch.float64, device=q.device)
        want_field = not (self.opts.flags & FMM_NO_FIELD)
        if want_field and field is None:
            field = torch.empty((n, self.dim), dtype=torch.float64, device=q.device)
        fmm_eval_batched(self.plan, len(off) - 1, self._d_off, self._d_lev, pos, q, pot,
                         field if want_field else None, stream)
        return pot, (field if want_field else None)

    def set_m2l_variant(self, tile_mb, xcd_remap=1):
        return _check(lib().fmm_set_m2l_variant(self.plan, tile_mb, xcd_remap),
                      "fmm_set_m2l_variant")

    def set_order_model(self, weights):
        return fmm_set_order_model(self.plan, weights)

    def set_level_orders(self, orders):
        return fmm_set_level_orders(self.plan, orders)

    def last_status(self):
        return fmm_last_status(self.plan)

    def stats(self):
        return fmm_get_stats(self.plan)

    def close(self):
        if self.plan:
            fmm_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
