"""CPU FP64 oracle for the shift-free FMM -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library under
``paper_2009_00767_amd``) never does; the two share no code.

Thin numpy wrappers over ``liboracle.so`` (built from the C sources here by
``oracle/build.py``).  Every function takes and returns FP64 numpy arrays.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_I64P = ctypes.POINTER(ctypes.c_int64)
_DP = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB", _build.LIB)  # e.g. a sanitizer build
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.oracle_direct.argtypes = [ctypes.c_int, ctypes.c_int64, _DP, _DP, ctypes.c_int64, _I64P,
                                    _DP, _DP]
        L.oracle_leaf_coord.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int]
        L.oracle_leaf_coord.restype = ctypes.c_int64
        L.oracle_ilist2d.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _I64P]
        L.oracle_ilist3d.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                     _I64P]
        L.oracle_fmm2d_ex.argtypes = [ctypes.c_int64, _DP, _DP, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, _DP, ctypes.c_int, ctypes.c_int64, _I64P,
                                      _DP, _DP, ctypes.c_int, _DP, _DP, _DP, _DP,
                                      ctypes.c_void_p]
        L.oracle_fmm2d_adaptive.argtypes = [ctypes.c_int64, _DP, _DP, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int64, ctypes.c_double, _DP,
                                            _DP, _DP, ctypes.c_void_p]
        L.oracle_p2m2d_point.argtypes = [ctypes.c_int64, _DP, _DP, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, _DP]
        L.oracle_m2p2d_point.argtypes = [_DP, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_m2p2d_point.restype = ctypes.c_double
        if hasattr(L, "oracle_fmm3d_ex"):
            L.oracle_fmm3d_ex.argtypes = [ctypes.c_int64, _DP, _DP, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, _DP, ctypes.c_int, ctypes.c_int64,
                                          _I64P, _DP, _DP, ctypes.c_int, _DP, _DP]
            L.oracle_sh_regular.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, _DP]
            L.oracle_sh_irregular.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, _DP]
        L.oracle_fmm3d_lagrange.argtypes = [ctypes.c_int64, _DP, _DP, ctypes.c_int,
                                            ctypes.c_double, _DP, ctypes.c_int64, _I64P, _DP,
                                            _DP, ctypes.c_int, _DP, _DP]
        L.oracle_lagrange_weights.argtypes = [ctypes.c_double, _DP, _DP]
        L.oracle_lagrange_weights_nodes.argtypes = [ctypes.c_int, _DP, ctypes.c_double, _DP, _DP]
        L.oracle_fmm3d_lagrange_nodes.argtypes = [ctypes.c_int, _DP, ctypes.c_int64, _DP, _DP,
                                                  ctypes.c_int, ctypes.c_double, _DP,
                                                  ctypes.c_int64, _I64P, _DP, _DP, ctypes.c_int,
                                                  _DP, _DP]
        L.oracle_fmm2d_lagrange_nodes.argtypes = [ctypes.c_int, _DP, ctypes.c_int64, _DP, _DP,
                                                  ctypes.c_int, ctypes.c_double, _DP,
                                                  ctypes.c_int64, _I64P, _DP, _DP, ctypes.c_int,
                                                  _DP, _DP]
        L.oracle_lagrange_transfer.argtypes = [ctypes.c_int, _DP, ctypes.c_double, _DP,
                                               ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                               ctypes.c_int64, _DP]
        L.oracle_lagrange_box_weights.argtypes = [ctypes.c_int, _DP, ctypes.c_double, _DP,
                                                  ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                                  ctypes.c_int64, _DP, _DP]
        L.oracle_fmm3d_lagrange_root.argtypes = [ctypes.c_int, _DP, ctypes.c_int64, _DP, _DP,
                                                 ctypes.c_int, ctypes.c_double, _DP,
                                                 ctypes.c_int64, _I64P, _DP, _DP, _DP]
        L.oracle_mlp_forward.argtypes = [_DP, ctypes.c_int64, _DP, _DP]
        L.oracle_mlp_loss_grad.argtypes = [_DP, ctypes.c_int64, _DP, _DP, _DP]
        L.oracle_mlp_loss_grad.restype = ctypes.c_double
        L.oracle_mlp_adam.argtypes = [ctypes.c_int64, _DP, _DP, _DP, _DP, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_DP) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_I64P) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with status {rc}")


def direct(pos, q, targets=None, field=True):
    """Exact pair sum (Neumaier-compensated).  pos [n, D], q [n]."""
    pos, q = _f64(pos), _f64(q)
    n, dim = pos.shape
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else len(tg)
    pot = np.zeros(nt)
    fld = np.zeros((nt, dim)) if field else None
    _check(lib().oracle_direct(dim, n, _d(pos), _d(q), nt, _i(tg), _d(pot), _d(fld)), "direct")
    return (pot, fld) if field else pot


def leaf_coord(x, origin, side, L):
    return lib().oracle_leaf_coord(float(x), float(origin), float(side), int(L))


def ilist2d(k, tx, ty):
    out = np.zeros(2 * 27, dtype=np.int64)
    c = lib().oracle_ilist2d(k, tx, ty, _i(out))
    return out[: 2 * c].reshape(c, 2)


def ilist3d(k, tx, ty, tz):
    out = np.zeros(3 * 189, dtype=np.int64)
    c = lib().oracle_ilist3d(k, tx, ty, tz, _i(out))
    return out[: 3 * c].reshape(c, 3)


def fmm2d_adaptive(pos, q, L, p, near_max, side=5.0, origin=(0.0, 0.0)):
    """Shift-free 2D FMM with an adaptive depth: a particle's tree stops at the
    first level k >= 2 whose 3 x 3 boxes around its box hold at most near_max
    particles (L if none).  Returns (pot, field, depth), depth[i] the level of
    particle i's leaf."""
    pos, q = _f64(pos), _f64(q)
    n = pos.shape[0]
    pot = np.zeros(n)
    fld = np.zeros((n, 2))
    dep = np.zeros(n, np.int32)
    rc = lib().oracle_fmm2d_adaptive(n, _d(pos), _d(q), L, p, int(near_max), side,
                                     _d(_f64(origin)), _d(pot), _d(fld), dep.ctypes.data)
    _check(rc, "fmm2d_adaptive")
    return pot, fld, dep


def fmm2d(pos, q, L, p, side=5.0, origin=(0.0, 0.0), classical=False, targets=None,
          field=True, dump_level=-1, split=False, level_p=None):
    """Shift-free (or, with classical=True, the shifted textbook) 2D FMM.

    Returns (pot, field) and, when dump_level >= 2, also (moments, locals) of
    every box at that level as complex arrays [n_boxes, p_k+1] in row-major box
    order; with split=True also (pot_far, pot_near).  level_p (length L + 1)
    sets the order of each level k >= 2 (shift-free only).
    """
    pos, q = _f64(pos), _f64(q)
    n = pos.shape[0]
    org = _f64(origin)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else len(tg)
    pot = np.zeros(nt)
    fld = np.zeros((nt, 2)) if field else None
    mom = loc = None
    lp = None
    if level_p is not None:
        lp = np.ascontiguousarray(level_p, dtype=np.int32)
        if lp.shape != (L + 1,):
            raise ValueError("level_p must have L + 1 entries")
    if dump_level >= 2:
        nbox = 4 ** dump_level
        pd = p if lp is None else int(lp[dump_level])
        mom = np.zeros((nbox, pd + 1, 2))
        loc = np.zeros((nbox, pd + 1, 2))
    pf = np.zeros(nt) if split else None
    pn = np.zeros(nt) if split else None
    rc = lib().oracle_fmm2d_ex(n, _d(pos), _d(q), L, p, side, _d(org), int(classical), nt,
                               _i(tg), _d(pot), _d(fld), dump_level, _d(mom), _d(loc), _d(pf),
                               _d(pn), None if lp is None else lp.ctypes.data)
    _check(rc, "fmm2d")
    out = [pot, fld]
    if dump_level >= 2:
        out += [mom[..., 0] + 1j * mom[..., 1], loc[..., 0] + 1j * loc[..., 1]]
    if split:
        out += [pf, pn]
    return tuple(out)


def p2m2d_point(pos, q, centre, s, p):
    pos, q = _f64(pos), _f64(q)
    out = np.zeros((p + 1, 2))
    lib().oracle_p2m2d_point(len(q), _d(pos), _d(q), centre[0], centre[1], s, p, _d(out))
    return out[:, 0] + 1j * out[:, 1]


def m2p2d_point(a, centre, s, x, y):
    a = np.ascontiguousarray(np.stack([a.real, a.imag], -1), dtype=np.float64)
    return lib().oracle_m2p2d_point(_d(a), len(a) - 1, centre[0], centre[1], s, x, y)


def fmm3d(pos, q, L, p, side=5.0, origin=(0.0, 0.0, 0.0), classical=False, targets=None,
          field=True, dump_level=-1):
    """Shift-free (or classical) 3D FMM with solid harmonics of degree <= p.

    With dump_level >= 2 also returns (moments, locals) at that level as complex
    arrays [n_boxes, (p+1)^2] indexed n*n + n + m (all orders -n..n)."""
    pos, q = _f64(pos), _f64(q)
    n = pos.shape[0]
    org = _f64(origin)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else len(tg)
    pot = np.zeros(nt)
    fld = np.zeros((nt, 3)) if field else None
    mom = loc = None
    nc = (p + 1) ** 2
    if dump_level >= 2:
        nbox = 8 ** dump_level
        mom = np.zeros((nbox, nc, 2))
        loc = np.zeros((nbox, nc, 2))
    rc = lib().oracle_fmm3d_ex(n, _d(pos), _d(q), L, p, side, _d(org), int(classical), nt,
                               _i(tg), _d(pot), _d(fld), dump_level, _d(mom), _d(loc))
    _check(rc, "fmm3d")
    out = [pot, fld]
    if dump_level >= 2:
        out += [mom[..., 0] + 1j * mom[..., 1], loc[..., 0] + 1j * loc[..., 1]]
    return tuple(out)


def sh_regular(p, r):
    out = np.zeros(((p + 1) ** 2, 2))
    lib().oracle_sh_regular(p, float(r[0]), float(r[1]), float(r[2]), _d(out))
    return out[:, 0] + 1j * out[:, 1]


def sh_irregular(p, r):
    out = np.zeros(((p + 1) ** 2, 2))
    lib().oracle_sh_irregular(p, float(r[0]), float(r[1]), float(r[2]), _d(out))
    return out[:, 0] + 1j * out[:, 1]


# ---------------------------------------------------------------------------
# Order-prediction MLP (3 -> 64 -> 64 -> 21, ReLU), FP64.  Parameter layout:
# W1[64][3], b1[64], W2[64][64], b2[64], W3[21][64], b3[21].
# ---------------------------------------------------------------------------
MLP_NPARAM = 64 * 3 + 64 + 64 * 64 + 64 + 21 * 64 + 21


def mlp_forward(w, x):
    w, x = _f64(w), _f64(x)
    y = np.zeros((x.shape[0], 21))
    lib().oracle_mlp_forward(_d(w), x.shape[0], _d(x), _d(y))
    return y


def mlp_loss_grad(w, x, t):
    """(loss, gradient) of the mean squared error over all outputs."""
    w, x, t = _f64(w), _f64(x), _f64(t)
    g = np.zeros(MLP_NPARAM)
    loss = lib().oracle_mlp_loss_grad(_d(w), x.shape[0], _d(x), _d(t), _d(g))
    return loss, g


def mlp_adam(w, g, m1, m2, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step, in place on w, m1, m2 (FP64 arrays)."""
    for a in (w, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().oracle_mlp_adam(len(w), _d(w), _d(g), _d(m1), _d(m2), step, lr, beta1, beta2, eps)


def lagrange_weights(u):
    """The four 1D weights f_i(u) and their derivatives at nodes (-2, -1, 1, 2)."""
    f = np.zeros(4)
    df = np.zeros(4)
    lib().oracle_lagrange_weights(float(u), _d(f), _d(df))
    return f, df


def fmm3d_lagrange(pos, q, L, side=5.0, origin=(0.0, 0.0, 0.0), targets=None, field=True,
                   dump_level=-1):
    """Shift-free 3D FMM with the fixed point-charge basis (4 x 4 x 4 points per box).

    With dump_level >= 2 also returns (moments, locals) of every box at that
    level as [n_boxes, 64] arrays (point i + 4 j + 16 l)."""
    pos, q = _f64(pos), _f64(q)
    n = pos.shape[0]
    org = _f64(origin)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else len(tg)
    pot = np.zeros(nt)
    fld = np.zeros((nt, 3)) if field else None
    mom = loc = None
    if dump_level >= 2:
        mom = np.zeros((8 ** dump_level, 64))
        loc = np.zeros((8 ** dump_level, 64))
    rc = lib().oracle_fmm3d_lagrange(n, _d(pos), _d(q), L, side, _d(org), nt, _i(tg), _d(pot),
                                     _d(fld), dump_level, _d(mom), _d(loc))
    _check(rc, "fmm3d_lagrange")
    out = [pot, fld]
    if dump_level >= 2:
        out += [mom, loc]
    return tuple(out)


PAPER_NODES = (-2.0, -1.0, 1.0, 2.0)


def chebyshev_nodes(n):
    """The n Chebyshev points of the first kind on a box of side s, in units of
    s / 5 about its centre, ascending: 2.5 cos((2i + 1) pi / (2n))."""
    return tuple(sorted(2.5 * np.cos((2 * i + 1) * np.pi / (2 * n)) for i in range(n)))


def lagrange_weights_nodes(u, nodes):
    """The 1D weights f_i(u) and their derivatives for an arbitrary node set."""
    nd = _f64(nodes)
    f = np.zeros(len(nd))
    df = np.zeros(len(nd))
    _check(lib().oracle_lagrange_weights_nodes(len(nd), _d(nd), float(u), _d(f), _d(df)),
           "lagrange_weights_nodes")
    return f, df


def fmm3d_lagrange_nodes(pos, q, L, nodes, side=5.0, origin=(0.0, 0.0, 0.0), targets=None,
                         field=True, dump_level=-1):
    """fmm3d_lagrange with n = len(nodes) points per axis at `nodes` (units of
    s / 5 from the box centre): d = n^3 point charges per box."""
    pos, q = _f64(pos), _f64(q)
    nd = _f64(nodes)
    d = len(nd) ** 3
    n = pos.shape[0]
    org = _f64(origin)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else len(tg)
    pot = np.zeros(nt)
    fld = np.zeros((nt, 3)) if field else None
    mom = loc = None
    if dump_level >= 2:
        mom = np.zeros((8 ** dump_level, d))
        loc = np.zeros((8 ** dump_level, d))
    rc = lib().oracle_fmm3d_lagrange_nodes(len(nd), _d(nd), n, _d(pos), _d(q), L, side, _d(org),
                                           nt, _i(tg), _d(pot), _d(fld), dump_level, _d(mom),
                                           _d(loc))
    _check(rc, "fmm3d_lagrange_nodes")
    out = [pot, fld]
    if dump_level >= 2:
        out += [mom, loc]
    return tuple(out)


def fmm2d_lagrange(pos, q, L, nodes=PAPER_NODES, side=5.0, origin=(0.0, 0.0), targets=None,
                   field=True, dump_level=-1):
    """Shift-free 2D FMM (log kernel) with the fixed point-charge basis: n x n
    points per box at `nodes` (units of s / 5 from the centre; the paper's
    4 x 4 by default), point i + n j.  With dump_level >= 2 also returns
    (moments, locals) of every box at that level as [4^level, n^2] arrays."""
    pos, q = _f64(pos), _f64(q)
    nd = _f64(nodes)
    d = len(nd) ** 2
    n = pos.shape[0]
    org = _f64(origin)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else len(tg)
    pot = np.zeros(nt)
    fld = np.zeros((nt, 2)) if field else None
    mom = loc = None
    if dump_level >= 2:
        mom = np.zeros((4 ** dump_level, d))
        loc = np.zeros((4 ** dump_level, d))
    rc = lib().oracle_fmm2d_lagrange_nodes(len(nd), _d(nd), n, _d(pos), _d(q), L, side, _d(org),
                                           nt, _i(tg), _d(pot), _d(fld), dump_level, _d(mom),
                                           _d(loc))
    _check(rc, "fmm2d_lagrange")
    out = [pot, fld]
    if dump_level >= 2:
        out += [mom, loc]
    return tuple(out)


def lagrange_transfer(k, box, nodes=PAPER_NODES, side=5.0, origin=(0.0, 0.0, 0.0)):
    """STEP4's M_m for box (bx, by, bz) of level k: [d, d], M[i, j] = h_m(p_j)[i]."""
    nd, org = _f64(nodes), _f64(origin)
    d = len(nd) ** 3
    M = np.zeros((d, d))
    _check(lib().oracle_lagrange_transfer(len(nd), _d(nd), side, _d(org), k, int(box[0]),
                                          int(box[1]), int(box[2]), _d(M)), "lagrange_transfer")
    return M


def lagrange_box_weights(k, box, x, nodes=PAPER_NODES, side=5.0, origin=(0.0, 0.0, 0.0)):
    """h_m(x) of a unit charge at x for box (bx, by, bz) of level k: [d]."""
    nd, org, xx = _f64(nodes), _f64(origin), _f64(x)
    w = np.zeros(len(nd) ** 3)
    _check(lib().oracle_lagrange_box_weights(len(nd), _d(nd), side, _d(org), k, int(box[0]),
                                             int(box[1]), int(box[2]), _d(xx), _d(w)),
           "lagrange_box_weights")
    return w


def fmm3d_lagrange_root(pos, q, L, nodes=PAPER_NODES, side=5.0, origin=(0.0, 0.0, 0.0),
                        targets=None, field=True):
    """The point-charge method in the root frame (Section 2.2.1 with Appendix
    STEP4-STEP5: child sums, M_m^T M_b M_mi bilinear forms, parent-to-child
    additions).  Returns (pot, field, largest |entry| of the transfers M_m)."""
    pos, q = _f64(pos), _f64(q)
    nd = _f64(nodes)
    n = pos.shape[0]
    org = _f64(origin)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else len(tg)
    pot = np.zeros(nt)
    fld = np.zeros((nt, 3)) if field else None
    mt = np.zeros(1)
    rc = lib().oracle_fmm3d_lagrange_root(len(nd), _d(nd), n, _d(pos), _d(q), L, side, _d(org),
                                          nt, _i(tg), _d(pot), _d(fld), _d(mt))
    _check(rc, "fmm3d_lagrange_root")
    return pot, fld, float(mt[0])
