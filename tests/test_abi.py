"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/fmm.h declares, validates arguments on the host and reports a
missing device."""
import ctypes
import os
import re

import pytest

import paper_2009_00767_amd as F

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "fmm.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z0-9_]+\*?\s+\*?(fmm_[a-z0-9_]+)\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "fmm_plan" in names and "fmm_eval" in names
    lib = F.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(F.EXPORTED) == sorted(names)


def test_binding_constants_match_the_header():
    src = open(HEADER).read()
    consts = dict(re.findall(r"^\s*(FMM_[A-Z0-9_]+)\s*=\s*(-?\d+)", src, re.M))
    consts.update(re.findall(r"^#define\s+(FMM_[A-Z0-9_]+)\s+(-?\d+)", src, re.M))
    assert len(consts) > 20
    for name, value in consts.items():
        assert hasattr(F, name), name
        assert getattr(F, name) == int(value), name


def test_status_strings_cover_all_codes():
    for s in (0, -1, -2, -3, -4, -5, -6, 1):
        assert F.fmm_status_str(s) not in ("", "unknown status")
    assert F.fmm_status_str(12345) == "unknown status"


def test_default_options():
    o = F.fmm_default_options(F.FMM_LOG2D)
    assert o.side == 5.0 and o.kernel == F.FMM_LOG2D and o.precision == F.FMM_FP64
    with pytest.raises(F.FmmError):
        F.fmm_default_options(7)


@pytest.mark.parametrize("field,value", [("levels", -1), ("levels", 13), ("order_p", 0),
                                         ("order_p", 31), ("precision", 5), ("side", -1.0),
                                         ("max_particles", -5), ("flags", 256),
                                         ("order_policy", 3), ("adaptive_near", -1)])
def test_plan_rejects_invalid_options(field, value):
    o = F.fmm_default_options(F.FMM_LOG2D)
    setattr(o, field, value)
    with pytest.raises(F.FmmError) as e:
        F.fmm_plan(o)
    assert e.value.status == F.FMM_ERR_INVALID_ARG


def test_null_plan_and_arguments():
    lib = F.lib()
    assert lib.fmm_eval(None, 1, None, None, None, None, None) == F.FMM_ERR_INVALID_ARG
    assert lib.fmm_last_status(None) == F.FMM_ERR_INVALID_ARG
    assert lib.fmm_destroy(None) == F.FMM_OK
    assert lib.fmm_plan(None, None) == F.FMM_ERR_INVALID_ARG


def test_no_device_reported_on_cpu_host():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    o = F.fmm_default_options(F.FMM_LOG2D)
    with pytest.raises(F.FmmError) as e:
        F.fmm_plan(o)
    assert e.value.status == F.FMM_ERR_DEVICE


def test_learned_order_option_checks():
    o = F.fmm_default_options(F.FMM_LOG2D)
    o.flags = F.FMM_JUDGE  # the judge needs the learned policy
    with pytest.raises(F.FmmError) as e:
        F.fmm_plan(o)
    assert e.value.status == F.FMM_ERR_INVALID_ARG
    o = F.fmm_default_options(F.FMM_LOG2D)
    o.order_policy = F.FMM_ORDER_LEARNED
    o.tol = 0.0
    with pytest.raises(F.FmmError) as e:
        F.fmm_plan(o)
    assert e.value.status == F.FMM_ERR_INVALID_ARG
    o = F.fmm_default_options(F.FMM_COULOMB3D)
    o.order_policy = F.FMM_ORDER_LEARNED
    with pytest.raises(F.FmmError) as e:
        F.fmm_plan(o)
    assert e.value.status == F.FMM_ERR_UNSUPPORTED


def test_adaptive_depth_option_checks():
    """adaptive_near > 0: 2D, one system, fixed order, levels >= 2 only."""
    cases = [(F.FMM_COULOMB3D, "levels", 3), (F.FMM_LOG2D, "max_systems", 8),
             (F.FMM_LOG2D, "levels", 1), (F.FMM_LOG2D, "order_policy", F.FMM_ORDER_LEARNED)]
    for kernel, field, value in cases:
        o = F.fmm_default_options(kernel)
        o.adaptive_near = 32
        setattr(o, field, value)
        with pytest.raises(F.FmmError) as e:
            F.fmm_plan(o)
        assert e.value.status == F.FMM_ERR_UNSUPPORTED, field


def test_mlp_entry_points_check_arguments():
    lib = F.lib()
    assert lib.fmm_set_order_model(None, None, F.FMM_MLP_NPARAM) == F.FMM_ERR_INVALID_ARG
    assert lib.fmm_mlp_forward(None, None, 5, None, None) == F.FMM_ERR_INVALID_ARG
    assert lib.fmm_mlp_forward(None, None, -1, None, None) == F.FMM_ERR_INVALID_ARG
    assert lib.fmm_mlp_loss_grad(None, None, None, 4, None, None, None) == F.FMM_ERR_INVALID_ARG
    assert lib.fmm_mlp_adam_step(None, None, None, None, 1, 1e-3, None) == F.FMM_ERR_INVALID_ARG
    assert lib.fmm_mlp_train(None, None, None, 4, 10, 1e-3, None, None) == F.FMM_ERR_INVALID_ARG
    assert lib.fmm_set_level_orders(None, None, 3) == F.FMM_ERR_INVALID_ARG


@pytest.mark.parametrize("kernel", [F.FMM_COULOMB3D_POINTS, F.FMM_COULOMB3D_CHEBYSHEV,
                                    F.FMM_LOG2D_POINTS, F.FMM_LOG2D_CHEBYSHEV])
def test_point_charge_basis_option_checks(kernel):
    o = F.fmm_default_options(kernel)
    two_d = kernel in (F.FMM_LOG2D_POINTS, F.FMM_LOG2D_CHEBYSHEV)
    assert o.kernel == kernel and o.order_p == 4 and o.levels == (4 if two_d else 3)
    # 4 points per axis, or 2..8 for the 2D Chebyshev points, 2..5 for the 3D ones
    for n in {F.FMM_LOG2D_CHEBYSHEV: (1, 9), F.FMM_COULOMB3D_CHEBYSHEV: (1, 6)}.get(kernel,
                                                                                  (3, 5)):
        o.order_p = n
        with pytest.raises(F.FmmError) as e:
            F.fmm_plan(o)
        assert e.value.status == F.FMM_ERR_UNSUPPORTED
    bad = [("order_policy", F.FMM_ORDER_LEARNED), ("precision", F.FMM_BF16_M2L),
           ("max_systems", 8)]
    if two_d:  # adaptive depth and the root frame: not for the 2D point charges
        bad += [("adaptive_near", 100), ("flags", F.FMM_ROOT_FRAME)]
    for field, value in bad:
        o = F.fmm_default_options(kernel)
        setattr(o, field, value)
        if field == "flags":
            o.precision = F.FMM_FP64
        with pytest.raises(F.FmmError) as e:
            F.fmm_plan(o)
        assert e.value.status == F.FMM_ERR_UNSUPPORTED, field
    o = F.fmm_default_options(kernel)
    for k in (0, 7, -1):
        o.kernel = k
        with pytest.raises(F.FmmError) as e:
            F.fmm_plan(o)
        assert e.value.status == F.FMM_ERR_INVALID_ARG
    with pytest.raises(F.FmmError) as e:
        F.fmm_default_options(7)


def test_noalloc_limits_are_checked_on_the_host():
    """The plan-free entry point rejects inputs beyond its fixed scratch, and
    options it does not cover, before touching the device."""
    o = F.fmm_default_options(F.FMM_LOG2D)
    o.levels, o.order_p = 4, 12
    for field, value in (("levels", 7), ("order_p", 21)):
        bad = F.fmm_default_options(F.FMM_LOG2D)
        ctypes.pointer(bad)[0] = o
        setattr(bad, field, value)
        with pytest.raises(F.FmmError) as e:
            F.fmm_eval_noalloc(bad, 16, 1, 1, 1, 1, 0)
        assert e.value.status == F.FMM_ERR_SCRATCH
    with pytest.raises(F.FmmError) as e:
        F.fmm_eval_noalloc(o, (1 << 16) + 1, 1, 1, 1, 1, 0)
    assert e.value.status == F.FMM_ERR_SCRATCH
    for field, value in (("kernel", F.FMM_COULOMB3D), ("precision", F.FMM_BF16_M2L),
                         ("order_policy", F.FMM_ORDER_LEARNED), ("flags", F.FMM_TIMING),
                         ("max_systems", 2)):
        bad = F.fmm_default_options(F.FMM_LOG2D)
        ctypes.pointer(bad)[0] = o
        setattr(bad, field, value)
        with pytest.raises(F.FmmError) as e:
            F.fmm_eval_noalloc(bad, 16, 1, 1, 1, 1, 0)
        assert e.value.status == F.FMM_ERR_UNSUPPORTED
    with pytest.raises(F.FmmError) as e:  # a missing output
        F.fmm_eval_noalloc(o, 16, 1, 1, None, 1, 0)
    assert e.value.status == F.FMM_ERR_INVALID_ARG
    assert F.fmm_eval_noalloc(o, 0, None, None, None, None, 0) == F.FMM_OK


def test_root_frame_needs_point_charges_in_fp64():
    for kernel, prec in ((F.FMM_COULOMB3D, F.FMM_FP64), (F.FMM_LOG2D, F.FMM_FP64),
                         (F.FMM_COULOMB3D_POINTS, F.FMM_FP32),
                         (F.FMM_COULOMB3D_CHEBYSHEV, F.FMM_FP32)):
        o = F.fmm_default_options(kernel)
        o.precision, o.flags = prec, F.FMM_ROOT_FRAME
        with pytest.raises(F.FmmError) as e:
            F.fmm_plan(o)
        assert e.value.status == F.FMM_ERR_UNSUPPORTED
    o = F.fmm_default_options(F.FMM_COULOMB3D_CHEBYSHEV)
    assert o.order_p == 4 and o.kernel == F.FMM_COULOMB3D_CHEBYSHEV
    for n in (3, 5):  # the root frame takes 4 points per axis only
        o.order_p, o.precision, o.flags = n, F.FMM_FP64, F.FMM_ROOT_FRAME
        with pytest.raises(F.FmmError) as e:
            F.fmm_plan(o)
        assert e.value.status == F.FMM_ERR_UNSUPPORTED
