"""The plan-free, allocation-free entry point fmm_eval_noalloc against the plan
entry point fmm_eval, through the C ABI, on the same seeded inputs.

Two calls in a row share the library's fixed device array; the second takes a
smaller input (fewer particles, a shallower tree, a lower order), so that what
the first call left in the array must not leak into the second.  Tolerances
are the parity bar of each mode: FP64 1e-12 relative L2 (and every element
within 1e-11 of the RMS), FP32 1e-6 relative L2 of the potential.  Both entry
points run the same kernels in the same order, so the differences come only
from the operators, which the plan builds on the host and the plan-free call
builds on the device.  The plan-free results are also held to the oracle at
the same bars.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_over_rms(a, b):
    d = np.abs(a - b) if a.ndim == 1 else np.linalg.norm(a - b, axis=1)
    return float(d.max() / (np.linalg.norm(b) / np.sqrt(len(b))))


def noalloc(pos, q, L, p, precision):
    o = F.fmm_default_options(F.FMM_LOG2D)
    o.levels, o.order_p, o.precision = L, p, precision
    n = len(q)
    dpos, dq = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
    pot = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    fld = torch.full((n, 2), float("nan"), dtype=torch.float64, device="cuda")
    rc = F.fmm_eval_noalloc(o, n, dpos, dq, pot, fld)
    assert rc == F.FMM_OK
    torch.cuda.synchronize()
    return pot.cpu().numpy(), fld.cpu().numpy()


def planned(pos, q, L, p, precision):
    f = F.FMM(F.FMM_LOG2D, levels=L, order=p, max_particles=len(q), precision=precision,
              flags=F.FMM_SYNC_CHECK)
    pot, fld = f.evaluate(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    out = pot.cpu().numpy(), fld.cpu().numpy()
    f.close()
    return out


CASES = [  # (kind, n, L, p): the first call, then a smaller one
    (("mixture", 65536, 6, 20), ("uniform", 3000, 4, 12)),
    (("uniform", 40000, 6, 16), ("mixture", 20000, 5, 9)),
]


@pytest.mark.parametrize("precision", [F.FMM_FP64, F.FMM_FP32])
@pytest.mark.parametrize("calls", CASES)
def test_noalloc_matches_plan_on_two_calls(calls, precision):
    for kind, n, L, p in calls:
        gen = workloads.uniform if kind == "uniform" else workloads.gaussian_mixture
        pos, q = gen(n, 2, seed=n + L)
        print(f"noalloc {kind} n={n} L={L} p={p} precision={precision}", flush=True)
        got, gotf = noalloc(pos, q, L, p, precision)
        want, wantf = planned(pos, q, L, p, precision)
        assert np.all(np.isfinite(got)) and np.all(np.isfinite(gotf))
        if precision == F.FMM_FP64:
            assert rel(got, want) <= 1e-12, rel(got, want)
            assert rel(gotf, wantf) <= 1e-12, rel(gotf, wantf)
            assert max_over_rms(got, want) <= 1e-11
            assert max_over_rms(gotf, wantf) <= 1e-11
        else:
            assert rel(got, want) <= 1e-6, rel(got, want)
        # and against the oracle at the same bar (the oracle's FP64 method)
        if n <= 40000:
            ref, reff = oracle.fmm2d(pos, q, L, p)
            assert rel(got, ref) <= (1e-12 if precision == F.FMM_FP64 else 1e-6)


def test_noalloc_reports_a_position_outside_the_box():
    pos, q = workloads.uniform(1000, 2, seed=9)
    pos[17, 0] = 5.5
    o = F.fmm_default_options(F.FMM_LOG2D)
    o.levels, o.order_p, o.flags = 3, 8, F.FMM_SYNC_CHECK
    pot = torch.empty(1000, dtype=torch.float64, device="cuda")
    fld = torch.empty((1000, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(F.FmmError) as e:
        F.fmm_eval_noalloc(o, 1000, torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda(),
                           pot, fld)
    assert e.value.status == F.FMM_ERR_DOMAIN
    # the next call starts with clean status words
    pos[17, 0] = 4.5
    assert F.fmm_eval_noalloc(o, 1000, torch.from_numpy(pos).cuda(),
                              torch.from_numpy(q).cuda(), pot, fld) == F.FMM_OK
