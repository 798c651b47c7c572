"""What the packaged order model gains on the 512-system batched workload
(N log-uniform in [1k, 64k], uniform or Gaussian mixture; held out from the
model's training systems): the learned orders must keep every system within
the tolerance of the fixed order p = 20 in FP64 (the judge's reference) while
cutting the far-field work (interaction-list contractions, 8 (p + 1)^2 flop per
pair at each level's order) at least in half.  The step times of both are
printed, not asserted: the near field of the mixture systems is most of the
step and runs beside the far field, so the far-field saving shows in the step
time only within the noise of one run."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")
from paper_2009_00767_amd import order_model  # noqa: E402

TOL = 1e-6


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def batch():
    systems = workloads.batched_systems(512, 2, seed=5)
    off = np.zeros(len(systems) + 1, np.int64)
    off[1:] = np.cumsum([len(qs) for _, qs in systems])
    pos = torch.from_numpy(np.concatenate([ps for ps, _ in systems])).cuda()
    q = torch.from_numpy(np.concatenate([qs for _, qs in systems])).cuda()
    return systems, off, pos, q


def plan(n, precision, learned, flags=0):
    f = F.FMM(F.FMM_LOG2D, levels=8, order=20, max_particles=n, precision=precision,
              flags=flags, max_systems=512, max_levels=8, tol=TOL,
              order_policy=F.FMM_ORDER_LEARNED if learned else F.FMM_ORDER_FIXED)
    if learned:
        w, _ = order_model.load()
        f.set_order_model(w)
    return f


def timed(f, off, pos, q, reps=10):
    pot = torch.empty(q.shape[0], dtype=torch.float64, device="cuda")
    fld = torch.empty((q.shape[0], 2), dtype=torch.float64, device="cuda")
    for _ in range(3):
        f.evaluate_batched(off, pos, q, pot=pot, field=fld)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        f.evaluate_batched(off, pos, q, pot=pot, field=fld)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return pot.cpu().numpy(), fld.cpu().numpy(), float(np.median(ts))


@pytest.mark.parametrize("precision", [F.FMM_FP64, F.FMM_FP32])
def test_learned_orders_meet_tolerance_and_cut_far_field_work(batch, precision):
    systems, off, pos, q = batch
    n = q.shape[0]
    ref = plan(n, F.FMM_FP64, False)
    p20, f20, _ = timed(ref, off, pos, q, reps=1)
    ref.close()
    fixed = plan(n, precision, False)
    _, _, t_fixed = timed(fixed, off, pos, q)
    fixed.close()
    lrn = plan(n, precision, True)
    pl, fl, t_learned = timed(lrn, off, pos, q)
    st = lrn.stats()
    orders = list(st.order_per_level[:9])
    assert lrn.last_status() == F.FMM_OK and st.fallback == 0
    lrn.close()
    err = rel(pl, p20)
    per_sys = max(rel(pl[off[s]:off[s + 1]], p20[off[s]:off[s + 1]]) for s in range(len(systems)))
    # far-field work at the chosen orders against the fixed order 20 (per depth
    # group the order of each level is the largest over its systems, an upper
    # bound of what ran)
    work_fixed = work_learned = 0.0
    for ps, qs in systems:
        L = order_model.default_depth(len(qs), 8)
        for k in range(2, L + 1):
            n = 1 << k
            pairs = (6 * n - 8) ** 2 - (3 * n - 2) ** 2
            work_fixed += 8 * 21 ** 2 * pairs
            work_learned += 8 * (orders[k] + 1) ** 2 * pairs
    print(f"precision {precision}: orders {orders}, rel-L2 vs fixed p=20 FP64 {err:.3e} "
          f"(worst system {per_sys:.3e}), far-field work x{work_learned / work_fixed:.3f}, "
          f"fixed {t_fixed:.3f} ms, learned {t_learned:.3f} ms")
    assert err <= TOL
    assert per_sys <= TOL
    assert max(orders[2:]) <= 24 and min(o for o in orders[2:] if o) >= 4
    assert work_learned < 0.5 * work_fixed


def test_judge_accepts_the_packaged_model(batch):
    systems, off, pos, q = batch
    f = plan(q.shape[0], F.FMM_FP32, True, flags=F.FMM_JUDGE)
    f.evaluate_batched(off, pos, q)
    torch.cuda.synchronize()
    st = f.stats()
    print(f"judge: largest per-system rel-L2 {st.judge_rel_err:.3e}")
    assert f.last_status() == F.FMM_OK
    assert st.fallback == 0 and st.judge_rel_err <= TOL
    f.close()
