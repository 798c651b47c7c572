"""GPU parity of per-level expansion orders (2D) against the oracle run with
the same orders: FP64 1e-12 relative L2, FP32 1e-6 on potentials; box vectors
of every level up to that level's order; batched trees; argument errors."""
import numpy as np
import pytest

import oracle
import workloads

from test_gpu_fmm2d import dev, gpu_level_coeffs, rel, FP32_FIELD_TOL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")


def run_orders(pos, q, L, p, orders, precision=F.FMM_FP64, keep=False):
    f = F.FMM(F.FMM_LOG2D, levels=L, order=p, max_particles=len(q), precision=precision,
              flags=F.FMM_SYNC_CHECK)
    f.set_level_orders(orders)
    pot, fld = f.evaluate(dev(pos), dev(q))
    torch.cuda.synchronize()
    out = pot.cpu().numpy(), fld.cpu().numpy()
    if keep:
        return out, f
    f.close()
    return out


@pytest.mark.parametrize("orders", [[0, 0, 20, 14, 9, 5, 12], [0, 0, 3, 7, 20, 1, 16],
                                    [0, 0, 20, 20, 20, 20, 20]])
@pytest.mark.parametrize("precision,tp,tf", [(F.FMM_FP64, 1e-12, 1e-12),
                                             (F.FMM_FP32, 1e-6, FP32_FIELD_TOL)])
def test_level_orders_match_oracle(orders, precision, tp, tf):
    pos, q = workloads.uniform(60000, 2, seed=401)
    L, p = 6, 20
    pot, fld = run_orders(pos, q, L, p, orders, precision)
    want, wfld = oracle.fmm2d(pos, q, L, p, level_p=orders)
    assert rel(pot, want) < tp and rel(fld, wfld) < tf


@pytest.mark.parametrize("precision,tol", [(F.FMM_FP64, 1e-13), (F.FMM_FP32, 1e-6)])
def test_level_orders_box_vectors(precision, tol):
    pos, q = workloads.uniform(8000, 2, seed=402)
    L, p = 4, 24
    orders = [0, 0, 11, 24, 6]
    (_, _), f = run_orders(pos, q, L, p, orders, precision, keep=True)
    for k in range(2, L + 1):
        pk = orders[k]
        _, _, om, ol = oracle.fmm2d(pos, q, L, p, level_p=orders, dump_level=k)
        gm = gpu_level_coeffs(f, k, F.FMM_DBG_MOMENTS, p)
        gl = gpu_level_coeffs(f, k, F.FMM_DBG_LOCALS, pk)
        assert rel(gm[:, :pk + 1], om) < tol, k
        assert np.all(gm[:, pk + 1:] == 0), k  # moments above the level's order are zero
        ol[:, 0] = ol[:, 0].real  # Im B_0 is not formed (it enters no result)
        assert rel(gl, ol) < tol, k
    f.close()


def test_level_orders_batched():
    systems = workloads.batched_systems(20, 2, seed=403, nmin=300, nmax=30000)
    off = np.zeros(len(systems) + 1, np.int64)
    off[1:] = np.cumsum([len(qs) for _, qs in systems])
    pos = np.concatenate([ps for ps, _ in systems])
    q = np.concatenate([qs for _, qs in systems])
    lmax, p = 6, 20
    orders = [0, 0, 18, 13, 10, 8, 6]
    f = F.FMM(F.FMM_LOG2D, levels=lmax, order=p, max_particles=len(q), max_systems=len(systems),
              max_levels=lmax, flags=F.FMM_SYNC_CHECK)
    f.set_level_orders(orders)
    pot, fld = f.evaluate_batched(off, dev(pos), dev(q))
    torch.cuda.synchronize()
    pot, fld = pot.cpu().numpy(), fld.cpu().numpy()
    for s, (ps, qs) in enumerate(systems):
        n = len(qs)
        L = int(min(max(int(np.floor(np.log(n / 16.0) / np.log(4.0) + 0.5)), 2), lmax))
        want, wfld = oracle.fmm2d(ps, qs, L, p, level_p=orders[:L + 1])
        a, b = off[s], off[s + 1]
        assert rel(pot[a:b], want) < 1e-12 and rel(fld[a:b], wfld) < 1e-12, s
    f.close()


def test_level_orders_errors_and_stats():
    f = F.FMM(F.FMM_LOG2D, levels=4, order=12, max_particles=100)
    with pytest.raises(F.FmmError):
        f.set_level_orders([0, 0, 12, 12])  # one entry per level 0..4 needed
    with pytest.raises(F.FmmError):
        f.set_level_orders([0, 0, 12, 13, 12])  # above the plan's order
    with pytest.raises(F.FmmError):
        f.set_level_orders([0, 0, 12, 0, 12])
    f.set_level_orders([0, 0, 5, 8, 12])
    assert list(f.stats().order_per_level[:5]) == [0, 0, 5, 8, 12]
    f.close()
    g = F.FMM(F.FMM_COULOMB3D, levels=3, order=4, max_particles=100)
    with pytest.raises(F.FmmError):
        g.set_level_orders([0, 0, 4, 4])
    g.close()
