"""GPU parity of the 2D log-kernel method with the paper's fixed point-charge
box vectors (4 x 4 points per box, Appendix STEP1-STEP3 in the square box)
against the CPU oracle, for the paper's node set and the Chebyshev points.

FP64 mode must match the oracle to 1e-12 relative L2 (potentials and fields,
and every element within 1e-11 of the RMS) and per-level box vectors to 1e-13;
FP32 mode 1e-6 on potentials and 1e-3 on fields, the bars of the 2D expansion
path.  Edge cases: trees without an interaction list (levels 0, 1), a ragged
particle count, clustered inputs with empty boxes, one particle, and the
deepest tree the oracle finishes in seconds."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")

FP32_FIELD_TOL = 1e-3
KERNELS = {F.FMM_LOG2D_POINTS: oracle.PAPER_NODES,
           F.FMM_LOG2D_CHEBYSHEV: oracle.chebyshev_nodes(4)}


def rel(a, b):
    b = np.asarray(b)
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def max_over_rms(a, b):
    d = np.abs(a - b) if a.ndim == 1 else np.linalg.norm(a - b, axis=1)
    return float(d.max() / max(np.linalg.norm(b) / np.sqrt(len(b)), 1e-300))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(kernel, pos, q, L, precision=F.FMM_FP64, keep=False, npts=4):
    n = len(q)
    print(f"points2d kernel={kernel} n={n} L={L} precision={precision} points/axis={npts}",
          flush=True)
    f = F.FMM(kernel, levels=L, order=npts, max_particles=max(n, 1), flags=F.FMM_SYNC_CHECK,
              precision=precision)
    pot, fld = f.evaluate(dev(pos), dev(q))
    torch.cuda.synchronize()
    out = pot.cpu().numpy(), fld.cpu().numpy()
    if keep:
        return out, f
    f.close()
    return out


def compact2(v):
    v = v & 0x55555555
    v = (v | (v >> 1)) & 0x33333333
    v = (v | (v >> 2)) & 0x0F0F0F0F
    v = (v | (v >> 4)) & 0x00FF00FF
    v = (v | (v >> 8)) & 0x0000FFFF
    return v


def gpu_level_rows(f, k, which):
    """[4^k, 16] rows of level k in row-major box order (x fastest)."""
    cs = F.fmm_coef_stride(f.plan)
    nb = 4 ** k
    raw = np.frombuffer(F.fmm_debug_level_data(f.plan, k, which, 8 * nb * cs),
                        np.float64).reshape(nb, cs)
    b = np.arange(nb)
    rm = compact2(b >> 1) * (1 << k) + compact2(b)
    res = np.empty_like(raw)
    res[rm] = raw
    return res


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("precision,tol", [(F.FMM_FP64, 1e-13), (F.FMM_FP32, 5e-6)])
def test_box_vectors_match_oracle(kernel, precision, tol):
    pos, q = workloads.plus_minus_one(20000, 2, seed=91)
    L = 5
    (_, _), f = run(kernel, pos, q, L, precision=precision, keep=True)
    assert F.fmm_coef_stride(f.plan) == 16 and F.fmm_coef_order(f.plan) == 4
    for k in (2, 3, 5):
        _, _, om, ol = oracle.fmm2d_lagrange(pos, q, L, nodes=KERNELS[kernel], dump_level=k,
                                             field=False, targets=np.array([0]))
        gm = gpu_level_rows(f, k, F.FMM_DBG_MOMENTS)
        gl = gpu_level_rows(f, k, F.FMM_DBG_LOCALS)
        em = np.abs(gm - om).max() / np.abs(om).max()
        el = np.abs(gl - ol).max() / np.abs(ol).max()
        print(f"level {k}: moments {em:.2e}, locals {el:.2e}")
        assert em < tol and el < tol
    f.close()


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("kind,n,L", [("pm1", 30000, 5), ("uniform", 12345, 4),
                                      ("mixture", 40000, 6), ("pm1", 20000, 2)])
def test_potentials_match_oracle(kernel, kind, n, L):
    gen = {"pm1": workloads.plus_minus_one, "uniform": workloads.uniform,
           "mixture": workloads.gaussian_mixture}[kind]
    pos, q = gen(n, 2, seed=n + L)
    want, wantf = oracle.fmm2d_lagrange(pos, q, L, nodes=KERNELS[kernel])
    got, gotf = run(kernel, pos, q, L)
    print(f"{kind} n={n} L={L}: FP64 pot {rel(got, want):.2e} field {rel(gotf, wantf):.2e}")
    assert rel(got, want) <= 1e-12 and rel(gotf, wantf) <= 1e-12
    assert max_over_rms(got, want) <= 1e-11 and max_over_rms(gotf, wantf) <= 1e-11
    g32, g32f = run(kernel, pos, q, L, precision=F.FMM_FP32)
    print(f"{kind} n={n} L={L}: FP32 pot {rel(g32, want):.2e} field {rel(g32f, wantf):.2e}")
    assert rel(g32, want) <= 1e-6
    assert rel(g32f, wantf) <= FP32_FIELD_TOL


def test_trees_without_interaction_lists_equal_the_direct_sum():
    pos, q = workloads.plus_minus_one(3000, 2, seed=7)
    d, fd = oracle.direct(pos, q)
    for L in (0, 1):
        got, gotf = run(F.FMM_LOG2D_POINTS, pos, q, L)
        assert rel(got, d) < 1e-13 and rel(gotf, fd) < 1e-13


def test_one_particle_and_zero_charges():
    pos = np.array([[1.3, 2.7]])
    got, gotf = run(F.FMM_LOG2D_POINTS, pos, np.array([0.5]), 4)
    assert got[0] == 0 and np.all(gotf == 0)
    pos, q = workloads.uniform(5000, 2, seed=8)
    got, gotf = run(F.FMM_LOG2D_POINTS, pos, 0 * q, 5, precision=F.FMM_FP32)
    assert np.all(got == 0) and np.all(gotf == 0)


def test_accuracy_against_the_direct_sum_at_level_8():
    """2^18 random +1/-1 charges at level 8 (4 particles per leaf): the GPU
    result against the oracle's direct sum at 1000 seeded targets, and against
    the oracle's own point-charge evaluation there."""
    pos, q = workloads.plus_minus_one(1 << 18, 2, seed=9)
    tg = workloads.sample_targets(len(q), 1000, 1009)
    d, _ = oracle.direct(pos, q, targets=tg)
    want, _ = oracle.fmm2d_lagrange(pos, q, 8, targets=tg)
    got, _ = run(F.FMM_LOG2D_POINTS, pos, q, 8)
    g32, _ = run(F.FMM_LOG2D_POINTS, pos, q, 8, precision=F.FMM_FP32)
    print(f"level 8: FP64 vs oracle {rel(got[tg], want):.2e}, vs direct {rel(got[tg], d):.2e}; "
          f"FP32 vs oracle {rel(g32[tg], want):.2e}")
    assert rel(got[tg], want) <= 1e-12
    assert rel(g32[tg], want) <= 1e-6
    assert 1e-6 < rel(got[tg], d) < 1e-3


def test_repeated_evaluations_are_identical():
    pos, q = workloads.gaussian_mixture(30000, 2, seed=10)
    f = F.FMM(F.FMM_LOG2D_POINTS, levels=6, order=4, max_particles=len(q), precision=F.FMM_FP32)
    dpos, dq = dev(pos), dev(q)
    a, af = f.evaluate(dpos, dq)
    other = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, len(q))).cuda()
    f.evaluate(dpos, other)  # overwrite every box row with other values
    b, bf = f.evaluate(dpos, dq)
    torch.cuda.synchronize()
    f.close()
    assert torch.equal(a, b) and torch.equal(af, bf)


@pytest.mark.parametrize("npts", [2, 3, 5, 6, 7, 8])
def test_other_point_counts_match_oracle(npts):
    """n x n Chebyshev points per box (d = n^2, padded to 16, 32, 48 or 64 on
    the matrix cores): box vectors and potentials against the oracle with the
    same node set."""
    pos, q = workloads.plus_minus_one(20000, 2, seed=100 + npts)
    L = 5
    nodes = oracle.chebyshev_nodes(npts)
    want, wantf, om, ol = oracle.fmm2d_lagrange(pos, q, L, nodes=nodes, dump_level=4)
    (got, gotf), f = run(F.FMM_LOG2D_CHEBYSHEV, pos, q, L, keep=True, npts=npts)
    d = npts * npts
    assert F.fmm_coef_order(f.plan) == npts and F.fmm_coef_stride(f.plan) == (d + 15) // 16 * 16
    gm = gpu_level_rows(f, 4, F.FMM_DBG_MOMENTS)
    gl = gpu_level_rows(f, 4, F.FMM_DBG_LOCALS)
    f.close()
    assert np.abs(gm[:, :d] - om).max() <= 1e-13 * np.abs(om).max()
    assert np.abs(gl[:, :d] - ol).max() <= 1e-13 * np.abs(ol).max()
    assert np.all(gm[:, d:] == 0)
    print(f"n={npts}: FP64 pot {rel(got, want):.2e} field {rel(gotf, wantf):.2e}")
    assert rel(got, want) <= 1e-12 and rel(gotf, wantf) <= 1e-12
    g32, g32f = run(F.FMM_LOG2D_CHEBYSHEV, pos, q, L, precision=F.FMM_FP32, npts=npts)
    print(f"n={npts}: FP32 pot {rel(g32, want):.2e} field {rel(g32f, wantf):.2e}")
    assert rel(g32, want) <= 1e-6 and rel(g32f, wantf) <= FP32_FIELD_TOL


def test_accuracy_falls_with_the_points_per_axis():
    """Discussion (4): d is a free parameter.  On the GPU (FP64) the error
    against the direct sum at 2000 seeded targets falls by more than 3x per
    added Chebyshev point from n = 3 to 8."""
    pos, q = workloads.plus_minus_one(1 << 17, 2, seed=12)
    tg = workloads.sample_targets(len(q), 2000, 1012)
    d, _ = oracle.direct(pos, q, targets=tg)
    errs = []
    for npts in range(3, 9):
        got, _ = run(F.FMM_LOG2D_CHEBYSHEV, pos, q, 7, npts=npts)
        errs.append(rel(got[tg], d))
    print("n = 3..8:", ", ".join(f"{e:.2e}" for e in errs))
    for a, b in zip(errs, errs[1:]):
        assert b < a / 3
