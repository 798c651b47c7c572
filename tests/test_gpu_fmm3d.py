"""GPU parity of the 3D (1/r, solid harmonics) shift-free FMM against the CPU
oracle.  FP64 mode must match the oracle to 1e-12 relative L2, per-level box
vectors to 1e-13; FP32 mode 1e-6 on potentials (fields stated: 1e-3, see the
2D tests for why).  Sort results must be bit-exact."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")

FP32_FIELD_TOL = 1e-3


def rel(a, b):
    b = np.asarray(b)
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(pos, q, L, p, precision=F.FMM_FP64, flags=F.FMM_SYNC_CHECK, keep=False, side=5.0,
        origin=(0.0, 0.0, 0.0)):
    n = len(q)
    f = F.FMM(F.FMM_COULOMB3D, levels=L, order=p, max_particles=max(n, 1), flags=flags,
              precision=precision, side=side, origin=origin)
    pot, fld = f.evaluate(dev(pos), dev(q))
    torch.cuda.synchronize()
    out = pot.cpu().numpy(), (fld.cpu().numpy() if fld is not None else None)
    if keep:
        return out, f
    f.close()
    return out


def spread3(v):
    v = v & 0x3FF
    v = (v | (v << 16)) & 0x030000FF
    v = (v | (v << 8)) & 0x0300F00F
    v = (v | (v << 4)) & 0x030C30C3
    v = (v | (v << 2)) & 0x09249249
    return v


def compact3(v):
    v = v & 0x09249249
    v = (v | (v >> 2)) & 0x030C30C3
    v = (v | (v >> 4)) & 0x0300F00F
    v = (v | (v >> 8)) & 0x030000FF
    v = (v | (v >> 16)) & 0x000003FF
    return v


def leaf_keys3(pos, L, side=5.0):
    nl = 1 << L
    c = np.minimum(np.floor(pos * (float(nl) / side)).astype(np.int64), nl - 1)
    return spread3(c[:, 0]) | (spread3(c[:, 1]) << 1) | (spread3(c[:, 2]) << 2)


def gpu_level_coeffs3(f, k, which, p):
    """Coefficients (n, m >= 0) of every box at level k, row-major boxes, as a
    complex array indexed like the oracle's n*n + n + m (m < 0 left zero)."""
    cs = F.fmm_coef_stride(f.plan)
    pb = F.fmm_coef_order(f.plan)
    nb = 8 ** k
    raw = np.frombuffer(F.fmm_debug_level_data(f.plan, k, which, 8 * nb * cs),
                        np.float64).reshape(nb, cs)
    out = np.zeros((nb, (p + 1) ** 2), complex)
    out[:, 0] = raw[:, (pb + 1) ** 2 - 1]
    for n in range(1, p + 1):
        out[:, n * n + n] = raw[:, n * n - 1]
        for m in range(1, n + 1):
            out[:, n * n + n + m] = raw[:, n * n - 1 + 2 * m - 1] + 1j * raw[:, n * n - 1 + 2 * m]
    b = np.arange(nb)
    rm = (compact3(b >> 2) * (1 << k) + compact3(b >> 1)) * (1 << k) + compact3(b)
    res = np.empty_like(out)
    res[rm] = out
    return res


def nonneg(c, p):
    idx = [n * n + n + m for n in range(p + 1) for m in range(0, n + 1)]
    return c[:, idx]


# (20000, 3): 9-bit keys beyond the two-digit sort's mean-bucket bound (LSD
# passes); (50000, 5) and (4000, 3): the two-digit sort, in both precisions.
@pytest.mark.parametrize("n,L,prec", [(20000, 3, F.FMM_FP64), (50000, 5, F.FMM_FP64),
                                      (3000, 1, F.FMM_FP64), (50000, 5, F.FMM_FP32),
                                      (4000, 3, F.FMM_FP32)])
def test_sort_3d_bit_exact(n, L, prec):
    pos, q = workloads.uniform(n, 3, seed=70)
    (_, _), f = run(pos, q, L, 4, keep=True, precision=prec)
    perm = np.frombuffer(F.fmm_debug_level_data(f.plan, 0, F.FMM_DBG_PERM, 4 * n), np.int32)
    nleaf = 8 ** L
    ls = np.frombuffer(F.fmm_debug_level_data(f.plan, 0, F.FMM_DBG_LEAF_START, 4 * (nleaf + 1)),
                       np.int32)
    f.close()
    k = leaf_keys3(pos, L)
    want = np.argsort(k, kind="stable")
    np.testing.assert_array_equal(perm, want)
    np.testing.assert_array_equal(ls, np.searchsorted(k[want], np.arange(nleaf + 1), "left"))


# FP32 box vectors: every stored value carries a relative rounding of 2^-24 and
# each local is a sum over 189 offsets of 81-term products formed in FP32 with
# FP64 sums across offsets; 5e-6 leaves a margin of about 8x over sqrt(81) 2^-24.
@pytest.mark.parametrize("precision,tol", [(F.FMM_FP64, 1e-13), (F.FMM_FP32, 5e-6)])
def test_box_vectors_3d_match_oracle(precision, tol):
    pos, q = workloads.uniform(6000, 3, seed=71)
    L, p = 3, 8
    (_, _), f = run(pos, q, L, p, precision=precision, keep=True)
    for k in (2, 3):
        gm = gpu_level_coeffs3(f, k, F.FMM_DBG_MOMENTS, p)
        gl = gpu_level_coeffs3(f, k, F.FMM_DBG_LOCALS, p)
        _, _, om, ol = oracle.fmm3d(pos, q, L, p, dump_level=k)
        assert rel(nonneg(gm, p), nonneg(om, p)) < tol, k
        assert rel(nonneg(gl, p), nonneg(ol, p)) < tol, k
    f.close()


@pytest.mark.parametrize("L,p", [(3, 8), (2, 4), (4, 6), (3, 2)])
def test_fmm3d_end_to_end_fp64(L, p):
    pos, q = workloads.uniform(8000, 3, seed=72 + L + p)
    pot, fld = run(pos, q, L, p)
    want, wfld = oracle.fmm3d(pos, q, L, p)
    assert rel(pot, want) < 1e-12 and rel(fld, wfld) < 1e-12


def test_fmm3d_truncation_against_direct():
    pos, q = workloads.uniform(4096, 3, seed=73)
    pot, fld = run(pos, q, 3, 8)
    pd, fd = oracle.direct(pos, q)
    assert rel(pot, pd) < 1e-4 and rel(fld, fd) < 1e-3


@pytest.mark.parametrize("L,p", [(3, 8), (4, 4), (5, 8)])
def test_fmm3d_fp32(L, p):
    pos, q = workloads.uniform(30000, 3, seed=74 + L)
    pot, fld = run(pos, q, L, p, precision=F.FMM_FP32)
    want, wfld = oracle.fmm3d(pos, q, L, p)
    assert rel(pot, want) < 1e-6 and rel(fld, wfld) < FP32_FIELD_TOL


def test_fmm3d_degenerate_and_edges():
    pos, q = workloads.uniform(2500, 3, seed=75)
    pd, fd = oracle.direct(pos, q)
    for L in (0, 1):
        pot, fld = run(pos, q, L, 4)
        assert rel(pot, pd) < 1e-13 and rel(fld, fd) < 1e-13
    edge = pos.copy()
    edge[:30, 2] = 5.0
    edge[30:60, 0] = 0.0
    edge[60, :] = 5.0
    pot, fld = run(edge, q, 4, 8)
    want, wfld = oracle.fmm3d(edge, q, 4, 8)
    assert rel(pot, want) < 1e-12 and rel(fld, wfld) < 1e-12
    mix = workloads.gaussian_mixture(20000, 3, seed=76)
    pot, fld = run(mix[0], mix[1], 5, 8)
    want, wfld = oracle.fmm3d(mix[0], mix[1], 5, 8)
    assert rel(pot, want) < 1e-12 and rel(fld, wfld) < 1e-12
    pot, fld = run(mix[0], mix[1], 5, 8, precision=F.FMM_FP32)
    assert rel(pot, want) < 1e-6 and rel(fld, wfld) < FP32_FIELD_TOL


@pytest.mark.parametrize("L", [3, 2])
def test_fmm3d_coincident_points(L):
    """Exact duplicates of 500 particles with other charges: pairs at r = 0
    contribute nothing (the self term's rule) in both modes.  At level 2 a
    target meets about 8400 sources and the near field runs eight waves per 64
    targets, at level 3 four."""
    pos, q = workloads.uniform(20000, 3, seed=78)
    pos[-500:] = pos[:500]
    want, wfld = oracle.fmm3d(pos, q, L, 8)
    pot, fld = run(pos, q, L, 8)
    assert rel(pot, want) < 1e-12 and rel(fld, wfld) < 1e-12
    pot, fld = run(pos, q, L, 8, precision=F.FMM_FP32)
    assert np.all(np.isfinite(pot)) and np.all(np.isfinite(fld))
    assert rel(pot, want) < 1e-6 and rel(fld, wfld) < FP32_FIELD_TOL


def test_fmm3d_sign_symmetry_and_determinism():
    pos, q = workloads.uniform(40000, 3, seed=77)
    for prec in (F.FMM_FP64, F.FMM_FP32):
        a, fa = run(pos, q, 5, 8, precision=prec)
        b, fb = run(pos, -q, 5, 8, precision=prec)
        c, fc = run(pos, q, 5, 8, precision=prec)
        np.testing.assert_array_equal(b, -a)
        np.testing.assert_array_equal(fb, -fa)
        np.testing.assert_array_equal(c, a)


def test_4m_workload_sampled():
    """N = 2^22 uniform in a cube of side 5, level 7, order 8: FP32 against FP64
    over all particles, both against the oracle at 256 seeded targets."""
    pos, q = workloads.uniform(1 << 22, 3, seed=4)
    p64, f64 = run(pos, q, 7, 8)
    p32, f32 = run(pos, q, 7, 8, precision=F.FMM_FP32)
    assert rel(p32, p64) < 1e-6
    tg = workloads.sample_targets(1 << 22, 256, seed=1004)
    want, wfld = oracle.fmm3d(pos, q, 7, 8, targets=tg)
    assert rel(p64[tg], want) < 1e-12 and rel(f64[tg], wfld) < 1e-12
    assert rel(p32[tg], want) < 1e-6
