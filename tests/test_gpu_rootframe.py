"""GPU parity of the point-charge method on the Chebyshev node set
(FMM_COULOMB3D_CHEBYSHEV) and of the root-frame passes (FMM_ROOT_FRAME)
against the oracle.

Chebyshev points: FP64 1e-12 relative L2 end to end and 1e-13 for box vectors,
FP32 1e-6 on potentials, the bars of the paper's node set.

Root frame (FP64 only): the transfers M_m amplify rounding with the depth
(Discussion (3)); the oracle's own root frame differs from the box-local form
by 4e-11 at level 2, 3e-8 at level 3 and 2e-5 at level 4, so the bar is the
conditioning of the method, not FP64 rounding: 1e-9 at level 2, 1e-6 at level
3, 1e-3 at level 4 against the oracle's root frame (and the same against the
box-local result), exact agreement (1e-13) with the direct sum when there is
no far field (levels 0 and 1)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CHEB = oracle.chebyshev_nodes(4)
ROOT_TOL = {0: 1e-13, 1: 1e-13, 2: 1e-9, 3: 1e-6, 4: 1e-3}


def rel(a, b):
    b = np.asarray(b)
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(pos, q, L, kernel, precision=F.FMM_FP64, flags=F.FMM_SYNC_CHECK, keep=False):
    n = len(q)
    f = F.FMM(kernel, levels=L, order=4, max_particles=max(n, 1), flags=flags,
              precision=precision)
    print(f"kernel {kernel} n={n} L={L} precision={precision} flags={flags}", flush=True)
    pot, fld = f.evaluate(dev(pos), dev(q))
    torch.cuda.synchronize()
    out = pot.cpu().numpy(), (fld.cpu().numpy() if fld is not None else None)
    if keep:
        return out, f
    f.close()
    return out


def compact3(v):
    v = v & 0x09249249
    v = (v | (v >> 2)) & 0x030C30C3
    v = (v | (v >> 4)) & 0x0300F00F
    v = (v | (v >> 8)) & 0x030000FF
    v = (v | (v >> 16)) & 0x000003FF
    return v


def gpu_level_rows(f, k, which):
    cs = F.fmm_coef_stride(f.plan)
    nb = 8 ** k
    raw = np.frombuffer(F.fmm_debug_level_data(f.plan, k, which, 8 * nb * cs),
                        np.float64).reshape(nb, cs)
    b = np.arange(nb)
    rm = (compact3(b >> 2) * (1 << k) + compact3(b >> 1)) * (1 << k) + compact3(b)
    res = np.empty_like(raw)
    res[rm] = raw
    return res


@pytest.mark.parametrize("precision,tol", [(F.FMM_FP64, 1e-13), (F.FMM_FP32, 5e-6)])
def test_chebyshev_box_vectors_match_oracle(precision, tol):
    pos, q = workloads.plus_minus_one(6000, seed=181)
    L = 3
    (_, _), f = run(pos, q, L, F.FMM_COULOMB3D_CHEBYSHEV, precision=precision, keep=True)
    for k in (2, 3):
        gm = gpu_level_rows(f, k, F.FMM_DBG_MOMENTS)
        gl = gpu_level_rows(f, k, F.FMM_DBG_LOCALS)
        _, _, om, ol = oracle.fmm3d_lagrange_nodes(pos, q, L, CHEB, dump_level=k)
        s = 5.0 / 2 ** k
        assert rel(gm[:, :64], om) < tol, k
        assert rel(gl[:, :64] / s, ol) < tol, k
    f.close()


@pytest.mark.parametrize("n,L", [(3000, 2), (8000, 3), (20000, 4)])
def test_chebyshev_end_to_end(n, L):
    pos, q = workloads.plus_minus_one(n, seed=182 + L)
    tg = workloads.sample_targets(n, 1500, seed=1182)
    want, wfld = oracle.fmm3d_lagrange_nodes(pos, q, L, CHEB, targets=tg)
    pot, fld = run(pos, q, L, F.FMM_COULOMB3D_CHEBYSHEV)
    assert rel(pot[tg], want) < 1e-12 and rel(fld[tg], wfld) < 1e-12
    pot, fld = run(pos, q, L, F.FMM_COULOMB3D_CHEBYSHEV, precision=F.FMM_FP32)
    assert rel(pot[tg], want) < 1e-6 and rel(fld[tg], wfld) < 1e-3


def test_chebyshev_points_are_exact():
    nodes = np.array(CHEB)
    s = 5.0 / 4
    rng = np.random.default_rng(183)
    for _ in range(4):
        ps = (np.array([0, 1, 0]) + 0.5) * s + nodes[rng.integers(0, 4, 3)] * s / 5
        pt = (np.array([3, 2, 3]) + 0.5) * s + nodes[rng.integers(0, 4, 3)] * s / 5
        pos = np.stack([ps, pt])
        q = np.array([0.7, -1.3])
        pot, _ = run(pos, q, 2, F.FMM_COULOMB3D_CHEBYSHEV)
        r = np.linalg.norm(ps - pt)
        np.testing.assert_allclose(pot, [q[1] / r, q[0] / r], rtol=1e-13)


@pytest.mark.parametrize("kernel,nodes", [(F.FMM_COULOMB3D_POINTS, oracle.PAPER_NODES),
                                          (F.FMM_COULOMB3D_CHEBYSHEV, CHEB)])
@pytest.mark.parametrize("n,L", [(2000, 0), (2000, 1), (3000, 2), (6000, 3), (6000, 4)])
def test_root_frame_matches_oracle(kernel, nodes, n, L):
    pos, q = workloads.plus_minus_one(n, seed=190 + L)
    tg = workloads.sample_targets(n, 1000, seed=1190)
    flags = F.FMM_SYNC_CHECK | F.FMM_ROOT_FRAME
    pot, fld = run(pos, q, L, kernel, flags=flags)
    if L <= 1:
        want, wfld = oracle.direct(pos, q, targets=tg)
    elif L <= 3:
        want, wfld, _ = oracle.fmm3d_lagrange_root(pos, q, L, nodes, targets=tg)
    else:  # the oracle's level-4 root frame at these sizes is slow: its box-local form
        want, wfld = oracle.fmm3d_lagrange_nodes(pos, q, L, nodes, targets=tg)
    e, ef = rel(pot[tg], want), rel(fld[tg], wfld)
    print(f"root frame L={L}: rel-L2 {e:.2e} field {ef:.2e}")
    assert e < ROOT_TOL[L] and ef < ROOT_TOL[L]
    # and against the box-local GPU result, which meets 1e-12 against the oracle
    bp, bf = run(pos, q, L, kernel)
    assert rel(pot, bp) < ROOT_TOL[L] and rel(fld, bf) < ROOT_TOL[L]


def test_root_frame_paper_workload():
    """The paper's Table 2 run (200000 random +1/-1 charges, level 3) in the root
    frame: against the box-local result within the level-3 bar, and of the
    accuracy the paper prints against the direct sum."""
    pos, q, w = workloads.make("3d-pm1-200k-L3-n4")
    L = w["levels"]
    tg = workloads.sample_targets(w["n"], 1500, seed=1191)
    pr, fr = run(pos, q, L, F.FMM_COULOMB3D_POINTS, flags=F.FMM_SYNC_CHECK | F.FMM_ROOT_FRAME)
    pb, fb = run(pos, q, L, F.FMM_COULOMB3D_POINTS)
    assert rel(pr, pb) < ROOT_TOL[L] and rel(fr, fb) < ROOT_TOL[L]
    pd, fd = oracle.direct(pos, q, targets=tg)
    ep = np.mean(np.abs(pr[tg] - pd) / np.abs(pd))
    ef = np.mean(np.linalg.norm(fr[tg] - fd, axis=1) / np.linalg.norm(fd, axis=1))
    with open(os.path.join(GOLDEN, "lagrange_accuracy.json")) as f:
        paper = {(r["n"], r["levels"]): r["accuracy"] for r in json.load(f)["runs"]}
    acc = 0.5 * (ep + ef)
    assert paper[(w["n"], L)] / 4 < acc < 4 * paper[(w["n"], L)]


def test_root_frame_sign_symmetry_and_determinism():
    pos, q = workloads.plus_minus_one(30000, seed=192)
    flags = F.FMM_SYNC_CHECK | F.FMM_ROOT_FRAME
    a, fa = run(pos, q, 3, F.FMM_COULOMB3D_POINTS, flags=flags)
    b, fb = run(pos, -q, 3, F.FMM_COULOMB3D_POINTS, flags=flags)
    c, fc = run(pos, q, 3, F.FMM_COULOMB3D_POINTS, flags=flags)
    np.testing.assert_array_equal(b, -a)
    np.testing.assert_array_equal(fb, -fa)
    np.testing.assert_array_equal(c, a)
