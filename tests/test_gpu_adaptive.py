"""The adaptive-depth 2D evaluation (adaptive_near = T > 0) against the oracle's
adaptive evaluation on the same inputs: FP64 to 1e-12, FP32 and BF16-M2L to
1e-6 relative L2 of the potentials, on clustered inputs whose depths span
several levels; T = 0 (every particle at the finest level) reproduces the
uniform tree bit for bit in FP64."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def clustered(n, seed):
    pos, q = workloads.gaussian_mixture(n, 2, seed=seed, ncomp=4, sigma=0.08)
    rng = np.random.default_rng(seed + 1)
    bg = rng.uniform(0, 5.0, size=(n // 8, 2))
    return np.concatenate([pos, bg]), np.concatenate([q, rng.uniform(-1, 1, n // 8)])


def run(pos, q, L, p, near, precision=F.FMM_FP64, flags=F.FMM_SYNC_CHECK):
    f = F.FMM(F.FMM_LOG2D, levels=L, order=p, max_particles=len(q), precision=precision,
              flags=flags, adaptive_near=near)
    pot, fld = f.evaluate(dev(pos), dev(q))
    torch.cuda.synchronize()
    st = f.last_status()
    f.close()
    assert st == F.FMM_OK
    return pot.cpu().numpy(), fld.cpu().numpy()


CASES = [(20000, 11, 7, 12, 200), (30000, 12, 8, 16, 600), (8000, 13, 6, 20, 80)]


@pytest.mark.parametrize("n,seed,L,p,near", CASES)
def test_fp64_matches_oracle(n, seed, L, p, near):
    pos, q = clustered(n, seed)
    want, wfld, dep = oracle.fmm2d_adaptive(pos, q, L, p, near)
    assert len(set(dep.tolist())) >= 3
    pot, fld = run(pos, q, L, p, near)
    print(f"n={len(q)} L={L} s={near}: depths {np.bincount(dep)[2:]}, "
          f"pot {rel(pot, want):.2e} field {rel(fld, wfld):.2e}")
    assert rel(pot, want) < 1e-12 and rel(fld, wfld) < 1e-12


@pytest.mark.parametrize("precision", [F.FMM_FP32, F.FMM_BF16_M2L])
@pytest.mark.parametrize("n,seed,L,p,near", CASES)
def test_mixed_precision_within_tolerance(n, seed, L, p, near, precision):
    pos, q = clustered(n, seed)
    want, wfld, _ = oracle.fmm2d_adaptive(pos, q, L, p, near)
    pot, fld = run(pos, q, L, p, near, precision=precision)
    e, ef = rel(pot, want), rel(fld, wfld)
    print(f"precision {precision} n={len(q)} L={L} s={near}: pot {e:.2e} field {ef:.2e}")
    assert e < 1e-6 and ef < 1e-4


def test_zero_leaf_size_is_the_uniform_tree():
    pos, q = clustered(20000, 14)
    a, fa = run(pos, q, 6, 12, 0)
    f = F.FMM(F.FMM_LOG2D, levels=6, order=12, max_particles=len(q), flags=F.FMM_SYNC_CHECK)
    b, fb = f.evaluate(dev(pos), dev(q))
    torch.cuda.synchronize()
    f.close()
    np.testing.assert_array_equal(a, b.cpu().numpy())
    np.testing.assert_array_equal(fa, fb.cpu().numpy())


def test_repeat_and_smaller_input():
    """A second evaluation with fewer particles on the same plan (the depth
    mask and the rebased records are rewritten every call)."""
    pos, q = clustered(20000, 15)
    f = F.FMM(F.FMM_LOG2D, levels=7, order=12, max_particles=len(q), precision=F.FMM_FP32,
              flags=F.FMM_SYNC_CHECK, adaptive_near=200)
    for m in (len(q), 5000):
        want, _, _ = oracle.fmm2d_adaptive(pos[:m], q[:m], 7, 12, 200)
        pot, _ = f.evaluate(dev(pos[:m]), dev(q[:m]))
        torch.cuda.synchronize()
        assert rel(pot.cpu().numpy(), want) < 1e-6
    f.close()
