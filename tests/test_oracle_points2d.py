"""Pins of the oracle's 2D point-charge passes (Appendix STEP1-STEP3 in the
square box: n x n points per box, the paper's 4 x 4 at offsets {-2, -1, 1, 2}
s / 5 about the centre, the log kernel).

  * STEP2 (box vectors) against the polynomial moments it must preserve: for
    every box, sum_i M_i P(y_i) = sum_particles q P(x) for each tensor monomial
    of degree < n per axis (eq. (1)); a transposed point index, a wrong centre
    or a wrong scale fails this;
  * STEP3 and the local evaluation against charges placed exactly on points of
    boxes in each other's interaction list: the far field is then q log r with
    no interpolation error (a transposed operator, a wrong offset sign or a
    wrong spacing fails);
  * the field against the finite-difference gradient of the potential;
  * the direct sum: degenerate trees (levels 0 and 1: no interaction list)
    equal it to rounding, deeper trees lie within a few 1e-4, and with
    Chebyshev points the error falls geometrically with the points per axis;
  * zero charges give zero.
"""
import itertools

import numpy as np
import pytest

import oracle
import workloads

SIDE = 5.0


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("nodes", [oracle.PAPER_NODES, oracle.chebyshev_nodes(4),
                                   oracle.chebyshev_nodes(5)])
@pytest.mark.parametrize("k", [2, 3])
def test_box_vectors_preserve_polynomial_moments(nodes, k):
    pos, q = workloads.uniform(3000, 2, seed=21 + k)
    L = 4
    _, _, mom, _ = oracle.fmm2d_lagrange(pos, q, L, nodes=nodes, dump_level=k)
    a = np.array(nodes)
    n = len(a)
    nb = 1 << k
    s = SIDE / nb
    ix = np.minimum((pos[:, 0] / s).astype(int), nb - 1)
    iy = np.minimum((pos[:, 1] / s).astype(int), nb - 1)
    ux = 5.0 * (pos[:, 0] - (ix + 0.5) * s) / s
    uy = 5.0 * (pos[:, 1] - (iy + 0.5) * s) / s
    px = np.tile(a, n)       # point i + n j has x offset a_i
    py = np.repeat(a, n)     # and y offset a_j
    for b in range(nb * nb):
        sel = (iy * nb + ix) == b
        for ex, ey in itertools.product(range(n), range(n)):
            want = np.sum(q[sel] * ux[sel] ** ex * uy[sel] ** ey)
            got = np.sum(mom[b] * px ** ex * py ** ey)
            scale = np.sum(np.abs(q[sel])) * 2.5 ** (ex + ey) + 1e-300
            assert abs(got - want) <= 1e-12 * scale, (b, ex, ey, got, want)
    # the total charge of a box is its first moment
    assert np.allclose(mom.sum(axis=1).sum(), q.sum(), atol=1e-10)


def test_charges_on_points_are_exact():
    """Two charges on points of boxes (0, 1) and (3, 2) at level 2 (in each
    other's interaction list; no other particle): the far field equals the pair
    potential exactly, and so do the potentials, the near field being empty."""
    a = np.array(oracle.PAPER_NODES)
    s = SIDE / 4
    rng = np.random.default_rng(5)
    for _ in range(8):
        ps = (np.array([0, 1]) + 0.5) * s + a[rng.integers(0, 4, 2)] * s / 5
        pt = (np.array([3, 2]) + 0.5) * s + a[rng.integers(0, 4, 2)] * s / 5
        pos = np.stack([ps, pt])
        q = np.array([0.7, -1.3])
        pot, fld = oracle.fmm2d_lagrange(pos, q, 2)
        r = np.linalg.norm(ps - pt)
        assert abs(pot[0] - q[1] * np.log(r)) < 1e-13
        assert abs(pot[1] - q[0] * np.log(r)) < 1e-13
        # and against the direct sum
        d, _ = oracle.direct(pos, q)
        np.testing.assert_allclose(pot, d, rtol=0, atol=1e-13)


def test_field_is_minus_gradient():
    pos, q = workloads.plus_minus_one(1500, 2, seed=31)
    L = 4
    h = 1e-6
    tg = np.arange(0, 1500, 97)
    _, fld = oracle.fmm2d_lagrange(pos, q, L, targets=tg)
    for ax in range(2):
        pp, pm = pos.copy(), pos.copy()
        pp[tg, ax] += h
        pm[tg, ax] -= h
        # moving one target at a time keeps the others' contributions fixed
        fd = np.zeros(len(tg))
        for e, i in enumerate(tg):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, ax] += h
            p2[i, ax] -= h
            if (int(p1[i, ax] / (SIDE / 16)) != int(pos[i, ax] / (SIDE / 16))
                    or int(p2[i, ax] / (SIDE / 16)) != int(pos[i, ax] / (SIDE / 16))):
                fd[e] = np.nan  # the step leaves the leaf: the piecewise form jumps
                continue
            up, _ = oracle.fmm2d_lagrange(p1, q, L, targets=[i], field=False)
            dn, _ = oracle.fmm2d_lagrange(p2, q, L, targets=[i], field=False)
            fd[e] = -(up[0] - dn[0]) / (2 * h)
        ok = np.isfinite(fd)
        assert ok.sum() >= 10
        np.testing.assert_allclose(fld[ok, ax], fd[ok], rtol=1e-6, atol=1e-6)


def test_degenerate_trees_equal_the_direct_sum():
    pos, q = workloads.plus_minus_one(900, 2, seed=41)
    d, fd = oracle.direct(pos, q)
    for L in (0, 1):
        pot, fld = oracle.fmm2d_lagrange(pos, q, L)
        assert rel(pot, d) < 1e-13 and rel(fld, fd) < 1e-13
    pot, fld = oracle.fmm2d_lagrange(pos, 0 * q, 4)
    assert np.all(pot == 0) and np.all(fld == 0)


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_accuracy_against_the_direct_sum(L):
    pos, q = workloads.plus_minus_one(4000, 2, seed=3)
    d, fd = oracle.direct(pos, q)
    pot, fld = oracle.fmm2d_lagrange(pos, q, L)
    e, ef = rel(pot, d), rel(fld, fd)
    print(f"level {L}: potential {e:.2e}, field {ef:.2e}")
    assert 1e-6 < e < 5e-4 and ef < 5e-3


def test_chebyshev_points_converge_geometrically():
    pos, q = workloads.plus_minus_one(4000, 2, seed=3)
    d, _ = oracle.direct(pos, q)
    errs = [rel(oracle.fmm2d_lagrange(pos, q, 4, nodes=oracle.chebyshev_nodes(n))[0], d)
            for n in (3, 4, 5, 6, 8)]
    print("chebyshev n = 3, 4, 5, 6, 8:", ", ".join(f"{e:.2e}" for e in errs))
    for a, b in zip(errs, errs[1:]):
        assert b < 0.3 * a
    assert errs[-1] < 1e-6
