"""Pins of the oracle's fixed point-charge (Lagrange) form of the 3D method.

The paper's own realisation of V (Appendix, STEP1-STEP5): 4 x 4 x 4 point
charges per box at offsets (-2, -1, 1, 2) s / 5 from the centre.  The oracle is
pinned to what the paper and the mathematics fix:
  * the interpolation identity of STEP2 (exact for polynomials of degree < 4,
    and so for their derivatives);
  * the moment identities that follow from it (charge, dipole and every
    tensor moment of degree <= 3 per axis are preserved by h_m);
  * exactness when both charges sit on fixed points (the map h_m is then the
    identity and the bilinear form of STEP3 is the pair potential itself);
  * the accuracy printed in the paper for its own runs (Section 3, Tables 1-3).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NODES = np.array([-2.0, -1.0, 1.0, 2.0])


def test_weights_interpolate_cubics_exactly():
    rng = np.random.default_rng(3)
    for u in np.linspace(-2.5, 2.5, 41):
        f, df = oracle.lagrange_weights(u)
        for _ in range(4):
            c = rng.standard_normal(4)
            g = np.polynomial.Polynomial(c)
            assert abs(f @ g(NODES) - g(u)) < 1e-12 * (1 + abs(g(u)))
            assert abs(df @ g(NODES) - g.deriv()(u)) < 1e-12 * (1 + abs(g.deriv()(u)))
    for i, a in enumerate(NODES):
        f, _ = oracle.lagrange_weights(a)
        assert np.allclose(f, np.eye(4)[i], atol=1e-15)


def _box_members(pos, L, k, side=5.0):
    nb = 2 ** k
    lc = np.minimum(np.floor(pos * (2 ** L / side)).astype(np.int64), 2 ** L - 1) >> (L - k)
    return lc[:, 0] + nb * lc[:, 1] + nb * nb * lc[:, 2], lc


@pytest.mark.parametrize("k", [2, 3])
def test_moments_keep_polynomial_moments(k):
    """h_m keeps sum q x^a y^b z^c for a, b, c <= 3 (a consequence of STEP2)."""
    L = 3
    pos, q = workloads.uniform(3000, dim=3, seed=11)
    _, _, mom, _ = oracle.fmm3d_lagrange(pos, q, L, dump_level=k, field=False)
    nb = 2 ** k
    s = 5.0 / nb
    box, lc = _box_members(pos, L, k)
    cen = (lc + 0.5) * s
    ii = np.arange(64)
    ux, uy, uz = NODES[ii & 3], NODES[(ii >> 2) & 3], NODES[ii >> 4]
    upos = 5.0 * (pos - cen) / s  # particle offsets in units s / 5
    for b in [0, 5, nb ** 3 - 1, (nb ** 3) // 2 + 3]:
        sel = box == b
        for a, bb, c in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 1, 0), (3, 3, 3),
                         (1, 2, 3)]:
            want = np.sum(q[sel] * upos[sel, 0] ** a * upos[sel, 1] ** bb * upos[sel, 2] ** c)
            got = np.sum(mom[b] * ux ** a * uy ** bb * uz ** c)
            assert abs(got - want) < 1e-10 * (1 + np.sum(np.abs(q[sel]))), (b, a, bb, c)


def test_point_charges_on_fixed_points_are_exact():
    """Two charges on fixed points of level-2 boxes in each other's interaction
    list: the far field is the exact pair potential (STEP2 maps each to itself)."""
    s = 5.0 / 4
    rng = np.random.default_rng(5)
    for _ in range(6):
        src_box = np.array([0, 1, 0])
        tgt_box = np.array([3, 2, 3])
        ps = (src_box + 0.5) * s + NODES[rng.integers(0, 4, 3)] * s / 5
        pt = (tgt_box + 0.5) * s + NODES[rng.integers(0, 4, 3)] * s / 5
        pos = np.stack([ps, pt])
        q = np.array([0.7, -1.3])
        pot, _ = oracle.fmm3d_lagrange(pos, q, 2)
        r = np.linalg.norm(ps - pt)
        assert abs(pot[0] - q[1] / r) < 1e-13 * abs(q[1] / r)
        assert abs(pot[1] - q[0] / r) < 1e-13 * abs(q[0] / r)


def test_adjacent_boxes_use_the_near_field_only():
    pos = np.array([[0.1, 0.1, 0.1], [1.3, 1.3, 1.3]])  # level-2 boxes (0,0,0) and (1,1,1)
    q = np.array([1.0, 2.0])
    pot, fld = oracle.fmm3d_lagrange(pos, q, 2)
    d, fd = oracle.direct(pos, q)
    assert np.allclose(pot, d, rtol=1e-14) and np.allclose(fld, fd, rtol=1e-13)


def test_linear_in_charges_and_translation_invariant():
    pos, q = workloads.plus_minus_one(4000, seed=12)
    tg = workloads.sample_targets(4000, 300)
    p1, f1 = oracle.fmm3d_lagrange(pos, q, 3, targets=tg)
    p2, f2 = oracle.fmm3d_lagrange(pos, -2.5 * q, 3, targets=tg)
    assert np.allclose(p2, -2.5 * p1, rtol=1e-12, atol=1e-12)
    # shifting particles and box together changes nothing but rounding
    p3, f3 = oracle.fmm3d_lagrange(pos + 7.25, q, 3, origin=(7.25, 7.25, 7.25), targets=tg)
    assert np.max(np.abs(p3 - p1)) < 1e-9 * np.max(np.abs(p1))


@pytest.mark.slow
def test_accuracy_matches_the_papers_tables():
    """Averaged relative error of potential and force against the direct sum
    at the paper's sizes (Section 3): the same order as the printed value (within
    a factor 4; the paper does not state how it drew its positions)."""
    with open(os.path.join(GOLDEN, "lagrange_accuracy.json")) as f:
        runs = json.load(f)["runs"]
    for run in runs:
        pos, q = workloads.plus_minus_one(run["n"], seed=20 + run["table"])
        tg = workloads.sample_targets(run["n"], 1500)
        pot, fld = oracle.fmm3d_lagrange(pos, q, run["levels"], targets=tg)
        pd, fd = oracle.direct(pos, q, targets=tg)
        ep = np.mean(np.abs(pot - pd) / np.abs(pd))
        ef = np.mean(np.linalg.norm(fld - fd, axis=1) / np.linalg.norm(fd, axis=1))
        acc = 0.5 * (ep + ef)
        assert run["accuracy"] / 4 < acc < 4 * run["accuracy"], (run, ep, ef)
