"""Pins of the oracle's root-frame passes and of its point charges on other node
sets (Chebyshev points, Discussion (1)).

Root frame (Section 2.2.1 with Appendix STEP4-STEP5): every box vector is a
vector of the root box's point charges (U-bar-1 sums over particles, U-bar-2
sums over children), the bilinear form of two boxes is M_mi^T M_b M_m, and the
linear forms pass from parent to child by addition (D-bar-2).  Pinned by:
  * STEP4's transfer against the box weights it must reproduce: M_m h_{m^0}(x)
    = h_m(x) for x in m (the Note closing Section 2.2.2, through eq. (1)); a
    transposed M_m, a wrong node offset or a wrong box centre fails this;
  * equality with the box-local form (itself pinned in test_oracle_lagrange.py)
    within the rounding that the growing transfer entries allow, the
    conditioning Discussion (3) warns about: measured 4e-11 at level 2, 3e-8 at
    level 3 and 2e-5 at level 4 (largest |M_m| 2.7e8, 2.7e11, 1.8e14);
  * degenerate cases (no far field below level 2, zero charges).
Chebyshev points: the node formula against numpy's Chebyshev points, the
interpolation identity of STEP2 for any distinct nodes, exactness for charges
on fixed points, and the geometric decay of the error with the number of
points per axis (tests/golden/lagrange_nodes_accuracy.json, written by
tests/golden/make_lagrange_nodes_accuracy.py from the oracle).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PAPER = np.array(oracle.PAPER_NODES)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("nodes", [oracle.PAPER_NODES, oracle.chebyshev_nodes(4),
                                   oracle.chebyshev_nodes(5)])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_transfer_maps_root_weights_to_box_weights(nodes, k):
    rng = np.random.default_rng(40 + k)
    nb = 2 ** k
    s = 5.0 / nb
    for _ in range(4):
        box = rng.integers(0, nb, 3)
        M = oracle.lagrange_transfer(k, box, nodes)
        for _ in range(3):
            x = (box + rng.uniform(0, 1, 3)) * s
            w0 = oracle.lagrange_box_weights(0, (0, 0, 0), x, nodes)
            wm = oracle.lagrange_box_weights(k, box, x, nodes)
            # rounding of a d-term sum of entries up to max|M|
            tol = 1e-14 * len(w0) * np.abs(M).max() * np.abs(w0).max()
            assert np.max(np.abs(M @ w0 - wm)) < tol
            assert np.max(np.abs(M.T @ w0 - wm)) > 1e3 * tol or k == 0


def test_transfer_of_the_root_is_the_identity():
    M = oracle.lagrange_transfer(0, (0, 0, 0))
    assert np.allclose(M, np.eye(64), atol=1e-14)


@pytest.mark.parametrize("L,tol", [(2, 1e-9), (3, 1e-6)])
def test_root_frame_equals_the_box_local_form(L, tol):
    pos, q = workloads.plus_minus_one(3000, 3, seed=11)
    want, wfld = oracle.fmm3d_lagrange(pos, q, L)
    got, gfld, mt = oracle.fmm3d_lagrange_root(pos, q, L)
    print(f"level {L}: root vs box-local {rel(got, want):.2e} (field {rel(gfld, wfld):.2e}), "
          f"largest transfer entry {mt:.2e}")
    assert rel(got, want) < tol and rel(gfld, wfld) < tol
    # the difference is rounding amplified by the transfers, far below the
    # method's own error against the direct sum
    d, fd = oracle.direct(pos, q)
    assert rel(got, want) < 1e-2 * rel(want, d)


def test_root_frame_with_chebyshev_points():
    pos, q = workloads.plus_minus_one(2500, 3, seed=14)
    nodes = oracle.chebyshev_nodes(4)
    want, wfld = oracle.fmm3d_lagrange_nodes(pos, q, 2, nodes)
    got, gfld, _ = oracle.fmm3d_lagrange_root(pos, q, 2, nodes)
    assert rel(got, want) < 1e-9 and rel(gfld, wfld) < 1e-9


def test_root_frame_degenerate_cases():
    pos, q = workloads.plus_minus_one(800, 3, seed=15)
    d, fd = oracle.direct(pos, q)
    for L in (0, 1):  # no interaction list: the near field covers every pair
        got, gfld, _ = oracle.fmm3d_lagrange_root(pos, q, L)
        assert rel(got, d) < 1e-13 and rel(gfld, fd) < 1e-13
    got, gfld, _ = oracle.fmm3d_lagrange_root(pos, 0 * q, 3)
    assert np.all(got == 0) and np.all(gfld == 0)


# ----- other node sets -------------------------------------------------------

@pytest.mark.parametrize("n", [3, 4, 5, 6, 8])
def test_chebyshev_nodes_are_the_first_kind_points(n):
    want = 2.5 * np.sort(np.polynomial.chebyshev.chebpts1(n))
    assert np.allclose(oracle.chebyshev_nodes(n), want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("nodes", [oracle.chebyshev_nodes(4), oracle.chebyshev_nodes(6),
                                   tuple(np.linspace(-2.0, 2.0, 5))])
def test_weights_interpolate_polynomials_for_any_nodes(nodes):
    a = np.array(nodes)
    n = len(a)
    rng = np.random.default_rng(n)
    for u in np.linspace(-2.5, 2.5, 23):
        f, df = oracle.lagrange_weights_nodes(u, nodes)
        for _ in range(3):
            g = np.polynomial.Polynomial(rng.standard_normal(n))
            assert abs(f @ g(a) - g(u)) < 1e-11 * (1 + abs(g(u)))
            assert abs(df @ g(a) - g.deriv()(u)) < 1e-10 * (1 + abs(g.deriv()(u)))
    for i in range(n):
        f, _ = oracle.lagrange_weights_nodes(a[i], nodes)
        assert np.allclose(f, np.eye(n)[i], atol=1e-14)


def test_paper_node_set_through_the_general_path():
    pos, q = workloads.plus_minus_one(2000, 3, seed=16)
    a, fa = oracle.fmm3d_lagrange(pos, q, 3)
    b, fb = oracle.fmm3d_lagrange_nodes(pos, q, 3, oracle.PAPER_NODES)
    assert np.array_equal(a, b) and np.array_equal(fa, fb)


def test_charges_on_chebyshev_points_are_exact():
    nodes = np.array(oracle.chebyshev_nodes(4))
    s = 5.0 / 4
    rng = np.random.default_rng(17)
    for _ in range(6):
        ps = (np.array([0, 1, 0]) + 0.5) * s + nodes[rng.integers(0, 4, 3)] * s / 5
        pt = (np.array([3, 2, 3]) + 0.5) * s + nodes[rng.integers(0, 4, 3)] * s / 5
        pos = np.stack([ps, pt])
        q = np.array([0.7, -1.3])
        pot, _ = oracle.fmm3d_lagrange_nodes(pos, q, 2, tuple(nodes))
        r = np.linalg.norm(ps - pt)
        assert abs(pot[0] - q[1] / r) < 1e-13 * abs(q[1] / r)
        assert abs(pot[1] - q[0] / r) < 1e-13 * abs(q[0] / r)


def test_accuracy_against_points_per_axis():
    """The stored accuracy-vs-d table (relative L2 error against the direct sum,
    20000 random +1/-1 charges, level 3) decays geometrically with the points
    per axis for the Chebyshev points, which are more accurate than the paper's
    set at the same d = 64; the oracle reproduces one row of it."""
    with open(os.path.join(GOLDEN, "lagrange_nodes_accuracy.json")) as f:
        tab = json.load(f)
    cheb = {r["n"]: r for r in tab["rows"] if r["nodes"] == "chebyshev"}
    for n in (3, 4, 5):
        assert cheb[n + 1]["rel_l2_pot"] < 0.3 * cheb[n]["rel_l2_pot"]
    paper = [r for r in tab["rows"] if r["nodes"] == "paper"][0]
    assert cheb[4]["rel_l2_pot"] < paper["rel_l2_pot"]
    assert cheb[4]["rel_l2_field"] < paper["rel_l2_field"]
    # one row recomputed
    pos, q = workloads.plus_minus_one(tab["n"], 3, seed=tab["seed"])
    tg = workloads.sample_targets(tab["n"], 2000, 1013)
    d, fd = oracle.direct(pos, q, targets=tg)
    got, gfld = oracle.fmm3d_lagrange_nodes(pos, q, tab["levels"], oracle.chebyshev_nodes(4),
                                            targets=tg)
    assert abs(rel(got, d) - cheb[4]["rel_l2_pot_sampled"]) < 1e-9
