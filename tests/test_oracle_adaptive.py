"""Pins of the oracle's adaptive-depth 2D evaluation.

The paper's tree is uniform; for clustered inputs a particle's tree stops at
the first level whose 3 x 3 boxes around its box hold at most near_max
particles, and every particle runs the shift-free method of its own depth d(i):
the interaction-list forms of its ancestors at levels 2..d(i) plus the direct
sum over the 3 x 3 boxes around its level-d(i) box (Section 2.2.1 with the tree
of Section 2.1 cut at d(i)).  Pinned by:
  * the depth rule against brute-force box counts;
  * the partition identity: for every particle, the interaction lists at
    levels 2..d(i) and the level-d(i) neighbourhood cover every other particle
    exactly once (a missing or doubled box fails it);
  * agreement with the direct sum at p = 30 on clustered inputs whose depths
    span several levels (the method's error bound there is far below 1e-10);
  * the special cases that reduce to the pinned uniform oracle: near_max = 0
    (every leaf at level L, bit-identical) and near_max >= N (every leaf at
    level 2).
"""
import numpy as np
import pytest

import oracle
import workloads

SIDE = 5.0


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def clustered(n, seed):
    # tight and loose clusters, so that the depths span several levels
    pos, q = workloads.gaussian_mixture(n, 2, seed=seed, ncomp=4, sigma=0.08)
    rng = np.random.default_rng(seed + 1)
    bg = rng.uniform(0, SIDE, size=(n // 8, 2))
    return np.concatenate([pos, bg]), np.concatenate([q, rng.uniform(-1, 1, n // 8)])


def leaf_coords(pos, L):
    return np.array([[oracle.leaf_coord(x, 0.0, SIDE, L) for x in p] for p in pos], np.int64)


def brute_depth(pos, L, near_max):
    lc = leaf_coords(pos, L)
    d = np.empty(len(pos), np.int32)
    for i in range(len(pos)):
        k = 2
        while k < L:
            sh = L - k
            around = np.all(np.abs((lc >> sh) - (lc[i] >> sh)) <= 1, axis=1)
            if around.sum() <= near_max:
                break
            k += 1
        d[i] = k
    return d


@pytest.mark.parametrize("near_max", [0, 40, 150, 500, 10 ** 6])
def test_depth_rule(near_max):
    pos, q = clustered(1200, 3)
    L = 6
    _, _, dep = oracle.fmm2d_adaptive(pos, q, L, 6, near_max)
    np.testing.assert_array_equal(dep, brute_depth(pos, L, near_max))


def test_partition_identity():
    pos, q = clustered(600, 4)
    L, near_max = 6, 80
    _, _, dep = oracle.fmm2d_adaptive(pos, q, L, 4, near_max)
    assert len(set(dep.tolist())) >= 3
    lc = leaf_coords(pos, L)
    n = len(pos)
    for i in range(0, n, 7):
        cover = np.zeros(n, np.int64)
        for k in range(2, dep[i] + 1):
            b = lc >> (L - k)
            for bx, by in oracle.ilist2d(k, *(lc[i] >> (L - k))):
                cover += (b[:, 0] == bx) & (b[:, 1] == by)
        b = lc >> (L - dep[i])
        cover += np.all(np.abs(b - b[i]) <= 1, axis=1)
        want = np.ones(n, np.int64)
        want[i] = 1  # its own box covers the particle once; the sum skips it
        assert np.array_equal(cover, want), i


@pytest.mark.parametrize("seed,L,near_max", [(5, 6, 120), (6, 7, 300), (7, 5, 60)])
def test_matches_direct_sum(seed, L, near_max):
    pos, q = clustered(1500, seed)
    pot, fld, dep = oracle.fmm2d_adaptive(pos, q, L, 30, near_max)
    d, fd = oracle.direct(pos, q)
    print(f"depths {np.bincount(dep)[2:]}, rel-L2 pot {rel(pot, d):.2e} field {rel(fld, fd):.2e}")
    assert len(set(dep.tolist())) >= 3
    assert rel(pot, d) < 1e-12 and rel(fld, fd) < 1e-11


def test_zero_leaf_size_is_the_uniform_tree():
    pos, q = clustered(1000, 8)
    a, fa, dep = oracle.fmm2d_adaptive(pos, q, 5, 12, 0)
    assert np.all(dep == 5)
    b, fb = oracle.fmm2d(pos, q, 5, 12)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(fa, fb)


def test_large_leaf_size_is_level_two():
    pos, q = clustered(1000, 9)
    a, fa, dep = oracle.fmm2d_adaptive(pos, q, 6, 12, len(q))
    assert np.all(dep == 2)
    b, fb = oracle.fmm2d(pos, q, 2, 12)
    assert rel(a, b) < 1e-13 and rel(fa, fb) < 1e-13
