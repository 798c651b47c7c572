"""Pins of the oracle's per-level order and of its order-prediction MLP
(forward, loss gradient, Adam), checked against properties that do not come
from the oracle itself: exact special cases, finite differences, closed forms
of the Adam recursion and the independence of the levels in the shift-free
method."""
import numpy as np
import pytest

import oracle
import workloads


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


# --- per-level order --------------------------------------------------------

def test_level_order_equal_orders_is_fixed_order():
    pos, q = workloads.uniform(3000, 2, seed=301)
    a, fa = oracle.fmm2d(pos, q, 4, 12)
    b, fb = oracle.fmm2d(pos, q, 4, 12, level_p=[0, 0, 12, 12, 12])
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(fa, fb)


def test_level_order_single_far_level():
    """With L = 2 only level 2 has an interaction list: its order is the order."""
    pos, q = workloads.uniform(2000, 2, seed=302)
    for pk in (3, 9, 17):
        a, fa = oracle.fmm2d(pos, q, 2, pk)
        b, fb = oracle.fmm2d(pos, q, 2, 25, level_p=[0, 0, pk])
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(fa, fb)


def test_level_orders_act_on_their_own_level_only():
    """No shifts couple the levels, so changing level 3's order changes the
    result by the same amount whatever level 2's order is (and vice versa)."""
    pos, q = workloads.uniform(6000, 2, seed=303)
    L = 4

    def run(p2, p3, p4):
        return oracle.fmm2d(pos, q, L, 20, level_p=[0, 0, p2, p3, p4])

    aa, faa = run(6, 6, 14)
    ab, fab = run(6, 15, 14)
    ba, fba = run(15, 6, 14)
    bb, fbb = run(15, 15, 14)
    d1, d2 = ab - aa, bb - ba
    assert np.linalg.norm(d1) > 1e-6 * np.linalg.norm(aa)  # the order matters
    assert np.linalg.norm(d1 - d2) < 1e-12 * np.linalg.norm(aa)
    assert np.linalg.norm((fab - faa) - (fbb - fba)) < 1e-12 * np.linalg.norm(faa)
    # and the truncation error of each level falls with its own order
    ref, _ = run(30, 30, 30)
    e_lo, e_hi = rel(run(6, 30, 30)[0], ref), rel(run(12, 30, 30)[0], ref)
    assert e_hi < e_lo * 0.547 ** 5


def test_level_order_reaches_the_right_level():
    """Charges inside one level-2 box: the interaction lists of levels 2 and 3
    hold no charge (its level-3 children are mutually adjacent), so only level
    4's order may change the result."""
    rng = np.random.default_rng(305)
    pos = rng.uniform(0.0, 1.25, size=(3000, 2))
    q = rng.uniform(-1, 1, size=3000)
    base, fb = oracle.fmm2d(pos, q, 4, 20, level_p=[0, 0, 10, 10, 10])
    for p2, p3 in ((3, 10), (10, 3), (25, 2)):
        a, fa = oracle.fmm2d(pos, q, 4, 20, level_p=[0, 0, p2, p3, 10])
        np.testing.assert_array_equal(a, base)
        np.testing.assert_array_equal(fa, fb)
    c, _ = oracle.fmm2d(pos, q, 4, 20, level_p=[0, 0, 10, 10, 4])
    assert rel(c, base) > 1e-7


def test_level_order_rejects_bad_input():
    pos, q = workloads.uniform(100, 2, seed=304)
    with pytest.raises(ValueError):
        oracle.fmm2d(pos, q, 3, 8, level_p=[0, 0, 8])
    with pytest.raises(ValueError):
        oracle.fmm2d(pos, q, 3, 8, level_p=[0, 0, 8, 31])
    with pytest.raises(ValueError):
        oracle.fmm2d(pos, q, 3, 8, classical=True, level_p=[0, 0, 8, 8])


# --- MLP ----------------------------------------------------------------------

def random_weights(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=oracle.MLP_NPARAM)


def test_mlp_layout_represents_a_linear_map_exactly():
    """Weights that route x through ReLU(x) - ReLU(-x) make the network the
    affine map A x + c: pins the parameter layout, the row/column convention of
    every layer and the place of the ReLUs (64 x 3 and 21 x 64 are not square)."""
    rng = np.random.default_rng(310)
    A = rng.normal(size=(21, 3))
    c = rng.normal(size=21)
    w = np.zeros(oracle.MLP_NPARAM)
    W1 = np.zeros((64, 3))
    for i in range(3):
        W1[i, i] = 1.0
        W1[3 + i, i] = -1.0
    W2 = np.zeros((64, 64))
    W2[:6, :6] = np.eye(6)
    W3 = np.zeros((21, 64))
    W3[:, :3] = A
    W3[:, 3:6] = -A
    o = 0
    for arr in (W1, np.zeros(64), W2, np.zeros(64), W3, c):
        w[o:o + arr.size] = arr.ravel()
        o += arr.size
    assert o == oracle.MLP_NPARAM == 5781
    x = rng.normal(size=(50, 3))
    np.testing.assert_allclose(oracle.mlp_forward(w, x), x @ A.T + c, rtol=0, atol=1e-13)


def test_mlp_constant_network_loss():
    """All weights zero but the output bias b: y = b for every sample, so the
    loss is the mean squared deviation of the targets from b."""
    rng = np.random.default_rng(311)
    w = np.zeros(oracle.MLP_NPARAM)
    b = rng.normal(size=21)
    w[-21:] = b
    x = rng.normal(size=(40, 3))
    t = rng.normal(size=(40, 21))
    loss, g = oracle.mlp_loss_grad(w, x, t)
    assert loss == pytest.approx(np.mean((b - t) ** 2), rel=1e-14)
    # d loss / d b = 2 mean over samples of (b - t) / 21; every hidden weight
    # sits behind a zero activation and gets no gradient except W3 (h2 = 0 too)
    np.testing.assert_allclose(g[-21:], 2.0 * (b - t).mean(axis=0) / 21, rtol=1e-13)
    assert np.all(g[:-21] == 0)


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(312)
    w = random_weights(313)
    x = rng.normal(size=(25, 3))
    t = rng.normal(size=(25, 21))
    _, g = oracle.mlp_loss_grad(w, x, t)
    idx = np.concatenate([rng.choice(oracle.MLP_NPARAM, 300, replace=False),
                          np.arange(oracle.MLP_NPARAM - 21, oracle.MLP_NPARAM),
                          np.arange(0, 192, 7)])
    h = 1e-6
    fd = np.empty(len(idx))
    for n, i in enumerate(idx):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd[n] = (oracle.mlp_loss_grad(wp, x, t)[0] - oracle.mlp_loss_grad(wm, x, t)[0]) / (2 * h)
    assert rel(g[idx], fd) < 1e-7


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step, so each step moves w by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(314)
    n = 257
    w0 = rng.normal(size=n)
    g = rng.normal(size=n)
    w, m1, m2 = w0.copy(), np.zeros(n), np.zeros(n)
    lr, eps = 3e-3, 1e-8
    for step in range(1, 8):
        oracle.mlp_adam(w, g, m1, m2, step, lr=lr, eps=eps)
    np.testing.assert_allclose(w, w0 - 7 * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-14)


def test_adam_minimises_a_quadratic():
    rng = np.random.default_rng(315)
    n = 64
    c = rng.normal(size=n)
    w, m1, m2 = np.zeros(n), np.zeros(n), np.zeros(n)
    for step in range(1, 3001):
        oracle.mlp_adam(w, 2 * (w - c), m1, m2, step, lr=1e-2)
    assert np.max(np.abs(w - c)) < 1e-3
