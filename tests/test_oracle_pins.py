"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test pins the oracle to something other than itself: hand-worked closed
forms (tests/golden), finite differences, conservation laws, brute-force
enumeration of the tree definitions, library special functions (scipy), the
convergence of the truncated expansions to the exact pair sum, the textbook
method with shifts (Section 2.1) that the shift-free passes (Section 2.2)
must reproduce, and invariances of the whole computation.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


# --------------------------------------------------------------------------
# Direct sum (the exact quantity)
# --------------------------------------------------------------------------
def test_direct_closed_forms():
    cases = json.load(open(os.path.join(GOLDEN, "closed_forms.json")))["cases"]
    env = {"log": math.log, "sqrt": math.sqrt}
    for c in cases:
        pos, q = np.array(c["pos"], float), np.array(c["q"], float)
        pot, fld = oracle.direct(pos, q)
        want = [eval(e, env) for e in c["pot"]]
        np.testing.assert_allclose(pot, want, rtol=1e-14, atol=1e-15, err_msg=c["name"])
        np.testing.assert_allclose(fld, np.array(c["field"]), rtol=1e-13, atol=1e-15,
                                   err_msg=c["name"])


@pytest.mark.parametrize("dim", [2, 3])
def test_direct_field_is_minus_gradient(dim):
    pos, q = workloads.uniform(60, dim, seed=11)
    _, fld = oracle.direct(pos, q)
    h = 1e-6
    for i in [0, 7, 33]:
        for d in range(dim):
            pp, pm = pos.copy(), pos.copy()
            pp[i, d] += h
            pm[i, d] -= h
            fd = -(oracle.direct(pp, q, field=False)[i] - oracle.direct(pm, q, field=False)[i]) / (2 * h)
            assert abs(fd - fld[i, d]) <= 1e-6 * max(1.0, abs(fld[i, d]))


@pytest.mark.parametrize("dim", [2, 3])
def test_direct_newton_third_law(dim):
    pos, q = workloads.uniform(500, dim, seed=12)
    _, fld = oracle.direct(pos, q)
    total = (q[:, None] * fld).sum(0)
    scale = np.abs(q[:, None] * fld).sum()
    assert np.all(np.abs(total) <= 1e-12 * scale)


def test_direct_targets_subset_matches_full():
    pos, q = workloads.uniform(300, 2, seed=13)
    pot, fld = oracle.direct(pos, q)
    tg = np.array([3, 100, 299])
    p2, f2 = oracle.direct(pos, q, targets=tg)
    np.testing.assert_array_equal(p2, pot[tg])
    np.testing.assert_array_equal(f2, fld[tg])


# --------------------------------------------------------------------------
# Tree and interaction lists (Section 2.1 items 1-5)
# --------------------------------------------------------------------------
def test_leaf_coordinate_expression():
    # 2^L / S evaluated in FP64; the upper face is clamped into the last leaf.
    assert oracle.leaf_coord(0.0, 0.0, 5.0, 3) == 0
    assert oracle.leaf_coord(5.0, 0.0, 5.0, 3) == 7
    assert oracle.leaf_coord(0.625, 0.0, 5.0, 3) == 1
    assert oracle.leaf_coord(0.62499999, 0.0, 5.0, 3) == 0
    assert oracle.leaf_coord(2.6, 0.1, 5.0, 1) == 1


def _adjacent(a, b):
    return all(abs(int(x) - int(y)) <= 1 for x, y in zip(a, b))


def test_ilist_counts_and_offsets():
    g = json.load(open(os.path.join(GOLDEN, "interaction_list_offsets.json")))
    k = 4
    union2 = set()
    for tx in range(16):
        for ty in range(16):
            il = oracle.ilist2d(k, tx, ty)
            offs = {(int(b[0]) - tx, int(b[1]) - ty) for b in il}
            union2 |= offs
            if 2 <= tx <= 13 and 2 <= ty <= 13:
                assert len(il) == g["2d_interior_count"]
                lo, hi = g["2d_even_even_offset_range"] if tx % 2 == 0 else g["2d_odd_odd_offset_range"]
                assert all(lo <= o[0] <= hi for o in offs)
    assert len(union2) == g["2d_union_count"]
    union3 = set()
    n = 8
    for tx in range(n):
        for ty in range(n):
            for tz in range(n):
                il = oracle.ilist3d(3, tx, ty, tz)
                union3 |= {(int(b[0]) - tx, int(b[1]) - ty, int(b[2]) - tz) for b in il}
                if all(2 <= c <= 5 for c in (tx, ty, tz)):
                    assert len(il) == g["3d_interior_count"]
    assert len(union3) == g["3d_union_count"]


def test_ilist_matches_definition_by_brute_force():
    # b in IL(t) <=> parents adjacent (or equal) and b, t not adjacent.
    for k in (2, 3, 4):
        n = 1 << k
        for tx in range(n):
            for ty in range(n):
                want = {(bx, by) for bx in range(n) for by in range(n)
                        if _adjacent((bx >> 1, by >> 1), (tx >> 1, ty >> 1))
                        and not _adjacent((bx, by), (tx, ty))}
                got = {tuple(int(v) for v in b) for b in oracle.ilist2d(k, tx, ty)}
                assert got == want


@pytest.mark.parametrize("dim,L", [(2, 2), (2, 3), (2, 4), (2, 5), (3, 2), (3, 3)])
def test_partition_identity(dim, L):
    """Every ordered pair of leaves is near at level L or in exactly one IL."""
    n = 1 << L
    leaves = [c for c in np.ndindex(*([n] * dim))]
    for a in leaves:
        cover = {}
        for b in leaves:
            if _adjacent(a, b):
                cover[b] = cover.get(b, 0) + 1
        for k in range(2, L + 1):
            anc = tuple(c >> (L - k) for c in a)
            il = oracle.ilist2d(k, *anc) if dim == 2 else oracle.ilist3d(k, *anc)
            span = 1 << (L - k)
            for box in il:
                for off in np.ndindex(*([span] * dim)):
                    leaf = tuple(int(box[d]) * span + off[d] for d in range(dim))
                    cover[leaf] = cover.get(leaf, 0) + 1
        assert len(cover) == len(leaves) and all(v == 1 for v in cover.values()), a


def test_ilist_pair_totals_level4():
    tot = []
    for k in (2, 3, 4):
        n = 1 << k
        tot.append(sum(len(oracle.ilist2d(k, x, y)) for x in range(n) for y in range(n)))
    # brute force from the definition
    want = []
    for k in (2, 3, 4):
        n = 1 << k
        c = 0
        for t in np.ndindex(n, n):
            for b in np.ndindex(n, n):
                if _adjacent((b[0] >> 1, b[1] >> 1), (t[0] >> 1, t[1] >> 1)) and not _adjacent(b, t):
                    c += 1
        want.append(c)
    assert tot == want == [156, 1116, 5628]


# --------------------------------------------------------------------------
# 2D expansions
# --------------------------------------------------------------------------
def test_single_box_multipole_truncation_bound():
    """Multipole series of one box at far points is within Greengard's bound
    sum|q| alpha^(p+1) / ((p+1)(1 - alpha)), alpha = r / R."""
    rng = np.random.default_rng(5)
    s = 0.5
    c = np.array([1.25, 1.25])
    src = c + rng.uniform(-s / 2, s / 2, size=(40, 2))
    q = rng.uniform(-1, 1, 40)
    r = np.max(np.linalg.norm(src - c, axis=1))
    for p in (4, 8, 12, 20):
        a = oracle.p2m2d_point(src, q, c, s, p)
        for ang in np.linspace(0, 2 * np.pi, 7):
            R = 3.0 * s
            x, y = c + R * np.array([np.cos(ang), np.sin(ang)])
            exact = np.sum(q * np.log(np.hypot(x - src[:, 0], y - src[:, 1])))
            approx = oracle.m2p2d_point(a, c, s, x, y)
            alpha = r / R
            bound = np.abs(q).sum() * alpha ** (p + 1) / ((p + 1) * (1 - alpha))
            assert abs(approx - exact) <= bound * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("p", [4, 8, 12, 16])
def test_fmm2d_error_decays_geometrically(p):
    pos, q = workloads.uniform(2048, 2, seed=21)
    pd = oracle.direct(pos, q, field=False)
    e1 = rel(oracle.fmm2d(pos, q, 4, p, field=False)[0], pd)
    e2 = rel(oracle.fmm2d(pos, q, 4, p + 4, field=False)[0], pd)
    # per-order ratio alpha = sqrt(2)/(4 - sqrt(2)) of the M2L error bound
    alpha = math.sqrt(2) / (4 - math.sqrt(2))
    assert e2 <= e1 * 2 * alpha ** 4


def test_fmm2d_high_order_equals_direct():
    """At p = 30 the truncation error is far below 1e-12: any wrong sign, index
    or dropped term in P2M, M2L, L2P or the lists would show up here."""
    pos, q = workloads.uniform(4096, 2, seed=1)
    pd, fd = oracle.direct(pos, q)
    pf, ff = oracle.fmm2d(pos, q, 4, 30)
    assert rel(pf, pd) < 1e-12
    assert rel(ff, fd) < 1e-11


def test_fmm2d_field_is_minus_gradient():
    pos, q = workloads.uniform(600, 2, seed=22)
    _, fld = oracle.fmm2d(pos, q, 3, 10)
    h = 1e-6
    for i in [1, 100, 400]:
        for d in range(2):
            pp, pm = pos.copy(), pos.copy()
            pp[i, d] += h
            pm[i, d] -= h
            fp = oracle.fmm2d(pp, q, 3, 10, field=False)[0][i]
            fm = oracle.fmm2d(pm, q, 3, 10, field=False)[0][i]
            assert abs(-(fp - fm) / (2 * h) - fld[i, d]) <= 1e-6 * max(1.0, abs(fld[i, d]))


@pytest.mark.parametrize("L,p", [(3, 8), (4, 12), (5, 16)])
def test_fmm2d_shift_free_equals_classical(L, p):
    """Truncated M2M and L2L are exact for Laurent / Taylor coefficients, so the
    textbook method with shifts (Section 2.1) gives the shift-free result
    (Section 2.2) up to rounding."""
    pos, q = workloads.uniform(3000, 2, seed=23)
    a, fa = oracle.fmm2d(pos, q, L, p)
    b, fb = oracle.fmm2d(pos, q, L, p, classical=True)
    assert rel(a, b) < 1e-13
    assert rel(fa, fb) < 1e-13


def test_fmm2d_linearity_and_sign():
    pos, q = workloads.uniform(1500, 2, seed=24)
    q2 = workloads.uniform(1500, 2, seed=25)[1]
    a = oracle.fmm2d(pos, q, 4, 12)[0]
    b = oracle.fmm2d(pos, q2, 4, 12)[0]
    c = oracle.fmm2d(pos, 0.5 * q - 2.0 * q2, 4, 12)[0]
    assert rel(c, 0.5 * a - 2.0 * b) < 1e-13
    neg, nf = oracle.fmm2d(pos, -q, 4, 12)
    pa, pf = oracle.fmm2d(pos, q, 4, 12)
    np.testing.assert_array_equal(neg, -pa)
    np.testing.assert_array_equal(nf, -pf)


def test_fmm2d_translation_and_scaling():
    pos, q = workloads.uniform(2000, 2, seed=26)
    pot, fld = oracle.fmm2d(pos, q, 4, 12)
    shift = np.array([0.75, -1.25])
    p2, f2 = oracle.fmm2d(pos + shift, q, 4, 12, origin=tuple(shift))
    assert rel(p2, pot) < 1e-12 and rel(f2, fld) < 1e-12
    lam = 4.0  # a power of two keeps the tree identical bit for bit
    p3, f3 = oracle.fmm2d(pos * lam, q, 4, 12, side=5.0 * lam)
    assert rel(p3, pot + math.log(lam) * (q.sum() - q)) < 1e-12
    assert rel(f3, fld / lam) < 1e-13


def test_fmm2d_reflection_symmetry():
    pos, q = workloads.uniform(2000, 2, seed=27)
    pot, fld = oracle.fmm2d(pos, q, 4, 12)
    refl = pos.copy()
    refl[:, 0] = 5.0 - refl[:, 0]
    p2, f2 = oracle.fmm2d(refl, q, 4, 12)
    assert rel(p2, pot) < 1e-12
    assert rel(f2 * np.array([-1, 1]), fld) < 1e-12
    swap = pos[:, ::-1].copy()
    p3, f3 = oracle.fmm2d(swap, q, 4, 12)
    assert rel(p3, pot) < 1e-12 and rel(f3[:, ::-1], fld) < 1e-12


def test_fmm2d_degenerate_cases():
    pos, q = workloads.uniform(700, 2, seed=28)
    pd, fd = oracle.direct(pos, q)
    # L = 1: every leaf is adjacent to every other -> near field only = direct
    p1, f1 = oracle.fmm2d(pos, q, 1, 12)
    assert rel(p1, pd) < 1e-13 and rel(f1, fd) < 1e-13
    # zero charges
    p0, f0 = oracle.fmm2d(pos, np.zeros_like(q), 4, 12)
    assert not np.any(p0) and not np.any(f0)
    # one particle
    p, f = oracle.fmm2d(pos[:1], q[:1], 4, 12)
    assert p[0] == 0 and not np.any(f)
    # all charges in one leaf -> near field only = direct
    tight = 0.1 + 0.01 * workloads.uniform(300, 2, seed=29)[0]
    qq = q[:300]
    pt, ft = oracle.fmm2d(tight, qq, 5, 8)
    pdt, fdt = oracle.direct(tight, qq)
    assert rel(pt, pdt) < 1e-13 and rel(ft, fdt) < 1e-13
    # out-of-domain and NaN positions are rejected
    bad = pos.copy()
    bad[5, 1] = 5.0000001
    with pytest.raises(ValueError):
        oracle.fmm2d(bad, q, 4, 12)
    bad[5, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.fmm2d(bad, q, 4, 12)


def test_fmm2d_targets_subset_matches_full():
    pos, q = workloads.uniform(3000, 2, seed=30)
    pot, fld = oracle.fmm2d(pos, q, 4, 12)
    tg = workloads.sample_targets(3000, 50, seed=1)
    p2, f2 = oracle.fmm2d(pos, q, 4, 12, targets=tg)
    assert rel(p2, pot[tg]) < 1e-15 and rel(f2, fld[tg]) < 1e-15


# --------------------------------------------------------------------------
# 3D solid harmonics
# --------------------------------------------------------------------------
def _scipy_harmonics(p, r):
    from scipy.special import lpmv
    x, y, z = r
    rr = math.sqrt(x * x + y * y + z * z)
    th, ph = math.acos(z / rr), math.atan2(y, x)
    R = np.zeros((p + 1) ** 2, complex)
    I = np.zeros((p + 1) ** 2, complex)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            # lpmv includes the Condon-Shortley phase and extends to m < 0
            P = lpmv(m, n, math.cos(th))
            R[n * n + n + m] = rr ** n * P * np.exp(1j * m * ph) / math.factorial(n + m)
            I[n * n + n + m] = math.factorial(n - m) * P * np.exp(1j * m * ph) / rr ** (n + 1)
    return R, I


def test_solid_harmonics_match_library_legendre():
    for r in ([0.3, -0.2, 0.5], [1.0, 2.0, -0.5], [-0.1, 0.05, -0.7]):
        Rw, Iw = _scipy_harmonics(10, r)
        np.testing.assert_allclose(oracle.sh_regular(10, r), Rw, rtol=1e-11, atol=1e-16)
        np.testing.assert_allclose(oracle.sh_irregular(10, r), Iw, rtol=1e-11, atol=1e-16)


def test_addition_theorem():
    """1/|x - y| = sum_{n,m} conj(R_n^m(y)) I_n^m(x) at |y|/|x| = 0.3, p = 30."""
    rng = np.random.default_rng(31)
    for _ in range(5):
        x = rng.normal(size=3)
        x *= 2.0 / np.linalg.norm(x)
        y = rng.normal(size=3)
        y *= 0.6 / np.linalg.norm(y)
        s = np.sum(np.conj(oracle.sh_regular(30, y)) * oracle.sh_irregular(30, x))
        assert abs(s.imag) < 1e-15
        assert abs(s.real - 1 / np.linalg.norm(x - y)) < 1e-14


def test_fmm3d_error_decays_and_high_order_matches_direct():
    pos, q = workloads.uniform(1500, 3, seed=32)
    pd, fd = oracle.direct(pos, q)
    errs = [rel(oracle.fmm3d(pos, q, 2, p, field=False)[0], pd) for p in (2, 6, 10, 14, 18)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-8
    pf, ff = oracle.fmm3d(pos, q, 2, 18)
    assert rel(ff, fd) < 1e-7


@pytest.mark.parametrize("L,p", [(3, 4), (3, 8)])
def test_fmm3d_shift_free_equals_classical(L, p):
    pos, q = workloads.uniform(1500, 3, seed=33)
    a, fa = oracle.fmm3d(pos, q, L, p)
    b, fb = oracle.fmm3d(pos, q, L, p, classical=True)
    assert rel(a, b) < 1e-13
    assert rel(fa, fb) < 1e-13


def test_fmm3d_field_is_minus_gradient():
    pos, q = workloads.uniform(400, 3, seed=34)
    _, fld = oracle.fmm3d(pos, q, 3, 6)
    h = 1e-6
    for i in [2, 200]:
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, d] += h
            pm[i, d] -= h
            fp = oracle.fmm3d(pp, q, 3, 6, field=False)[0][i]
            fm = oracle.fmm3d(pm, q, 3, 6, field=False)[0][i]
            assert abs(-(fp - fm) / (2 * h) - fld[i, d]) <= 1e-5 * max(1.0, abs(fld[i, d]))


def test_fmm3d_invariances_and_degenerate():
    pos, q = workloads.uniform(800, 3, seed=35)
    pot, fld = oracle.fmm3d(pos, q, 3, 6)
    lam = 2.0
    p2, f2 = oracle.fmm3d(pos * lam, q, 3, 6, side=5.0 * lam)
    assert rel(p2, pot / lam) < 1e-13 and rel(f2, fld / lam ** 2) < 1e-13
    refl = pos.copy()
    refl[:, 2] = 5.0 - refl[:, 2]
    p3, f3 = oracle.fmm3d(refl, q, 3, 6)
    assert rel(p3, pot) < 1e-12 and rel(f3 * np.array([1, 1, -1]), fld) < 1e-12
    neg = oracle.fmm3d(pos, -q, 3, 6)[0]
    np.testing.assert_array_equal(neg, -pot)
    pd, fd = oracle.direct(pos, q)
    p1, f1 = oracle.fmm3d(pos, q, 1, 6)
    assert rel(p1, pd) < 1e-13 and rel(f1, fd) < 1e-13
