"""Host-side logic of bench.py (CPU): the work counts its roofline objects divide
by, checked against brute-force counts from the definitions (Section 2.1: the
near field is the 3^D leaves around a particle's leaf, the interaction list of
a box the children of its parent's neighbours that are not its own
neighbours), the adaptive counts' reduction to the uniform ones, the counter
summaries' source check, and the one-GPU refusal."""
import hashlib
import itertools
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import workloads  # noqa: E402


def brute_il_pairs(dim, L):
    tot = 0
    for k in range(2, L + 1):
        n = 1 << k
        boxes = list(itertools.product(range(n), repeat=dim))
        for t in boxes:
            for s in boxes:
                adj = all(abs(a - b) <= 1 for a, b in zip(t, s))
                padj = all(abs((a >> 1) - (b >> 1)) <= 1 for a, b in zip(t, s))
                tot += int(padj and not adj)
    return tot


@pytest.mark.parametrize("dim,L", [(2, 2), (2, 3), (2, 4), (2, 5), (3, 2), (3, 3)])
def test_il_pairs_match_the_definition(dim, L):
    assert bench.il_pairs(dim, L) == brute_il_pairs(dim, L)


@pytest.mark.parametrize("dim,L", [(2, 3), (2, 4), (3, 2)])
def test_p2p_pairs_match_brute_force(dim, L):
    pos, _ = workloads.gaussian_mixture(700, dim, seed=31 + L)
    nl = 1 << L
    c = np.minimum(np.floor(pos * (nl / 5.0)).astype(np.int64), nl - 1)
    near = np.all(np.abs(c[:, None, :] - c[None, :, :]) <= 1, axis=2)
    want = int(near.sum()) - len(pos)  # ordered pairs, the self pair left out
    assert bench.p2p_pairs(pos, L) == want


def brute_depths(pos, L, near):
    """A particle's depth: the first level k >= 2 whose 3 x 3 boxes around its
    level-k box hold at most `near` particles, L if none."""
    n = len(pos)
    dep = np.full(n, L)
    for i in range(n):
        for k in range(2, L):
            nk = 1 << k
            c = np.minimum(np.floor(pos * (nk / 5.0)).astype(np.int64), nk - 1)
            around = int(np.all(np.abs(c - c[i]) <= 1, axis=1).sum())
            if around <= near:
                dep[i] = k
                break
    return dep


def test_adaptive_depths_and_pairs_match_brute_force():
    pos, _ = workloads.gaussian_mixture(600, 2, seed=41)
    L, near = 6, 40
    dep, _, _, _, _ = bench.adaptive_tree(pos, L, near)
    want = brute_depths(pos, L, near)
    np.testing.assert_array_equal(dep, want)
    # near-field pairs: each particle against the particles of the 3 x 3 boxes
    # around its box at its own depth
    tot = 0
    for i in range(len(pos)):
        k = dep[i]
        nk = 1 << k
        c = np.minimum(np.floor(pos * (nk / 5.0)).astype(np.int64), nk - 1)
        tot += int(np.all(np.abs(c - c[i]) <= 1, axis=1).sum()) - 1
    assert bench.p2p_pairs_adaptive(pos, L, near) == tot


def test_adaptive_counts_reduce_to_uniform_at_zero():
    pos, _ = workloads.uniform(20000, 2, seed=42)  # every level-5 box holds particles
    L = 5
    assert bench.p2p_pairs_adaptive(pos, L, 0) == bench.p2p_pairs(pos, L)
    assert bench.il_pairs_adaptive(pos, L, 0) == bench.il_pairs(2, L)


def test_traffic_key_names():
    assert bench.traffic_key("w", 0, 0, 10, False, "paper") == "w"
    assert bench.traffic_key("w", 12, 600, 12, False, "paper") == "w-adaptive-L12-T600"
    assert bench.traffic_key("w", 8, 0, 8, True, "chebyshev", 6) == "w-L8-rootframe-chebyshev-order6"
    assert bench.traffic_key("w", 0, 0, 3, False, "chebyshev", 5) == "w-chebyshev-order5"


def test_measured_traffic_needs_the_recorded_sources(tmp_path, monkeypatch):
    src = tmp_path / "kern.hip"
    src.write_text("kernel source\n")
    (tmp_path / "profiles").mkdir()
    entry = {"kernel": "k", "hbm_bytes_per_launch": 1234, "sources": ["kern.hip"],
             "sha256": hashlib.sha256(b"kernel source\n").hexdigest()}
    (tmp_path / "profiles" / "traffic_w_fp32.json").write_text(
        json.dumps({"kernels": {"p2p": entry}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", "fp32", "p2p") == 1234
    assert bench.measured_traffic("w", "fp32", "m2l") is None
    assert bench.measured_traffic("w", "fp64", "p2p") is None
    src.write_text("kernel source, changed\n")
    assert bench.measured_traffic("w", "fp32", "p2p") is None


def test_committed_traffic_summaries_name_existing_sources():
    d = os.path.join(ROOT, "profiles")
    for f in sorted(os.listdir(d)):
        if not f.startswith("traffic_"):
            continue
        table = json.load(open(os.path.join(d, f)))
        for kernel, e in table["kernels"].items():
            assert e["hbm_bytes_per_launch"] > 0, (f, kernel)
            for s in e["sources"]:
                assert os.path.exists(os.path.join(ROOT, s)), (f, s)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
