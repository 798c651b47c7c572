"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs a
small case of every entry point without a report (out-of-bounds accesses,
use after free, signed overflow, misaligned or invalid shifts and the like
would abort the child process)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
import oracle, workloads
pos, q = workloads.uniform(700, 2, seed=1)
oracle.direct(pos, q)
oracle.fmm2d(pos, q, 4, 8)
oracle.fmm2d(pos, q, 4, 8, classical=True)
oracle.fmm2d(pos, q, 3, 6, dump_level=3, split=True, level_p=[0, 0, 4, 6])
oracle.fmm2d(pos, q, 4, 8, targets=np.array([0, 5, 699]))
oracle.fmm2d_adaptive(pos, q, 5, 8, 12)
oracle.fmm2d_lagrange(pos, q, 4, dump_level=3)
oracle.fmm2d_lagrange(pos, q, 3, nodes=oracle.chebyshev_nodes(6), targets=np.array([1, 698]))
p3, q3 = workloads.uniform(600, 3, seed=2)
oracle.fmm3d(p3, q3, 3, 4)
oracle.fmm3d(p3, q3, 3, 4, classical=True)
oracle.fmm3d_lagrange(p3, q3, 3, dump_level=2)
oracle.fmm3d_lagrange_nodes(p3, q3, 3, oracle.chebyshev_nodes(5))
oracle.fmm3d_lagrange_root(p3, q3, 3)
oracle.lagrange_transfer(2, (1, 2, 3))
oracle.sh_regular(8, np.array([0.3, -0.2, 0.4]))
oracle.ilist2d(3, 2, 5)
oracle.ilist3d(3, 2, 5, 1)
w = np.random.default_rng(0).normal(size=5781) * 0.1
x = np.random.default_rng(1).normal(size=(9, 3))
t = np.random.default_rng(2).normal(size=(9, 21))
oracle.mlp_forward(w, x)
l, g = oracle.mlp_loss_grad(w, x, t)
oracle.mlp_adam(w, g, np.zeros_like(w), np.zeros_like(w), 1)
print("SANITIZED-OK")
"""


@pytest.mark.slow
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from oracle import build
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no libasan in this toolchain")
    lib = build.build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", CASES % ROOT], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0 and "SANITIZED-OK" in r.stdout, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
