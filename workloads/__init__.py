"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws random numbers only; it holds none of the method's
arithmetic.  Every array is FP64 from ``numpy.random.default_rng(seed)`` (PCG64),
drawn in the order: positions, then charges.

Workloads follow the problem statement of the paper (N charged particles in a
square or cube of side 5, Section 2.1 item 1; random charges, Section 3):
  * uniform positions in [0, 5)^D, charges uniform in [-1, 1];
  * an 8-component isotropic Gaussian mixture (sigma 0.1, centres uniform in
    the box, equal weights; samples outside [0, 5)^D are redrawn);
  * the paper's own Section 3 workload: charges +1 or -1 at random.
"""
import numpy as np

SIDE = 5.0


def uniform(n, dim=2, seed=0, side=SIDE):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, side, size=(n, dim))
    q = rng.uniform(-1.0, 1.0, size=n)
    return pos, q


def gaussian_mixture(n, dim=2, seed=0, ncomp=8, sigma=0.1, side=SIDE):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, side, size=(ncomp, dim))
    pos = np.empty((n, dim))
    filled = 0
    while filled < n:
        need = n - filled
        comp = rng.integers(0, ncomp, size=need)
        cand = centres[comp] + sigma * rng.standard_normal(size=(need, dim))
        ok = np.all((cand >= 0.0) & (cand < side), axis=1)
        cand = cand[ok]
        pos[filled:filled + len(cand)] = cand
        filled += len(cand)
    q = rng.uniform(-1.0, 1.0, size=n)
    return pos, q


def plus_minus_one(n, dim=3, seed=0, side=SIDE):
    """Random +1/-1 charges scattered uniformly (the paper's Section 3 workload)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, side, size=(n, dim))
    q = rng.choice(np.array([-1.0, 1.0]), size=n)
    return pos, q


def sample_targets(n, count=4096, seed=1000):
    """Seeded sample of particle indices at which a sampled check is made."""
    rng = np.random.default_rng(seed)
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def batched_systems(nsys=512, dim=2, seed=5, nmin=1024, nmax=65536):
    """Independent systems with N log-uniform in [nmin, nmax]; each system is
    uniform or Gaussian-mixture with probability 1/2.  Returns a list of
    (pos, q) pairs."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=nsys))).astype(np.int64)
    kinds = rng.integers(0, 2, size=nsys)
    seeds = rng.integers(0, 2**31 - 1, size=nsys)
    out = []
    for n, kind, s in zip(sizes, kinds, seeds):
        if kind == 0:
            out.append(uniform(int(n), dim, int(s)))
        else:
            out.append(gaussian_mixture(int(n), dim, int(s)))
    return out


# Named workloads (sizes of the paper-shaped test and benchmark cases).
WORKLOADS = {
    "2d-uniform-4k-L4-p12": dict(dim=2, n=4096, levels=4, p=12, kind="uniform", seed=1),
    "2d-uniform-1M-L8-p16": dict(dim=2, n=1 << 20, levels=8, p=16, kind="uniform", seed=2),
    "2d-mixture-16M-L10-p20": dict(dim=2, n=1 << 24, levels=10, p=20, kind="mixture", seed=3),
    "3d-uniform-4M-L7-p8": dict(dim=3, n=1 << 22, levels=7, p=8, kind="uniform", seed=4),
    # the paper's Section 3 runs: +1/-1 charges in the cube, 4 x 4 x 4 point
    # charges per box (p holds the points per axis)
    "3d-pm1-200k-L3-n4": dict(dim=3, n=200000, levels=3, p=4, kind="pm1", seed=6, basis="points"),
    "3d-pm1-80k-L3-n4": dict(dim=3, n=80000, levels=3, p=4, kind="pm1", seed=7, basis="points"),
    "3d-pm1-80k-L2-n4": dict(dim=3, n=80000, levels=2, p=4, kind="pm1", seed=8, basis="points"),
    # the same point charges in the square box (Appendix STEP1, 4 x 4 per box), log kernel
    "2d-pm1-1M-L8-n4": dict(dim=2, n=1 << 20, levels=8, p=4, kind="pm1", seed=11,
                            basis="points"),
}


def make(name):
    w = WORKLOADS[name]
    if w["kind"] == "uniform":
        pos, q = uniform(w["n"], w["dim"], w["seed"])
    elif w["kind"] == "pm1":
        pos, q = plus_minus_one(w["n"], w["dim"], w["seed"])
    else:
        pos, q = gaussian_mixture(w["n"], w["dim"], w["seed"])
    return pos, q, w
