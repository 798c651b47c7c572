"""Writes lagrange_nodes_accuracy.json: the accuracy of the point-charge method
against the direct sum for several node sets and numbers of points per axis
(d = n^3), on 20000 random +1/-1 charges in the cube of side 5 at level 3 (the
paper's Section 3 workload shape).  Calls only the oracle.

    python tests/golden/make_lagrange_nodes_accuracy.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

N, L, SEED = 20000, 3, 13


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def main():
    pos, q = workloads.plus_minus_one(N, 3, seed=SEED)
    d, fd = oracle.direct(pos, q)
    tg = workloads.sample_targets(N, 2000, 1013)
    rows = []
    sets = [("paper", 4, oracle.PAPER_NODES)]
    for n in (3, 4, 5, 6):
        sets.append(("chebyshev", n, oracle.chebyshev_nodes(n)))
        sets.append(("equispaced", n, tuple(np.linspace(-2.0, 2.0, n))))
    for name, n, nodes in sets:
        pot, fld = oracle.fmm3d_lagrange_nodes(pos, q, L, nodes)
        row = {"nodes": name, "n": n, "d": n ** 3, "offsets_s_over_5": list(nodes),
               "rel_l2_pot": rel(pot, d), "rel_l2_field": rel(fld, fd),
               "rel_l2_pot_sampled": rel(pot[tg], d[tg])}
        rows.append(row)
        print(row, flush=True)
    out = {"source": "oracle (oracle.fmm3d_lagrange_nodes against oracle.direct); written by "
                     "tests/golden/make_lagrange_nodes_accuracy.py",
           "workload": "random +1/-1 charges uniform in the cube of side 5",
           "n": N, "levels": L, "seed": SEED, "sampled_targets": {"count": 2000, "seed": 1013},
           "rows": rows}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                           "lagrange_nodes_accuracy.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
