"""Writes plummer16m_grid.json: the oracle's potential and field on sampled
leaves of the 2^24-point Plummer workload (scale radius 0.05, 6 levels) for
theta in {0.4, 0.5, 0.6} and p in {8, 12, 16}, in binary64.

The oracle runs the whole method (tree, lists, upward pass, M2L into the
sampled leaves' ancestors, L2L, L2P and P2P) and fills only the points of
the sampled leaves.  Calls only the oracle and the seeded input generator.

    python tests/golden/make_plummer16m_grid.py     # about 15 minutes on 3 cores
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

THETAS = (0.4, 0.5, 0.6)
ORDERS = (8, 12, 16)
LEAVES = (0, 131071, 262143)  # first, middle and last leaf of the 8^6
PER_LEAF = 16                 # first points of each sampled leaf (tree order)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plummer16m_grid.json")


def one_theta(theta):
    import oracle as orc
    from paper_2002_04894_amd import workloads as W
    x, y, z, q, w = W.workload("plummer16m")
    L = w["levels"]
    ot = orc.Tree(x, y, z, L, theta)
    perm, start = ot.perm(), ot.start(L)
    idx = np.concatenate([perm[start[b]:start[b] + PER_LEAF] for b in LEAVES])
    res = {"theta": theta, "index": [int(i) for i in idx], "orders": {}}
    for p in ORDERS:
        out = ot.evaluate(q, p, leaves=np.array(LEAVES))
        res["orders"][str(p)] = {k: [float(v) for v in a[idx]] for k, a in zip(("phi", "ex", "ey", "ez"), out)}
        print(f"theta {theta} p {p} done", flush=True)
    return res


def main():
    with Pool(len(THETAS)) as pool:
        rows = pool.map(one_theta, THETAS)
    doc = {
        "about": "Oracle (binary64) potential and field at the first 16 points (tree order) of leaves "
                 f"{list(LEAVES)} of the plummer16m workload (2^24 points, Plummer scale radius 0.05, "
                 "6 levels), per theta and order p; index = input positions of those points. "
                 "Written by make_plummer16m_grid.py.",
        "workload": "plummer16m",
        "leaves": list(LEAVES),
        "grid": rows,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
