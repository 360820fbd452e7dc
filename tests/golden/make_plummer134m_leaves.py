"""Writes plummer134m_leaves.json: the oracle's potential and field at every
point of five sampled leaves of the 2^27-point Plummer workload (scale
radius 0.02, charges in [-1, 1], 7 levels), for several (theta, p), in
binary64, together with those leaves' point sets and cells.

The full interaction lists of this tree do not fit in host memory (about
2e10 weak pairs at theta 0.5), so the oracle runs in targeted mode: the whole
tree and the whole upward pass (P2M, M2M), but lists, M2L and L2L only along
the chains of the sampled leaves, and L2P + P2P at their points -- the same
arithmetic as the full evaluation at those leaves (a CPU test pins this
equality on smaller trees).  M2L uses the rotational form, pinned against the
basic form.  Calls only the oracle and the seeded input generator.

    python tests/golden/make_plummer134m_leaves.py    # about 20 minutes on 8 cores, ~25 GB of memory
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

SETTINGS = ((0.6, 13), (0.6, 12), (0.5, 12), (0.4, 8))  # (theta, p)
LEAVES = (0, 699050, 1048576, 1398101, 2097151)          # spread over the 8^7 leaves
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plummer134m_leaves.json")


def main():
    import oracle as orc
    from paper_2002_04894_amd import workloads as W
    t0 = time.time()
    x, y, z, q, w = W.workload("plummer134m")
    L = w["levels"]
    print(f"inputs {time.time() - t0:.0f} s, {orc.set_threads(0)} threads", flush=True)
    orc.set_m2l_form(True)
    leaves = np.array(LEAVES, dtype=np.int64)
    ot = orc.Tree(x, y, z, L, SETTINGS[0][0], leaves=leaves)
    print(f"tree {time.time() - t0:.0f} s", flush=True)
    perm, start, geom = ot.perm(), ot.start(L), ot.geom(L)
    idx = [perm[start[b]:start[b + 1]] for b in LEAVES]
    allidx = np.concatenate(idx)
    doc = {
        "about": "Oracle (binary64, rotational M2L) potential and field at every point of leaves "
                 f"{list(LEAVES)} of the plummer134m workload (2^27 points, Plummer scale radius 0.02, "
                 "charges in [-1, 1], 7 levels), per (theta, p); the oracle ran in targeted mode. "
                 "Written by make_plummer134m_leaves.py.",
        "workload": "plummer134m",
        "levels": L,
        "leaves": list(LEAVES),
        "start": [int(start[b]) for b in LEAVES],
        "points": [[int(i) for i in a] for a in idx],
        "cell_hex": [[float(v).hex() for v in geom[b]] for b in LEAVES],
        "settings": [],
    }
    theta_now = SETTINGS[0][0]
    for theta, p in SETTINGS:
        if theta != theta_now:
            ot.set_theta(theta)
            theta_now = theta
        weak = []
        for l in range(1, L + 1):
            off, _ = ot.lists(l, 1)
            weak.append(int(sum(off[b // 8 ** (L - l) + 1] - off[b // 8 ** (L - l)] for b in LEAVES)))
        out = ot.evaluate(q, p, leaves=leaves)
        doc["settings"].append({"theta": theta, "p": p, "chain_weak_pairs": weak,
                                **{k: [float(v) for v in a[allidx]] for k, a in zip(("phi", "ex", "ey", "ez"), out)}})
        print(f"theta {theta} p {p}: {time.time() - t0:.0f} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(doc, f)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
