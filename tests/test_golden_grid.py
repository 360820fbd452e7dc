"""The stored oracle values of the 2^24-point Plummer grid (CPU): complete,
finite, and converging in p at every theta as Section 3.1 describes (the
change from p 12 to 16 is less than a tenth of that from 8 to 12), with the same sampled
points at every theta (the tree does not depend on theta)."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plummer16m_grid.json")


def test_plummer16m_grid_golden():
    with open(GOLDEN) as f:
        doc = json.load(f)
    grid = doc["grid"]
    assert sorted(r["theta"] for r in grid) == [0.4, 0.5, 0.6]
    idx = grid[0]["index"]
    assert len(idx) == 48 and len(set(idx)) == 48 and all(0 <= i < 1 << 24 for i in idx)
    for r in grid:
        assert r["index"] == idx
        v = {p: np.array([r["orders"][str(p)][k] for k in ("phi", "ex", "ey", "ez")]) for p in (8, 12, 16)}
        assert all(np.all(np.isfinite(a)) for a in v.values())
        # positive charges: the potential is positive everywhere
        assert np.all(v[16][0] > 0)
        d1 = np.linalg.norm(v[12] - v[8]) / np.linalg.norm(v[16])
        d2 = np.linalg.norm(v[16] - v[12]) / np.linalg.norm(v[16])
        assert d2 < d1 / 10, (r["theta"], d1, d2)


GOLDEN134 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plummer134m_leaves.json")


def test_plummer134m_leaves_golden():
    """The stored oracle values of the 2^27-point cloud (CPU): complete and
    finite; every sampled leaf holds 64 points (2^27 over 8^7 leaves, the
    closed form of the median splits) at consecutive tree positions 64 b;
    and the settings, each within about 1e-6 of the true potential and
    field, agree with each other to that order (theta 0.6 at p 12 and 13:
    the change is below 1e-6 relative)."""
    with open(GOLDEN134) as f:
        doc = json.load(f)
    leaves = doc["leaves"]
    assert len(doc["points"]) == len(leaves) == len(doc["start"])
    for b, s0, pts in zip(leaves, doc["start"], doc["points"]):
        assert s0 == 64 * b and len(pts) == 64 and len(set(pts)) == 64
        assert pts == sorted(pts) and all(0 <= i < 1 << 27 for i in pts)
    npts = 64 * len(leaves)
    vals = {}
    for st in doc["settings"]:
        v = np.array([st[k] for k in ("phi", "ex", "ey", "ez")])
        assert v.shape == (4, npts) and np.all(np.isfinite(v))
        assert all(c > 0 for c in st["chain_weak_pairs"][2:])  # levels 3..7 all contribute M2L
        vals[(st["theta"], st["p"])] = v
    a, b = vals[(0.6, 12)], vals[(0.6, 13)]
    for k in range(4):
        assert np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k]) < 2e-6
    c = vals[(0.5, 12)]
    for k in range(4):
        assert np.linalg.norm(c[k] - b[k]) / np.linalg.norm(b[k]) < 2e-6
