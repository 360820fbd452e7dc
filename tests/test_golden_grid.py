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
