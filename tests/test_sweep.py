"""The parameter-response sweep (Section 3.2): its plan, normalisation and
optimum rules and the four distributions on the CPU; on the GPU a small
sweep whose chosen orders are the smallest that meet the tolerance."""
import math

import numpy as np
import pytest

from paper_2002_04894_amd import sweep as S
from paper_2002_04894_amd import workloads as W
from test_gpu_parity import torch  # noqa: F401 (fixture)


def test_plan_one_parameter_at_a_time():
    rows = S.plan("cube")
    assert len(rows) == len(S.THETAS) + len(S.ETAS) + 4
    assert len(S.plan("gaussian")) == len(rows) + 1
    assert S.THETAS[0] == 0.0 and S.THETAS[-1] == 0.8 and S.ETAS[0] == 0.0 and S.ETAS[-1] == 1.0
    for r in rows:
        for k, v in S.DEFAULTS.items():
            if k != r["sweep"]:
                assert r[k] == v
    assert [r["theta"] for r in rows if r["sweep"] == "theta"] == list(S.THETAS)
    assert [r["levels"] for r in rows if r["sweep"] == "levels"] == [1, 2, 3, 4]


def _row(dist, sweep, value, times):
    r = {"dist": dist, "sweep": sweep, **S.DEFAULTS}
    r[sweep] = value
    if times is None:
        r["mean"] = r["min"] = r["max"] = None
    else:
        r["mean"], r["min"], r["max"] = sum(times) / len(times), min(times), max(times)
    return r


def test_normalise_and_optima():
    rows = [
        _row("cube", "theta", 0.4, [3.0, 5.0]),
        _row("cube", "theta", 0.5, [2.0, 2.0]),
        _row("cube", "theta", 0.8, None),              # tolerance not reached
        _row("cube", "levels", 1, [10.0, 10.0]),
        _row("cube", "levels", 3, [1.0, 3.0]),
        _row("cube", "eta", 0.5, [1.0, 1.0]),          # no eta = 0 row: no normalisation
    ]
    S.normalise(rows)
    assert rows[0]["norm_mean"] == 2.0 and rows[0]["norm_min"] == 1.5 and rows[0]["norm_max"] == 2.5
    assert rows[1]["norm_mean"] == 1.0
    assert "norm_mean" not in rows[2] and "norm_mean" not in rows[5]
    assert rows[4]["norm_mean"] == 0.2 and rows[4]["norm_max"] == 0.3
    opt = S.optima(rows)
    assert opt["cube"]["theta"] == (0.5, 1.0)
    assert opt["cube"]["levels"] == (3, 4.0)
    assert opt["cube"]["eta"] == (0.5, 0.0)


def test_response_distributions():
    n = 100_000
    for name, gen in W.RESPONSE_DISTRIBUTIONS.items():
        a = gen(n, seed=5)
        b = gen(n, seed=5)
        assert all(np.array_equal(u, v) for u, v in zip(a, b)), name
        assert all(u.dtype == np.float64 and u.shape == (n,) and u.flags.c_contiguous for u in a)
        assert np.all(np.abs(a[3]) <= 1.0)
    x, y, z, _ = W.spherical_gaussian(n, seed=1)
    P = np.stack([x, y, z])
    assert np.all(np.abs(P.mean(axis=1)) < 0.02) and np.all(np.abs(P.std(axis=1) - 1.0) < 0.01)
    x, y, z, _ = W.spherical_shell(n, seed=2)
    r = np.sqrt(x * x + y * y + z * z)
    assert r.min() >= 0.9 - 1e-12 and r.max() <= 1.0 + 1e-12
    # uniform in volume: the fraction inside the mid-volume radius is one half
    rm = ((0.9 ** 3 + 1.0) / 2) ** (1 / 3)
    assert abs(np.mean(r < rm) - 0.5) < 0.01
    x, y, z, _ = W.helix(n, seed=3)
    rxy = np.hypot(x, y)
    assert np.all(np.abs(rxy - 1.0) < 0.2) and np.all(np.abs(z) < 1.2)
    # the angle follows the height: 5 turns over the height 2
    ang = np.arctan2(y, x)
    want = 2 * np.pi * 5.0 * (z / 2.0 + 0.5)
    d = np.angle(np.exp(1j * (ang - want)))
    assert np.median(np.abs(d)) < 0.3


@pytest.mark.gpu
def test_small_sweep_orders_are_smallest(torch):
    """A reduced sweep on 20,000 points: every chosen order meets the
    tolerance against the direct sum and the next lower order does not."""
    from paper_2002_04894_amd import fmm
    from paper_2002_04894_amd.serve import direct_sum
    tol = 1e-6
    rows = S.run(n=20_000, tol=tol, repeats=1, dists=("shell", "helix"), thetas=(0.3, 0.5), etas=(0.0, 1.0),
                 levels=(1, 3))
    assert len(rows) == 2 * 6
    for dist in ("shell", "helix"):
        x, y, z, q = W.RESPONSE_DISTRIBUTIONS[dist](20_000, seed=0)
        dev = [torch.from_numpy(a).to("cuda") for a in (x, y, z, q)]
        ref = direct_sum(*dev)
        out = [torch.empty_like(dev[0]) for _ in range(4)]
        for r in (r for r in rows if r["dist"] == dist):
            assert r["p"] is not None and r["err"] <= tol and r["mean"] > 0
            tree = fmm.fmm_build_ex(*dev[:3], r["levels"], r["theta"], eta=r["eta"])
            fmm.fmm_evaluate_tree(tree, dev[3], r["p"], *out)
            torch.cuda.synchronize()
            assert math.isclose(S.rel_error(out, ref), r["err"], rel_tol=1e-9)
            if r["p"] > 0:
                fmm.fmm_evaluate_tree(tree, dev[3], r["p"] - 1, *out)
                torch.cuda.synchronize()
                assert S.rel_error(out, ref) > tol
            tree.free()
        norm = [r for r in rows if r["dist"] == dist and r[r["sweep"]] == S.NORMALISE_AT[r["sweep"]]]
        assert len(norm) == 3 and all(math.isclose(r["norm_mean"], 1.0) for r in norm)
