"""Parameter response of the balanced-tree FMM (Section 3.2), on the GPU.

The time of a solve at a fixed accuracy is measured while one of theta, eta
and the level count L varies and the other two stay at their defaults
(theta 0.5, eta 0.5, L 3), for point clouds of four distributions: uniform
cube, spherical Gaussian, spherical shell and helix.  For every setting the
order p is the smallest whose relative error against the direct sum
(eq. (2.1), at every point) meets the tolerance, so that settings are
compared at equal accuracy.  The solve (tree build plus binary64 evaluation)
is then timed several times, the build also on its own; each sweep is normalised by its mean time at
theta 0.5, eta 0 or one level, as the paper normalises its response curves,
and the setting of least mean time is reported per sweep and distribution.

The direct sum is itself computed on the device: a theta = 0 tree has every
pair of leaves strongly connected, so its evaluation is all P2P.  The device
work goes through the C ABI (`fmm.py`); nothing here computes.

    python -m paper_2002_04894_amd.sweep --n 100000 --repeats 4 --out sweep.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

from . import fmm, workloads
from .serve import direct_sum

DEFAULTS = {"theta": 0.5, "eta": 0.5, "levels": 3}
NORMALISE_AT = {"theta": 0.5, "eta": 0.0, "levels": 1}
THETAS = tuple(round(0.05 * k, 2) for k in range(17))      # 0 .. 0.8
ETAS = tuple(round(0.1 * k, 1) for k in range(11))         # 0 .. 1
LEVELS = (1, 2, 3, 4)
LEVELS_GAUSSIAN = (1, 2, 3, 4, 5)                          # the Gaussian has one more
PMAX = 20


def plan(dist: str, thetas=THETAS, etas=ETAS, levels=None) -> list[dict]:
    """The settings of the three one-parameter sweeps of one distribution."""
    if levels is None:
        levels = LEVELS_GAUSSIAN if dist == "gaussian" else LEVELS
    rows = []
    for sweep, values in (("theta", thetas), ("eta", etas), ("levels", levels)):
        for v in values:
            s = dict(DEFAULTS)
            s[sweep] = v
            rows.append({"dist": dist, "sweep": sweep, **s})
    return rows


def rel_error(out, ref) -> float:
    """max of the relative 2-norm errors of the potential and of the field."""
    import torch
    e_phi = float(torch.linalg.norm(out[0] - ref[0]) / torch.linalg.norm(ref[0]))
    num = sum(float(torch.sum((a - b) ** 2)) for a, b in zip(out[1:], ref[1:]))
    den = sum(float(torch.sum(b ** 2)) for b in ref[1:])
    return max(e_phi, math.sqrt(num / den))


def smallest_order(tree, q, ref, tol: float, out, stream=None, pmax: int = PMAX):
    """(p, error) for the smallest p in 0..pmax whose error meets tol, else
    (None, error at pmax)."""
    import torch
    err = math.inf
    for p in range(pmax + 1):
        fmm.fmm_evaluate_tree(tree, q, p, *out, stream)
        torch.cuda.synchronize()
        err = rel_error(out, ref)
        if err <= tol:
            return p, err
    return None, err


def time_solve(dev, levels: int, theta: float, eta: float, p: int, repeats: int, out, stream=None):
    """Wall times of build + evaluation (binary64) and of the build alone,
    after one warm-up solve."""
    import torch
    x, y, z, q = dev
    times, builds = [], []
    for k in range(repeats + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tree = fmm.fmm_build_ex(x, y, z, levels, theta, eta=eta, stream=stream)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        fmm.fmm_evaluate_tree(tree, q, p, *out, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tree.free()
        if k > 0:
            times.append(t1 - t0)
            builds.append(tb - t0)
    return times, builds


def normalise(rows: list[dict]) -> list[dict]:
    """Adds norm_mean/min/max: each sweep of each distribution divided by its
    mean time at the NORMALISE_AT value (rows without a time are left as
    they are)."""
    ref = {}
    for r in rows:
        if r.get("mean") is not None and r[r["sweep"]] == NORMALISE_AT[r["sweep"]]:
            ref[(r["dist"], r["sweep"])] = r["mean"]
    for r in rows:
        m = ref.get((r["dist"], r["sweep"]))
        if r.get("mean") is None or m is None:
            continue
        r["norm_mean"] = r["mean"] / m
        r["norm_min"] = r["min"] / m
        r["norm_max"] = r["max"] / m
    return rows


def optima(rows: list[dict]) -> dict:
    """{dist: {sweep: (best value, spread)}}: the value of least mean time
    and the spread max(mean)/min(mean) - 1 of the sweep's timed settings."""
    best: dict = {}
    for r in rows:
        if r.get("mean") is None:
            continue
        d = best.setdefault(r["dist"], {}).setdefault(r["sweep"], [None, math.inf, 0.0])
        if r["mean"] < d[1]:
            d[0], d[1] = r[r["sweep"]], r["mean"]
        d[2] = max(d[2], r["mean"])
    return {k: {s: (v[0], v[2] / v[1] - 1.0) for s, v in sw.items()} for k, sw in best.items()}


def run(n: int = 100_000, tol: float = 1e-6, repeats: int = 4, dists=None, thetas=THETAS, etas=ETAS,
        levels=None, seed: int = 0, pmax: int = PMAX, log=None) -> list[dict]:
    import torch
    log = log or (lambda s: print(s, file=sys.stderr, flush=True))
    dists = dists or tuple(workloads.RESPONSE_DISTRIBUTIONS)
    rows = []
    for dist in dists:
        x, y, z, q = workloads.RESPONSE_DISTRIBUTIONS[dist](n, seed=seed)
        dev = [torch.from_numpy(a).to("cuda") for a in (x, y, z, q)]
        ref = direct_sum(*dev)
        torch.cuda.synchronize()
        out = [torch.empty_like(dev[0]) for _ in range(4)]
        for s in plan(dist, thetas, etas, levels):
            tree = fmm.fmm_build_ex(*dev[:3], s["levels"], s["theta"], eta=s["eta"])
            s["p"], s["err"] = smallest_order(tree, dev[3], ref, tol, out, pmax=pmax)
            tree.free()
            if s["p"] is None:
                s["mean"] = s["min"] = s["max"] = None
            else:
                t, b = time_solve(dev, s["levels"], s["theta"], s["eta"], s["p"], repeats, out)
                s["times"], s["build_times"] = t, b
                s["mean"], s["min"], s["max"] = sum(t) / len(t), min(t), max(t)
                s["build"] = sum(b) / len(b)
            rows.append(s)
            ms = "-" if s["mean"] is None else f"{1e3 * s['mean']:.2f} ms (build {1e3 * s['build']:.2f} ms)"
            log(f"[sweep] {dist} {s['sweep']}: theta {s['theta']} eta {s['eta']} L {s['levels']}"
                f" -> p {s['p']} err {s['err']:.2e} {ms}")
        del dev, ref, out
    return normalise(rows)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--repeats", type=int, default=4)
    ap.add_argument("--dists", default=",".join(workloads.RESPONSE_DISTRIBUTIONS))
    ap.add_argument("--levels", default=None, help="level counts of the level sweep, e.g. 3,4,5,6")
    ap.add_argument("--out", default=None, help="write every row as JSON here")
    a = ap.parse_args(argv)
    levels = tuple(int(v) for v in a.levels.split(",")) if a.levels else None
    rows = run(a.n, a.tol, a.repeats, dists=tuple(a.dists.split(",")), levels=levels)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)
    for dist, sw in optima(rows).items():
        print(json.dumps({"dist": dist, **{k: {"best": v[0], "spread": round(v[1], 4)} for k, v in sw.items()}}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
