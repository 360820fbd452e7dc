"""Serving loop for streams of N-body solves, with a parameter tuner.

A request carries a point cloud with charges and a requested relative
accuracy.  The server admits requests in arrival order as soon as a worker is
free and the device-memory estimate of the request (`fmm_bytes_estimate`)
fits in the budget next to the requests already on the device: continuous
batching, not a queue drained one at a time.  Every worker owns a HIP stream,
so the solves of different requests overlap on the GPU.  Each request's
result depends only on its own data and parameters (the solver is
deterministic), so it is the same alone and in the mix.

The tuner picks (levels, theta, p, precision) per request:
  * levels: about kPointsPerLeaf points per leaf (8^levels leaves);
  * theta: fixed (the paper's optimum lies near 0.5 for these distributions,
    Section 3.2);
  * p: the smallest order whose modelled error is below the requested
    accuracy, the model being the worst error measured on the GPU against
    direct sums (a theta = 0 tree is the direct sum) on sample clouds of the
    served distributions at orders 1..16, extended geometrically in p (the
    convergence of Section 3.1);
  * precision: the mixed mode (binary32 M2L) when the requested accuracy is
    1e-6 or looser, binary64 otherwise.

The device work goes through the C ABI (`fmm.py`); nothing here computes.
"""
from __future__ import annotations

import math
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import fmm, workloads

DISTRIBUTIONS = ("uniform", "gmix", "sphere")

@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the stream
    dist: str
    n: int
    tol: float
    seed: int


@dataclass
class Result:
    rid: int
    arrival: float
    start: float = 0.0
    done: float = 0.0
    params: tuple = ()
    bytes_est: int = 0
    outputs: list = field(default_factory=list)  # phi, ex, ey, ez (host), when kept
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_stream(nreq: int = 4000, rate: float = 200.0, nmin: float = 1e3, nmax: float = 2e5,
                seed: int = 2) -> list[Request]:
    """Poisson arrivals at `rate` per second, N log-uniform in [nmin, nmax],
    distribution uniform over DISTRIBUTIONS, accuracy 1e-4 or 1e-8 with equal
    probability; the data of request i is drawn with seed 1000 + i."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, nreq)
    arr = np.cumsum(gaps) - gaps[0]
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nreq))).astype(np.int64)
    ds = rng.integers(0, len(DISTRIBUTIONS), nreq)
    tols = np.where(rng.random(nreq) < 0.5, 1e-4, 1e-8)
    return [Request(i, float(arr[i]), DISTRIBUTIONS[ds[i]], int(ns[i]), float(tols[i]), 1000 + i)
            for i in range(nreq)]


def request_points(req: Request):
    """(x, y, z, q) of a request."""
    if req.dist == "uniform":
        return workloads.uniform_cube(req.n, seed=req.seed)
    if req.dist == "gmix":
        return workloads.gaussian_mixture(req.n, seed=req.seed)
    if req.dist == "sphere":
        return workloads.sphere_surface(req.n, seed=req.seed)
    raise ValueError(req.dist)


def direct_sum(x, y, z, q, stream=None):
    """The direct sum of eq. (2.1) on the device: with theta = 0 every pair
    of leaves is strongly connected, so the evaluation is all P2P (no
    expansions); a few levels spread it over many work items."""
    n = x.numel()
    levels = 0 if n < 512 else min(3, int(math.log(n / 64, 8)))
    return fmm.evaluate(x, y, z, q, levels, 0.0, 0, stream)


class Tuner:
    """Parameter choice from (n, tol); see the module docstring.

    The expansion order comes from measured errors: errors[p] is the largest
    relative error (potential or field) of the FMM against the direct sum at
    order p over calibration clouds of the served distributions.  Between and
    beyond the calibrated orders the error is extended geometrically (the
    convergence of Section 3.1 is geometric in p), and the model is made
    non-increasing in p.  The order for an accuracy tol is the smallest p with
    kSafety * model(p) <= tol, else pmax."""

    kPointsPerLeaf = 40.0
    kSafety = 2.0

    def __init__(self, theta: float = 0.5, errors: dict | None = None, pmax: int = fmm.FMM_MAX_ORDER):
        self.theta = theta
        self.errors = dict(errors) if errors else None
        self.pmax = pmax

    def levels(self, n: int) -> int:
        if n <= self.kPointsPerLeaf:
            return 0
        return int(min(fmm.FMM_MAX_LEVELS, max(0, round(math.log(n / self.kPointsPerLeaf, 8)))))

    def _raw(self, p: int) -> float:
        ps = sorted(self.errors)
        if p in self.errors:
            return self.errors[p]
        if len(ps) == 1:
            return self.errors[ps[0]] if p > ps[0] else math.inf
        # geometric inter- or extrapolation between the two nearest calibrated orders
        if p < ps[0]:
            a, b = ps[0], ps[1]
        elif p > ps[-1]:
            a, b = ps[-2], ps[-1]
        else:
            b = next(q for q in ps if q > p)
            a = max(q for q in ps if q < p)
        ea, eb = max(self.errors[a], 1e-300), max(self.errors[b], 1e-300)
        rate = (eb / ea) ** (1.0 / (b - a))
        return ea * rate ** (p - a)

    def model(self, p: int) -> float:
        """Modelled worst error at order p: non-increasing in p."""
        if self.errors is None:
            raise RuntimeError("the tuner is not calibrated")
        return max(self._raw(q) for q in range(p, self.pmax + 1))

    def order(self, tol: float) -> int:
        for p in range(self.pmax + 1):
            if self.kSafety * self.model(p) <= tol:
                return p
        return self.pmax

    def choose(self, n: int, tol: float) -> tuple[int, float, int, int]:
        p = self.order(tol)
        prec = fmm.FMM_PREC_MIXED if (tol >= 1e-6 and p <= 15) else fmm.FMM_PREC_F64
        return self.levels(n), self.theta, p, prec

    def calibrate(self, n: int = 20_000, orders=range(1, 17), seed: int = 7, stream=None) -> dict:
        """Measure errors[p] on the GPU: relative error (normwise, potential
        and field, the larger) of the FMM against the direct sum, the largest
        over the served distributions."""
        import torch
        table = {}
        worst: dict[int, float] = {}
        for dist in DISTRIBUTIONS:
            req = Request(-1, 0.0, dist, n, 0.0, seed)
            x, y, z, q = request_points(req)
            dev = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in (x, y, z, q)]
            ref = direct_sum(*dev, stream)
            lev = self.levels(n)
            tree = fmm.fmm_build(*dev[:3], lev, self.theta, stream)
            out = [torch.empty_like(dev[0]) for _ in range(4)]
            for p in orders:
                fmm.fmm_evaluate_tree(tree, dev[3], p, *out, stream)
                torch.cuda.synchronize()
                e_phi = float(torch.linalg.norm(out[0] - ref[0]) / torch.linalg.norm(ref[0]))
                num = sum(float(torch.sum((a - b) ** 2)) for a, b in zip(out[1:], ref[1:]))
                den = sum(float(torch.sum(b ** 2)) for b in ref[1:])
                err = max(e_phi, math.sqrt(num / den))
                table[(dist, p)] = err
                worst[p] = max(worst.get(p, 0.0), err)
            tree.free()
        self.errors = worst
        return table


class Server:
    """Continuous-batching server over `workers` HIP streams."""

    def __init__(self, tuner: Tuner, workers: int = 6, hbm_budget: int = 64 << 30, keep_outputs: bool = False):
        self.tuner = tuner
        self.workers = workers
        self.budget = hbm_budget
        self.keep = keep_outputs
        self._cv = threading.Condition()
        self._in_flight = 0
        self.peak_bytes = 0
        self.peak_concurrency = 0
        self._active = 0

    # admission: wait until the request's estimate fits next to those running
    def _admit(self, nbytes: int):
        with self._cv:
            while self._in_flight > 0 and self._in_flight + nbytes > self.budget:
                self._cv.wait()
            self._in_flight += nbytes
            self._active += 1
            self.peak_bytes = max(self.peak_bytes, self._in_flight)
            self.peak_concurrency = max(self.peak_concurrency, self._active)

    def _release(self, nbytes: int):
        with self._cv:
            self._in_flight -= nbytes
            self._active -= 1
            self._cv.notify_all()

    def solve(self, req: Request, data, stream) -> Result:
        """One request on `stream` (host data in, host results out)."""
        import torch
        res = Result(req.rid, req.arrival)
        lev, theta, p, prec = self.tuner.choose(req.n, req.tol)
        res.params = (lev, theta, p, prec)
        x, y, z, q = data
        with torch.cuda.stream(stream):
            dev = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda", non_blocking=False) for a in (x, y, z, q)]
            outs = [torch.empty_like(dev[0]) for _ in range(4)]
            tree = fmm.fmm_build(*dev[:3], lev, theta, stream)
            try:
                fmm.fmm_evaluate_tree(tree, dev[3], p, *outs, stream, precision=prec)
            finally:
                tree.free()
            host = [o.cpu() for o in outs]  # waits for this stream's work
        if self.keep:
            res.outputs = [h.numpy() for h in host]
        return res

    def run(self, requests: list[Request], realtime: bool = True) -> list[Result]:
        """Serve `requests` (sorted by arrival).  With `realtime`, a request
        becomes visible at its arrival time; latency is completion - arrival."""
        import torch
        reqs = sorted(requests, key=lambda r: r.arrival)
        ready: queue.Queue = queue.Queue(maxsize=64)
        results: list[Result] = []
        lock = threading.Lock()
        t0 = [0.0]

        def producer():
            # draws each request's data just before it arrives
            for r in reqs:
                data = request_points(r)
                if realtime:
                    delay = t0[0] + r.arrival - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                ready.put((r, data))
            for _ in range(self.workers):
                ready.put(None)

        def worker():
            stream = torch.cuda.Stream()
            while True:
                item = ready.get()
                if item is None:
                    return
                r, data = item
                lev = self.tuner.levels(r.n)
                est = int(fmm.fmm_bytes_estimate(r.n, lev, self.tuner.theta, self.tuner.order(r.tol)))
                self._admit(est)
                start = time.perf_counter() - t0[0]
                try:
                    res = self.solve(r, data, stream)
                except Exception as exc:  # reported per request
                    res = Result(r.rid, r.arrival, error=str(exc))
                finally:
                    self._release(est)
                res.start = start
                res.done = time.perf_counter() - t0[0]
                res.bytes_est = est
                if not realtime:
                    res.arrival = 0.0
                with lock:
                    results.append(res)

        t0[0] = time.perf_counter()
        threads = [threading.Thread(target=producer, daemon=True)]
        threads += [threading.Thread(target=worker, daemon=True) for _ in range(self.workers)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        return sorted(results, key=lambda r: r.rid)


def summary(results: list[Result], requests: list[Request]) -> dict:
    """p50 / p99 latency, throughput, failures."""
    ok = [r for r in results if not r.error]
    lat = np.array([r.latency for r in ok]) * 1e3
    npts = {q.rid: q.n for q in requests}
    span = max(r.done for r in ok) - min(r.arrival for r in ok) if ok else 0.0
    pts = sum(npts[r.rid] for r in ok)
    return {
        "requests": len(results),
        "failed": len(results) - len(ok),
        "p50_ms": round(float(np.percentile(lat, 50)), 3) if ok else None,
        "p99_ms": round(float(np.percentile(lat, 99)), 3) if ok else None,
        "mean_ms": round(float(lat.mean()), 3) if ok else None,
        "makespan_s": round(span, 3),
        "requests_per_s": round(len(ok) / span, 2) if span > 0 else None,
        "points_per_s": round(pts / span, 1) if span > 0 else None,
    }


def run_stream(nreq: int = 4000, rate: float = 200.0, workers: int = 6, check_every: int = 500,
               hbm_budget: int = 64 << 30) -> dict:
    """Calibrate the tuner, serve the request stream in real time, and check
    every `check_every`-th result against the direct sum (`direct_sum`,
    binary64): p50/p99 latency, throughput and the accuracy checks."""
    import torch
    tuner = Tuner()
    t0 = time.perf_counter()
    tuner.calibrate()
    cal_s = time.perf_counter() - t0
    reqs = make_stream(nreq, rate)
    srv = Server(tuner, workers=workers, hbm_budget=hbm_budget)
    results = srv.run(reqs, realtime=True)
    out = summary(results, reqs)
    out.update({"workers": workers, "hbm_budget_gb": round(hbm_budget / 2 ** 30, 1),
                "peak_concurrency": srv.peak_concurrency, "peak_bytes_gb": round(srv.peak_bytes / 1e9, 3),
                "tuner_errors": {p: float(f"{e:.3g}") for p, e in sorted(tuner.errors.items())},
                "orders": {str(t): tuner.order(t) for t in (1e-4, 1e-8)}, "calibration_s": round(cal_s, 2)})
    checks = []
    stream = torch.cuda.Stream()
    keep = Server(tuner, workers=1, keep_outputs=True)
    for r in reqs[::check_every]:
        data = request_points(r)
        got = keep.solve(r, data, stream).outputs
        dev = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in data]
        ref = [o.cpu().numpy() for o in direct_sum(*dev)]
        e_phi = float(np.linalg.norm(got[0] - ref[0]) / np.linalg.norm(ref[0]))
        e_f = float(np.linalg.norm(np.concatenate(got[1:]) - np.concatenate(ref[1:]))
                    / np.linalg.norm(np.concatenate(ref[1:])))
        checks.append({"rid": r.rid, "n": r.n, "tol": r.tol, "params": list(tuner.choose(r.n, r.tol)),
                       "err_phi": e_phi, "err_E": e_f, "ok": bool(max(e_phi, e_f) <= r.tol)})
    out["accuracy_checks"] = checks
    out["accuracy_ok"] = all(c["ok"] for c in checks)
    return out


def main(argv=None) -> int:
    """python -m paper_2002_04894_amd.serve [--requests N] [--rate R] [--workers W]:
    calibrate, serve the stream and print one JSON line."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--check-every", type=int, default=500)
    a = ap.parse_args(argv)
    print(json.dumps(run_stream(a.requests, a.rate, a.workers, a.check_every)), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
