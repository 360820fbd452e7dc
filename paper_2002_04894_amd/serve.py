"""Serving loop for streams of N-body solves, with a parameter tuner.

A request carries a point cloud with charges and a requested relative
accuracy.  The server admits requests in arrival order as soon as a worker is
free and the device-memory estimate of the request (`fmm_bytes_estimate`)
fits in the budget next to the requests already on the device: continuous
batching, not a queue drained one at a time.  Once a request's tree is built
its reservation is replaced by the exact bytes (`fmm_tree_bytes`: the tree
plus the evaluation's scratch), which on clustered clouds can exceed the
estimate.  With `hard_budget` the library's device allocations go through a
budgeted allocator as well (`fmm.TorchAllocator`): an allocation beyond the
budget fails the solve with FMM_ENOMEM, its memory is given back, and the
request waits for running requests to finish and runs again.  Every worker
owns a HIP stream, so the solves of different requests overlap on the GPU.
Each request's result depends only on its own data and parameters (the
solver is deterministic), so it is the same alone and in the mix.

The tuner picks (levels, theta, p, precision) per request:
  * levels: about kPointsPerLeaf points per leaf (8^levels leaves), a priori;
  * theta, p and precision: the cheapest combination, by the evaluation time
    per point measured on the GPU, whose modelled error times a safety factor
    meets the requested accuracy.  The error model is the worst error
    measured against direct sums (a theta = 0 tree is the direct sum) on
    sample clouds of the served distributions, per level count and theta, at
    orders 1..16, extended geometrically in p (the convergence of Section
    3.1).  Mixed precision (binary32 M2L) is a candidate for accuracies of
    1e-6 and looser.

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
    bytes_exact: int = 0
    retries: int = 0
    dev_ms: tuple = ()  # device start and end of the solve (ms after the run's reference event)
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

    levels: about kPointsPerLeaf points per leaf (fixed a priori, as the
    paper advises).  theta, p and the precision: the cheapest choice whose
    modelled error meets the accuracy with a safety factor, from a table
    measured on the GPU (`calibrate`) for each level count and theta:
    errors[(L, theta)][p] is the worst relative error (potential or field)
    against the direct sum over sample clouds of the served distributions,
    cost[(L, theta, prec)][p] the measured evaluation time per point.  In p
    the errors are extended geometrically (the convergence of Section 3.1 is
    geometric in p) and made non-increasing; costs beyond the measured orders
    grow like (p+1)^3.  A level count that was not calibrated uses the worst
    calibrated one at or above it (deeper trees carry larger errors), else the
    deepest."""

    kPointsPerLeaf = 40.0
    kSafety = 2.0
    kMixedMinTol = 1e-6  # mixed precision adds about 1e-7 relative error
    kF32MinTol = 1e-4    # the binary32 near field adds up to a few 1e-5

    def __init__(self, theta: float = 0.5, errors: dict | None = None, cost: dict | None = None,
                 pmax: int = fmm.FMM_MAX_ORDER):
        self.theta = theta
        self.pmax = pmax
        # errors: {(L, theta): {p: err}}; a plain {p: err} applies to every L at `theta`
        if errors and all(isinstance(k, int) for k in errors):
            errors = {(None, theta): dict(errors)}
        self.errors = {k: dict(v) for k, v in errors.items()} if errors else None
        self.cost = {k: dict(v) for k, v in cost.items()} if cost else {}

    def levels(self, n: int) -> int:
        if n <= self.kPointsPerLeaf:
            return 0
        return int(min(fmm.FMM_MAX_LEVELS, max(0, round(math.log(n / self.kPointsPerLeaf, 8)))))

    def _table(self, L, theta) -> dict:
        if self.errors is None:
            raise RuntimeError("the tuner is not calibrated")
        if (None, theta) in self.errors:
            return self.errors[(None, theta)]
        if (L, theta) in self.errors:
            return self.errors[(L, theta)]
        levs = sorted(l for (l, t) in self.errors if t == theta)
        if not levs:
            raise KeyError(f"theta {theta} is not calibrated")
        above = [l for l in levs if L is not None and l >= L]
        cand = above if above else [levs[-1]]
        # the worst (largest) error of the candidate level counts, order by order
        tabs = [self.errors[(l, theta)] for l in cand]
        ps = sorted(set().union(*tabs))
        return {p: max(t.get(p, 0.0) for t in tabs) for p in ps}

    @staticmethod
    def _geometric(tab: dict, p: int) -> float:
        ps = sorted(tab)
        if p in tab:
            return tab[p]
        if len(ps) == 1:
            return tab[ps[0]] if p > ps[0] else math.inf
        if p < ps[0]:
            a, b = ps[0], ps[1]
        elif p > ps[-1]:
            a, b = ps[-2], ps[-1]
        else:
            b = next(q for q in ps if q > p)
            a = max(q for q in ps if q < p)
        ea, eb = max(tab[a], 1e-300), max(tab[b], 1e-300)
        return ea * (eb / ea) ** ((p - a) / (b - a))

    def model(self, p: int, L: int | None = None, theta: float | None = None) -> float:
        """Modelled worst error at order p: non-increasing in p."""
        tab = self._table(L, self.theta if theta is None else theta)
        return max(self._geometric(tab, q) for q in range(p, self.pmax + 1))

    def order(self, tol: float, L: int | None = None, theta: float | None = None) -> int:
        for p in range(self.pmax + 1):
            if self.kSafety * self.model(p, L, theta) <= tol:
                return p
        return self.pmax

    def _cost(self, L, theta, prec, p) -> float:
        c = None
        for key in ((L, theta, prec), (None, theta, prec)):
            if key in self.cost:
                c = self.cost[key]
                break
        if not c:
            return float(p + 1) ** 3  # no measurement: the work of the translations
        if p in c:
            return c[p]
        q = max(c) if p > max(c) else min(c)
        return c[q] * ((p + 1) / (q + 1)) ** 3

    def choose(self, n: int, tol: float, allow_mixed: bool = True) -> tuple[int, float, int, int]:
        """(levels, theta, p, precision) of least measured cost that meets
        tol; allow_mixed = False keeps every candidate in binary64."""
        L = self.levels(n)
        thetas = sorted({t for (_, t) in self.errors}) if self.errors else [self.theta]
        best = None
        for th in thetas:
            p = self.order(tol, L, th)
            precs = [fmm.FMM_PREC_F64]
            if allow_mixed and tol >= self.kMixedMinTol and p <= 15:
                precs.append(fmm.FMM_PREC_MIXED)
            if allow_mixed and tol >= self.kF32MinTol and p <= 15:
                precs.append(fmm.FMM_PREC_F32)
            # the lowest precision allowed unless a measured cost says otherwise
            for prec in precs:
                key = (self._cost(L, th, prec, p), p, th, -prec)
                if best is None or key < best[0]:
                    best = (key, (L, th, p, prec))
        return best[1]

    def calibrate(self, levels=(2, 3, 4), thetas=(0.4, 0.5), orders=range(1, 17), seed: int = 7,
                  stream=None) -> dict:
        """Measure errors and costs on the GPU: for each level count L a cloud
        of about kPointsPerLeaf * 8^L points of every served distribution, its
        direct sum, and the FMM at every theta and order (binary64; mixed
        precision timed as well up to order 10)."""
        import torch
        table = {}
        errs: dict = {}
        cost: dict = {}
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for L in levels:
            n = int(self.kPointsPerLeaf * 8 ** L)
            for dist in DISTRIBUTIONS:
                req = Request(-1, 0.0, dist, n, 0.0, seed)
                x, y, z, q = request_points(req)
                dev = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in (x, y, z, q)]
                ref = direct_sum(*dev, stream)
                out = [torch.empty_like(dev[0]) for _ in range(4)]
                for th in thetas:
                    tree = fmm.fmm_build(*dev[:3], L, th, stream)
                    for p in orders:
                        precs = [fmm.FMM_PREC_F64] + ([fmm.FMM_PREC_MIXED, fmm.FMM_PREC_F32] if p <= 10 else [])
                        for prec in precs:
                            fmm.fmm_evaluate_tree(tree, dev[3], p, *out, stream, precision=prec)  # warm
                            ev0.record()
                            fmm.fmm_evaluate_tree(tree, dev[3], p, *out, stream, precision=prec)
                            ev1.record()
                            torch.cuda.synchronize()
                            c = cost.setdefault((L, th, prec), {})
                            c[p] = max(c.get(p, 0.0), ev0.elapsed_time(ev1) * 1e-3 / n)
                            if prec != fmm.FMM_PREC_F64:
                                continue
                            e_phi = float(torch.linalg.norm(out[0] - ref[0]) / torch.linalg.norm(ref[0]))
                            num = sum(float(torch.sum((a - b) ** 2)) for a, b in zip(out[1:], ref[1:]))
                            den = sum(float(torch.sum(b ** 2)) for b in ref[1:])
                            err = max(e_phi, math.sqrt(num / den))
                            table[(L, dist, th, p)] = err
                            e = errs.setdefault((L, th), {})
                            e[p] = max(e.get(p, 0.0), err)
                    tree.free()
        self.errors = errs
        self.cost = cost
        return table


class Server:
    """Continuous-batching server over `workers` HIP streams."""

    def __init__(self, tuner: Tuner, workers: int = 6, hbm_budget: int = 64 << 30, keep_outputs: bool = False,
                 hard_budget: bool = False):
        self.tuner = tuner
        self.workers = workers
        self.budget = hbm_budget
        self.keep = keep_outputs
        self.hard = hard_budget
        self._cv = threading.Condition()
        self._in_flight = 0
        self.peak_bytes = 0
        self.peak_concurrency = 0
        self.deferred = 0   # admissions that had to wait for memory
        self.retried = 0    # solves that failed on the hard budget and ran again
        self._active = 0
        self._alloc = None
        self._ref_event = None

    # admission: wait until the request's reservation fits next to those running
    def _admit(self, nbytes: int):
        with self._cv:
            waited = False
            while self._in_flight > 0 and self._in_flight + nbytes > self.budget:
                waited = True
                self._cv.wait()
            if waited:
                self.deferred += 1
            self._in_flight += nbytes
            self._active += 1
            self.peak_bytes = max(self.peak_bytes, self._in_flight)
            self.peak_concurrency = max(self.peak_concurrency, self._active)

    # the reservation of a running request becomes its exact figure (no wait:
    # the memory is already in use; later admissions see the new total)
    def _resize(self, old: int, new: int):
        with self._cv:
            self._in_flight += new - old
            self.peak_bytes = max(self.peak_bytes, self._in_flight)
            if new < old:
                self._cv.notify_all()

    def _release(self, nbytes: int):
        with self._cv:
            self._in_flight -= nbytes
            self._active -= 1
            self._cv.notify_all()

    def solve(self, req: Request, data, stream, reserve=None) -> Result:
        """One request on `stream` (host data in, host results out).
        reserve(tree, params) -> None is called once the tree is built."""
        import torch
        res = Result(req.rid, req.arrival)
        lev, theta, p, prec = self.tuner.choose(req.n, req.tol)
        res.params = (lev, theta, p, prec)
        x, y, z, q = data
        with torch.cuda.stream(stream):
            host_in = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in (x, y, z, q)]
            dev = [h.to("cuda", non_blocking=True) for h in host_in]
            outs = [torch.empty_like(dev[0]) for _ in range(4)]
            e0 = e1 = None
            if self._ref_event is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            tree = fmm.fmm_build(*dev[:3], lev, theta, stream)
            try:
                tb, eb = fmm.fmm_tree_bytes(tree, p, prec)
                res.bytes_exact = tb + eb + 8 * 8 * req.n
                if reserve is not None:
                    reserve(res.bytes_exact)
                fmm.fmm_evaluate_tree(tree, dev[3], p, *outs, stream, precision=prec)
            finally:
                tree.free()
            if e1 is not None:
                e1.record(stream)
            host = [o.cpu() for o in outs]  # waits for this stream's work
            if e1 is not None:
                res.dev_ms = (self._ref_event.elapsed_time(e0), self._ref_event.elapsed_time(e1))
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
        if self.hard:
            self._alloc = fmm.TorchAllocator(budget=self.budget).install()
        self._ref_event = torch.cuda.Event(enable_timing=True)
        self._ref_event.record()

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
                lev, th, p, _ = self.tuner.choose(r.n, r.tol)
                est = int(fmm.fmm_bytes_estimate(r.n, lev, th, p))
                start = None
                retries = 0
                while True:
                    self._admit(est)
                    held = [est]

                    def reserve(nbytes, held=held):
                        self._resize(held[0], nbytes)
                        held[0] = nbytes

                    if start is None:
                        start = time.perf_counter() - t0[0]
                    try:
                        res = self.solve(r, data, stream, reserve)
                    except fmm.FMMError as exc:
                        res = Result(r.rid, r.arrival, error=str(exc))
                        if exc.code == fmm.FMM_ENOMEM and self.hard and retries < 100:
                            # over the hard budget: wait until the others are done
                            # (the reservation becomes the whole budget) and run again
                            self._resize(held[0], self.budget)
                            held[0] = self.budget
                            retries += 1
                            with self._cv:
                                self.retried += 1
                            self._release(held[0])
                            continue
                    except Exception as exc:  # reported per request
                        res = Result(r.rid, r.arrival, error=str(exc))
                    self._release(held[0])
                    break
                res.start = start
                res.done = time.perf_counter() - t0[0]
                res.bytes_est = est
                res.retries = retries
                if not realtime:
                    res.arrival = 0.0
                with lock:
                    results.append(res)

        t0[0] = time.perf_counter()
        threads = [threading.Thread(target=producer, daemon=True)]
        threads += [threading.Thread(target=worker, daemon=True) for _ in range(self.workers)]
        try:
            for th in threads:
                th.start()
            for th in threads:
                th.join()
        finally:
            if self.hard:
                torch.cuda.synchronize()
                fmm.fmm_set_allocator()
        return sorted(results, key=lambda r: r.rid)


class GraphBatch:
    """Many built trees evaluated by one launch of a captured HIP graph
    (small instances fused; the paper reuses a tree for new charges, Section 4).

    items: (tree, q, p, precision, outs) per instance, with q and the four
    outputs device tensors that stay alive as long as the batch.  The
    evaluations are captured once; every replay re-runs all of them with the
    current contents of the q tensors and writes the outputs.  The kernels are
    those of a solo evaluation, so the results are bitwise the same.

    branches = 1: one chain through the entry point that allocates nothing
    (fmm_evaluate_tree_noalloc; its fixed scratch array is shared, so no other
    no-allocation call may run while a replay is in flight).
    branches > 1: instance k runs on branch k % branches, the branches
    concurrently (streams forked from the capture stream and joined again);
    each branch has its own workspace, handed out during capture by an
    allocator hook (fmm_set_allocator) that the batch installs and removes
    again (the default pool is restored afterwards).

    Every order and precision must have been evaluated once through an
    allocating entry point before capture (its operator tables), and the
    trees' builds must be complete."""

    def __init__(self, items, branches: int = 1):
        import torch
        self._torch = torch
        self.items = list(items)
        self.branches = nb = max(1, min(int(branches), len(self.items)))
        self.graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        cap = torch.cuda.Stream()
        if nb == 1:
            with torch.cuda.graph(self.graph, stream=cap):
                self._enqueue()
            torch.cuda.synchronize()
            return
        # per branch: its instances' scratch, summed over one evaluation's
        # requests (at most twice the peak), plus alignment slack
        need = [0] * nb
        for k, (tree, q, p, prec, outs) in enumerate(self.items):
            need[k % nb] = max(need[k % nb], 2 * fmm.fmm_tree_bytes(tree, p, prec)[1] + (64 << 10))
        self._ws = [torch.empty(n, dtype=torch.uint8, device="cuda") for n in need]
        self._streams = [torch.cuda.Stream() for _ in range(nb)]
        base = {int(s.cuda_stream): (int(w.data_ptr()), w.numel()) for s, w in zip(self._streams, self._ws)}
        used = {h: 0 for h in base}

        def alloc(nbytes, stream):
            b0, size = base[stream]
            off = (used[stream] + 255) & ~255
            if off + nbytes > size:
                return 0
            used[stream] = off + nbytes
            return b0 + off

        fmm.fmm_set_allocator(alloc, lambda ptr, stream: None)
        try:
            with torch.cuda.graph(self.graph, stream=cap):
                for s in self._streams:
                    s.wait_stream(cap)
                for k, (tree, q, p, prec, outs) in enumerate(self.items):
                    s = self._streams[k % nb]
                    used[int(s.cuda_stream)] = 0  # the branch's previous instance is ordered before
                    fmm.fmm_evaluate_tree(tree, q, p, *outs, stream=s, precision=prec)
                for s in self._streams:
                    cap.wait_stream(s)
        finally:
            fmm.fmm_set_allocator()
        torch.cuda.synchronize()

    def _enqueue(self):
        for tree, q, p, prec, outs in self.items:
            fmm.fmm_evaluate_tree_noalloc(tree, q, p, *outs, precision=prec)

    def replay(self):
        """Enqueue every evaluation of the batch (one graph launch) on the
        current stream."""
        self.graph.replay()

    def eager(self):
        """The same evaluations launched one call at a time on the current
        stream (for comparison)."""
        for tree, q, p, prec, outs in self.items:
            fmm.fmm_evaluate_tree(tree, q, p, *outs, precision=prec)


def device_overlap(results: list[Result]) -> dict:
    """From the device start/end of every solve: the time with at least one
    solve on the device, and the share of it with two or more at once."""
    ev = []
    for r in results:
        if r.dev_ms:
            ev.append((r.dev_ms[0], 1))
            ev.append((r.dev_ms[1], -1))
    if not ev:
        return {"busy_ms": 0.0, "overlap_frac": 0.0, "max_concurrent": 0}
    ev.sort()
    busy = over = 0.0
    k = kmax = 0
    last = ev[0][0]
    for t, d in ev:
        if k >= 1:
            busy += t - last
        if k >= 2:
            over += t - last
        k += d
        kmax = max(kmax, k)
        last = t
    return {"busy_ms": round(busy, 3), "overlap_frac": round(over / busy, 4) if busy > 0 else 0.0,
            "max_concurrent": kmax}


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
        "device_overlap": device_overlap(ok),
    }


def run_stream(nreq: int = 4000, rate: float = 200.0, workers: int = 6, check_every: int = 500,
               hbm_budget: int = 64 << 30, hard_budget: bool = False) -> dict:
    """Calibrate the tuner, serve the request stream in real time, and check
    every `check_every`-th result against the direct sum (`direct_sum`,
    binary64): p50/p99 latency, throughput and the accuracy checks."""
    import torch
    tuner = Tuner()
    t0 = time.perf_counter()
    tuner.calibrate()
    cal_s = time.perf_counter() - t0
    reqs = make_stream(nreq, rate)
    srv = Server(tuner, workers=workers, hbm_budget=hbm_budget, hard_budget=hard_budget)
    results = srv.run(reqs, realtime=True)
    out = summary(results, reqs)
    out.update({"workers": workers, "hbm_budget_gb": round(hbm_budget / 2 ** 30, 1),
                "peak_concurrency": srv.peak_concurrency, "peak_bytes_gb": round(srv.peak_bytes / 1e9, 3),
                "deferred": srv.deferred, "retried": srv.retried,
                "exact_over_estimate_max": round(max((r.bytes_exact / r.bytes_est for r in results
                                                      if r.bytes_est and r.bytes_exact), default=0.0), 3),
                "tuner_errors": {f"L{l} theta{t}": {p: float(f"{e:.3g}") for p, e in sorted(v.items())}
                                 for (l, t), v in sorted(tuner.errors.items())},
                "choices": {f"n={n} tol={t:g}": list(tuner.choose(n, t)) for n in (1000, 20_000, 200_000)
                            for t in (1e-4, 1e-8)},
                "calibration_s": round(cal_s, 2)})
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
