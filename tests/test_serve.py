"""The serving loop: request stream, tuner rules and admission (CPU), and on
the GPU a stream of overlapping requests whose results equal the same
requests solved alone."""
import math
import threading
import time

import numpy as np
import pytest

from paper_2002_04894_amd import serve


def test_stream_recipe():
    reqs = serve.make_stream(4000, 200.0, seed=2)
    assert [r.rid for r in reqs] == list(range(4000))
    arr = np.array([r.arrival for r in reqs])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    # Poisson at 200/s: 4000 arrivals span about 20 s
    assert 18.0 < arr[-1] < 22.0
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 1000 and ns.max() <= 200_000
    # log-uniform: the median is near the geometric mean of the bounds
    assert abs(math.log(np.median(ns)) - 0.5 * (math.log(1e3) + math.log(2e5))) < 0.2
    assert {r.dist for r in reqs} == set(serve.DISTRIBUTIONS)
    assert {r.tol for r in reqs} == {1e-4, 1e-8}
    assert all(r.seed == 1000 + r.rid for r in reqs)
    again = serve.make_stream(4000, 200.0, seed=2)
    assert [(r.arrival, r.n, r.dist, r.tol) for r in again] == [(r.arrival, r.n, r.dist, r.tol) for r in reqs]


SYNTH = {p: 1e-3 * 0.5 ** p for p in range(1, 17)}  # errors halving per order


def test_tuner_rules():
    t = serve.Tuner(theta=0.5, errors=SYNTH)
    # levels: about 40 points per leaf
    assert t.levels(30) == 0
    assert t.levels(320) == 1
    assert t.levels(20_000) == 3
    assert t.levels(10 ** 9) == 8
    # calibrated orders: the model is the measurement; the order is the
    # smallest with 2 * model <= tol
    for p in range(1, 17):
        assert t.model(p) == SYNTH[p]
    for tol in (1e-2, 1e-4, 1e-6):
        p = t.order(tol)
        assert 2 * t.model(p) <= tol and (p == 0 or 2 * t.model(p - 1) > tol)
    # beyond the calibrated orders: geometric extension at the last rate
    assert np.isclose(t.model(18), SYNTH[16] * 0.25, rtol=1e-12)
    assert np.isclose(t.model(0), SYNTH[1] * 2.0, rtol=1e-12)
    assert t.order(1e-8) == 18
    # unreachable accuracy: the largest order
    assert t.order(1e-30) == t.pmax
    # without measured costs the lowest precision allowed: the binary32 near
    # field for 1e-4 and looser, mixed precision for 1e-6, binary64 below
    assert t.choose(5000, 1e-4)[3] == 2 and t.choose(5000, 1e-6)[3] == 1 and t.choose(5000, 1e-8)[3] == 0
    with pytest.raises(RuntimeError):
        serve.Tuner().order(1e-4)


def test_tuner_levels_theta_and_cost():
    """Per level count and theta: a request uses the table of its own level
    count (uncalibrated depths: the worst calibrated one at or above, else the
    deepest), and among the thetas that meet the accuracy the cheapest by
    measured cost wins."""
    e3 = {p: 1e-3 * 0.5 ** p for p in range(1, 17)}
    e4 = {p: 4e-3 * 0.5 ** p for p in range(1, 17)}           # deeper tree: 4x the error
    e4s = {p: 4e-3 * 0.4 ** p for p in range(1, 17)}          # smaller theta converges faster
    errors = {(3, 0.5): e3, (4, 0.5): e4, (4, 0.4): e4s, (3, 0.4): {p: 1e-3 * 0.4 ** p for p in range(1, 17)}}
    cost = {(4, 0.5, 0): {p: 1.0 * (p + 1) ** 2 for p in range(1, 17)},
            (4, 0.4, 0): {p: 1.3 * (p + 1) ** 2 for p in range(1, 17)}}
    t = serve.Tuner(errors=errors, cost=cost)
    L, th, p, prec = t.choose(150_000, 1e-8)
    assert L == 4 and prec == 0
    assert 2 * t.model(p, 4, th) <= 1e-8
    # theta 0.5 needs p 20 (2 * 4e-3 * 0.5^20 = 7.6e-9), theta 0.4 needs p 15
    # (8.6e-9); costs 1.3 * 16^2 = 333 against 17^2 * (21/17)^3 = 545 (p 20 lies
    # beyond the measured orders), so theta 0.4 is chosen
    assert (th, p) == (0.4, 15)
    # the same accuracy at 3 levels: its own, smaller errors
    assert t.order(1e-8, 3, 0.5) < t.order(1e-8, 4, 0.5)
    # uncalibrated depths: deeper than calibrated -> the deepest table
    assert t.model(10, 6, 0.5) == e4[10]
    # shallower -> the worst calibrated table at or above it
    assert t.model(10, 2, 0.5) == max(e3[10], e4[10])


def test_tuner_binary64_only_choice():
    """allow_mixed = False keeps every candidate in binary64 and then picks
    the cheapest binary64 theta, which may differ from the mixed choice."""
    e = {p: 1e-3 * 0.5 ** p for p in range(1, 17)}
    e6 = {p: 1e-3 * 0.6 ** p for p in range(1, 17)}
    errors = {(3, 0.5): e, (3, 0.6): e6}
    cost = {(3, 0.5, 1): {p: 1.0 for p in range(1, 17)}, (3, 0.5, 0): {p: 10.0 for p in range(1, 17)},
            (3, 0.6, 1): {p: 5.0 for p in range(1, 17)}, (3, 0.6, 0): {p: 3.0 for p in range(1, 17)}}
    t = serve.Tuner(errors=errors, cost=cost)
    L, th, p, prec = t.choose(20_000, 1e-6)
    assert (L, th, prec) == (3, 0.5, 1)
    L, th, p, prec = t.choose(20_000, 1e-6, allow_mixed=False)
    assert (L, th, prec) == (3, 0.6, 0) and 2 * t.model(p, 3, 0.6) <= 1e-6


def test_tuner_model_is_monotone():
    """A measurement that rises with p (noise, or the rounding floor) must
    not let the tuner pick the lower order."""
    e = dict(SYNTH)
    e[10] = 1e-5  # larger than e[8] = 3.9e-6
    t = serve.Tuner(errors=e)
    assert t.model(8) >= 1e-5 and t.model(9) >= 1e-5
    assert all(t.model(p) >= t.model(p + 1) for p in range(0, 20))
    # without the correction order 8 would pass (2 * 3.9e-6 <= 1.5e-5) although
    # order 10 measured 1e-5; with it the first order past the bump is chosen
    assert t.order(1.5e-5) == 11


class FakeServer(serve.Server):
    """The admission logic with a solve that only sleeps (CPU).  Once its
    'tree is built' a request reports exact bytes of `exact(rid)`; requests
    listed in `fail_once` fail their first solve with FMM_ENOMEM."""

    exact = None
    fail_once = ()

    def solve(self, req, data, stream, reserve=None):
        if req.rid in self.fail_once and req.rid not in self._failed:
            self._failed.add(req.rid)
            raise serve.fmm.FMMError(serve.fmm.FMM_ENOMEM, "over budget")
        if reserve is not None and self.exact is not None:
            reserve(self.exact(req.rid))
        with self._cv:
            self.max_seen = max(getattr(self, "max_seen", 0), self._in_flight)
        time.sleep(0.001 * (1 + req.rid % 3))
        return serve.Result(req.rid, req.arrival)


class _FakeEvent:
    def __init__(self, **kw):
        pass

    def record(self, *a):
        pass


def _fake_torch(monkeypatch):
    class FakeCuda:
        Event = _FakeEvent

        @staticmethod
        def Stream():
            return None

        @staticmethod
        def synchronize():
            pass

    import types
    monkeypatch.setitem(__import__("sys").modules, "torch", types.SimpleNamespace(cuda=FakeCuda))


def test_admission_respects_budget(monkeypatch):
    monkeypatch.setattr(serve.fmm, "fmm_bytes_estimate", lambda n, l, th, p: n)
    monkeypatch.setattr(serve, "request_points", lambda r: None)
    _fake_torch(monkeypatch)
    reqs = [serve.Request(i, 0.0, "uniform", 100 + 50 * (i % 5), 1e-4, i) for i in range(60)]
    srv = FakeServer(serve.Tuner(errors=SYNTH), workers=6, hbm_budget=500)
    srv._failed = set()
    res = srv.run(reqs, realtime=False)
    assert sorted(r.rid for r in res) == list(range(60))
    assert all(not r.error for r in res)
    assert srv.peak_bytes <= 500
    assert srv.peak_concurrency >= 2  # requests overlap
    assert srv.deferred > 0
    assert srv._in_flight == 0 and srv._active == 0


def test_admission_reaccounts_exact_bytes(monkeypatch):
    """A request whose exact bytes (known after its build) exceed the
    estimate raises the reservation: later admissions see the larger total,
    and every byte is returned at the end."""
    monkeypatch.setattr(serve.fmm, "fmm_bytes_estimate", lambda n, l, th, p: 100)
    monkeypatch.setattr(serve, "request_points", lambda r: None)
    _fake_torch(monkeypatch)
    reqs = [serve.Request(i, 0.0, "uniform", 1000, 1e-4, i) for i in range(40)]
    srv = FakeServer(serve.Tuner(errors=SYNTH), workers=6, hbm_budget=450)
    srv._failed = set()
    srv.exact = lambda rid: 300 if rid % 4 == 0 else 50
    res = srv.run(reqs, realtime=False)
    assert all(not r.error for r in res)
    # the exact figures are what the server held: 300 + at most one estimate
    # in flight before a 300-byte request's build reports
    assert srv.peak_bytes >= 300
    assert srv.max_seen <= 450 + 300
    assert srv._in_flight == 0 and srv._active == 0


def test_hard_budget_failure_runs_again(monkeypatch):
    """With a hard budget a solve that fails with FMM_ENOMEM waits for the
    running requests and runs again; it is reported once, without error."""
    monkeypatch.setattr(serve.fmm, "fmm_bytes_estimate", lambda n, l, th, p: 10)
    monkeypatch.setattr(serve, "request_points", lambda r: None)
    monkeypatch.setattr(serve.fmm, "TorchAllocator", lambda budget: type("A", (), {"install": lambda self: self})())
    monkeypatch.setattr(serve.fmm, "fmm_set_allocator", lambda *a: None)
    _fake_torch(monkeypatch)
    reqs = [serve.Request(i, 0.0, "uniform", 1000, 1e-4, i) for i in range(30)]
    srv = FakeServer(serve.Tuner(errors=SYNTH), workers=4, hbm_budget=100, hard_budget=True)
    srv._failed = set()
    srv.fail_once = {3, 7, 11}
    res = srv.run(reqs, realtime=False)
    assert sorted(r.rid for r in res) == list(range(30))
    assert all(not r.error for r in res)
    assert srv.retried == 3 and sorted(r.rid for r in res if r.retries) == [3, 7, 11]
    assert srv._in_flight == 0 and srv._active == 0


@pytest.mark.gpu
def test_results_same_alone_and_in_the_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(11)
    reqs = [serve.Request(i, 0.0, serve.DISTRIBUTIONS[i % 3], int(rng.integers(1000, 30_000)),
                          (1e-4, 1e-8)[i % 2], 5000 + i) for i in range(24)]
    tuner = serve.Tuner(errors=SYNTH)  # p 5 (binary32 near field) for 1e-4, p 18 (binary64) for 1e-8
    mixed = serve.Server(tuner, workers=6, keep_outputs=True).run(reqs, realtime=False)
    alone = serve.Server(tuner, workers=1, keep_outputs=True)
    stream = torch.cuda.Stream()
    for r, m in zip(reqs, mixed):
        assert not m.error, m.error
        a = alone.solve(r, serve.request_points(r), stream)
        for u, v in zip(a.outputs, m.outputs):
            assert np.array_equal(u, v)



def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.gpu
def test_served_results_match_the_oracle(orc):
    """Every served result against the CPU oracle at the parameters the tuner
    chose for it (same tree, lists and order): binary64 requests within
    1e-12, binary32-near-field ones (FMM_PREC_F32) within 1e-4, normwise over
    the points of sampled leaves.  Sizes lie on both sides of the chunked
    bisection thresholds (8192, 16384); accuracies 1e-4 (binary32 near field,
    p 5) and 1e-8 (binary64, p 18, the vector M2L) with the synthetic error
    table."""
    torch = _gpu()
    sizes = [3000, 8100, 8300, 12000, 16300, 17000, 21000]
    reqs = [serve.Request(i, 0.0, serve.DISTRIBUTIONS[i % 3], n, tol, 7000 + i)
            for i, (n, tol) in enumerate((n, tol) for n in sizes for tol in (1e-4, 1e-8))]
    tuner = serve.Tuner(errors=SYNTH)
    res = serve.Server(tuner, workers=4, keep_outputs=True).run(reqs, realtime=False)
    for r, got in zip(reqs, res):
        assert not got.error, got.error
        L, theta, p, prec = got.params
        x, y, z, q = serve.request_points(r)
        t = orc.Tree(x, y, z, L, theta)
        leaves = np.unique(np.linspace(0, 8 ** L - 1, 6).astype(np.int64))
        ref = t.evaluate(q, p, leaves=leaves)
        s, perm = t.start(L), t.perm()
        pts = np.concatenate([perm[s[b]:s[b + 1]] for b in leaves])
        tol = {0: 1e-12, 1: 1e-6, 2: 1e-4}[prec]
        print(f"[serve-oracle] rid {r.rid} n {r.n} L {L} theta {theta} p {p} prec {prec}", flush=True)
        for u, v in zip(got.outputs, ref):
            err = np.linalg.norm(u[pts] - v[pts]) / np.linalg.norm(v[pts])
            assert err <= tol, (r.rid, err)


@pytest.mark.gpu
def test_hard_budget_defers_and_results_unchanged():
    """A device budget of about two requests: admission has to defer, the
    library's allocations stay within the budget, and every result equals the
    same request solved alone."""
    torch = _gpu()
    rng = np.random.default_rng(5)
    reqs = [serve.Request(i, 0.0, serve.DISTRIBUTIONS[i % 3], int(rng.integers(20_000, 60_000)),
                          1e-4, 8000 + i) for i in range(16)]
    tuner = serve.Tuner(errors=SYNTH)
    alone = serve.Server(tuner, workers=1, keep_outputs=True)
    stream = torch.cuda.Stream()
    ref = [alone.solve(r, serve.request_points(r), stream) for r in reqs]
    budget = 2 * max(r.bytes_exact for r in ref)
    srv = serve.Server(tuner, workers=6, keep_outputs=True, hbm_budget=budget, hard_budget=True)
    res = srv.run(reqs, realtime=False)
    print(f"[serve-budget] budget {budget} B, deferred {srv.deferred}, retried {srv.retried}, "
          f"peak {srv.peak_bytes} B, library peak {srv._alloc.peak} B", flush=True)
    assert srv.deferred > 0
    assert srv._alloc.peak <= budget and srv._alloc.in_use == 0
    for a, m in zip(ref, res):
        assert not m.error, m.error
        for u, v in zip(a.outputs, m.outputs):
            assert np.array_equal(u, v)


@pytest.mark.gpu
def test_served_solves_overlap_on_the_device():
    """With several workers the solves of different requests run on the
    device at the same time (device timestamps of each solve)."""
    _gpu()
    rng = np.random.default_rng(9)
    reqs = [serve.Request(i, 0.0, serve.DISTRIBUTIONS[i % 3], int(rng.integers(30_000, 100_000)),
                          1e-4, 9000 + i) for i in range(24)]
    res = serve.Server(serve.Tuner(errors=SYNTH), workers=6).run(reqs, realtime=False)
    ov = serve.device_overlap(res)
    print(f"[serve-overlap] {ov}", flush=True)
    assert ov["max_concurrent"] >= 2 and ov["overlap_frac"] > 0.2
