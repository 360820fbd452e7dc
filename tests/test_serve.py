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


def test_tuner_rules():
    t = serve.Tuner(theta=0.5, c=1e-3)
    # levels: about 40 points per leaf
    assert t.levels(30) == 0
    assert t.levels(320) == 1
    assert t.levels(20_000) == 3
    assert t.levels(10 ** 9) == 8
    # the order is the smallest with 2 C theta^(p+1) <= tol
    for tol in (1e-2, 1e-4, 1e-6, 1e-8):
        p = t.order(tol)
        assert 2 * t.c * 0.5 ** (p + 1) <= tol
        assert p == 0 or 2 * t.c * 0.5 ** p > tol
    assert t.order(1e-4) < t.order(1e-8)
    assert t.choose(5000, 1e-4)[3] == 1 and t.choose(5000, 1e-8)[3] == 0
    with pytest.raises(RuntimeError):
        serve.Tuner().order(1e-4)


class FakeServer(serve.Server):
    """The admission logic with a solve that only sleeps (CPU)."""

    def solve(self, req, data, stream):
        time.sleep(0.001 * (1 + req.rid % 3))
        return serve.Result(req.rid, req.arrival)


def test_admission_respects_budget(monkeypatch):
    monkeypatch.setattr(serve.fmm, "fmm_bytes_estimate", lambda n, l, th, p: n)
    monkeypatch.setattr(serve, "request_points", lambda r: None)

    class FakeCuda:
        @staticmethod
        def Stream():
            return None

    import types
    fake_torch = types.SimpleNamespace(cuda=FakeCuda)
    monkeypatch.setitem(__import__("sys").modules, "torch", fake_torch)
    reqs = [serve.Request(i, 0.0, "uniform", 100 + 50 * (i % 5), 1e-4, i) for i in range(60)]
    srv = FakeServer(serve.Tuner(c=1e-3), workers=6, hbm_budget=500)
    res = srv.run(reqs, realtime=False)
    assert sorted(r.rid for r in res) == list(range(60))
    assert all(not r.error for r in res)
    assert srv.peak_bytes <= 500
    assert srv.peak_concurrency >= 2  # requests overlap
    assert srv._in_flight == 0 and srv._active == 0


@pytest.mark.gpu
def test_results_same_alone_and_in_the_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(11)
    reqs = [serve.Request(i, 0.0, serve.DISTRIBUTIONS[i % 3], int(rng.integers(1000, 30_000)),
                          (1e-4, 1e-8)[i % 2], 5000 + i) for i in range(24)]
    tuner = serve.Tuner(c=1e-3)
    mixed = serve.Server(tuner, workers=6, keep_outputs=True).run(reqs, realtime=False)
    alone = serve.Server(tuner, workers=1, keep_outputs=True)
    stream = torch.cuda.Stream()
    for r, m in zip(reqs, mixed):
        assert not m.error, m.error
        a = alone.solve(r, serve.request_points(r), stream)
        for u, v in zip(a.outputs, m.outputs):
            assert np.array_equal(u, v)

