"""Fused small instances (f2): many built trees evaluated by one launch of a
captured HIP graph, through the entry point that allocates nothing.  Every
replay must equal the solo evaluations bit for bit, also with other eager
work and host synchronisations between the replays (the charges are changed
in place between replays too)."""
import numpy as np
import pytest

from paper_2002_04894_amd import serve, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.mark.parametrize("branches", [1, 6])
def test_graph_batch_equals_solo_evaluations(torch, branches):
    from paper_2002_04894_amd import fmm
    rng = np.random.default_rng(21)
    gens = (W.uniform_cube, W.gaussian_mixture, W.sphere_surface)
    items, trees = [], []
    for k in range(24):
        n = int(rng.integers(1500, 30000))
        x, y, z, q = gens[k % 3](n, seed=300 + k)
        X = [torch.from_numpy(a).to("cuda") for a in (x, y, z)]
        qd = torch.from_numpy(q).to("cuda")
        L = 2 if n < 8000 else 3
        p, prec = (5, 1) if k % 2 else (12, 0)
        t = fmm.fmm_build(*X, L, 0.5)
        outs = [torch.empty_like(qd) for _ in range(4)]
        items.append((t, qd, p, prec, outs))
        trees.append(t)

    def solo():
        ref = []
        for t, qd, p, prec, _ in items:
            o = [torch.empty_like(qd) for _ in range(4)]
            fmm.fmm_evaluate_tree(t, qd, p, *o, precision=prec)
            ref.append(o)
        torch.cuda.synchronize()
        return [[a.cpu().numpy() for a in o] for o in ref]

    ref = solo()  # also makes every order's tables
    batch = serve.GraphBatch(items, branches=branches)
    for rep in range(3):
        for _, _, _, _, outs in items:
            for o in outs:
                o.fill_(np.nan)
        torch.cuda.synchronize()
        batch.replay()
        torch.cuda.synchronize()
        for (_, _, _, _, outs), r in zip(items, ref):
            for u, v in zip(outs, r):
                assert np.array_equal(u.cpu().numpy(), v), f"replay {rep}"
        # eager work in between: other kernels, an allocating evaluation, new charges
        _ = torch.randn(1 << 20, device="cuda").sum()
        for t, qd, p, prec, _ in items[::5]:
            qd.mul_(-1.0)
        ref = solo()
    for t in trees:
        t.free()
