"""The evaluation entry point that allocates nothing (fmm_evaluate_tree_noalloc):
its results against the allocating entry point (fmm_evaluate_tree_ex) on the
same tree, two calls in a row with the second on a smaller input (the fixed
scratch array keeps the first call's contents), no call to the allocator,
and its refusals (scratch too small, order's tables not made)."""
import sys

import numpy as np
import pytest

from paper_2002_04894_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def F():
    from paper_2002_04894_amd import fmm
    fmm.lib()
    yield fmm
    fmm.fmm_set_allocator()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _case(torch, F, gen, n, L, theta, p, prec, parts=3):
    x, y, z, q = gen(n, seed=n)
    X = [dev(torch, a) for a in (x, y, z)]
    qd = dev(torch, q)
    tree = F.fmm_build(*X, L, theta)
    ref = [torch.empty_like(qd) for _ in range(4)]
    F.fmm_evaluate_tree(tree, qd, p, *ref, parts=parts, precision=prec)  # allocating path (also makes the tables)
    torch.cuda.synchronize()
    return tree, qd, [r.cpu().numpy() for r in ref]


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_allocating_entry_point_twice(torch, F, prec):
    """Two calls in a row, the second on a smaller tree: each equals the
    allocating entry point bit for bit (the same kernels and sums), and the
    allocator is never called."""
    calls = []
    cases = [(W.gaussian_mixture, 150_000, 4, 0.5, 12), (W.plummer, 9_000, 3, 0.6, 12)]
    prepared = [_case(torch, F, g, n, L, th, p, prec) for g, n, L, th, p in cases]
    F.fmm_set_allocator(lambda nb, s: calls.append(nb) or 0, lambda ptr, s: None)
    try:
        for (g, n, L, th, p), (tree, qd, ref) in zip(cases, prepared):
            say(f"[noalloc] n={n} L={L} theta={th} p={p} precision={prec}")
            out = [torch.full_like(qd, np.nan) for _ in range(4)]
            F.fmm_evaluate_tree_noalloc(tree, qd, p, *out, precision=prec)
            torch.cuda.synchronize()
            for u, v in zip(out, ref):
                assert np.array_equal(u.cpu().numpy(), v)
    finally:
        F.fmm_set_allocator()
    assert calls == []
    for tree, _, _ in prepared:
        tree.free()


def test_noalloc_near_and_far_parts(torch, F):
    tree, qd, _ = _case(torch, F, W.uniform_cube, 20_000, 3, 0.5, 10, 0)
    for parts in (1, 2):
        ref = [torch.empty_like(qd) for _ in range(4)]
        F.fmm_evaluate_tree(tree, qd, 10, *ref, parts=parts)
        out = [torch.empty_like(qd) for _ in range(4)]
        F.fmm_evaluate_tree_noalloc(tree, qd, 10, *out, parts=parts)
        torch.cuda.synchronize()
        for u, v in zip(out, ref):
            assert torch.equal(u, v)
    tree.free()


def test_noalloc_refuses_beyond_its_scratch(torch, F):
    x, y, z, q = W.uniform_cube(1 << 20, seed=1)
    X = [dev(torch, a) for a in (x, y, z)]
    qd = dev(torch, q)
    tree = F.fmm_build(*X, 5, 0.5)
    _, need = F.fmm_tree_bytes(tree, 15, 0)
    assert need > 64 << 20
    out = [torch.empty_like(qd) for _ in range(4)]
    with pytest.raises(F.FMMError) as e:
        F.fmm_evaluate_tree_noalloc(tree, qd, 15, *out)
    assert e.value.code == F.FMM_EINVAL and "scratch" in str(e.value)
    tree.free()


def test_noalloc_needs_the_order_tables(torch, F):
    """An order whose tables were never made is refused with a message; after
    one allocating evaluation at that order the call works."""
    x, y, z, q = W.uniform_cube(5000, seed=3)
    X = [dev(torch, a) for a in (x, y, z)]
    qd = dev(torch, q)
    tree = F.fmm_build(*X, 2, 0.5)
    out = [torch.empty_like(qd) for _ in range(4)]
    try:
        F.fmm_evaluate_tree_noalloc(tree, qd, 1, *out)
    except F.FMMError as e:  # not made yet in this process
        assert e.code == F.FMM_EUNSUPPORTED and "tables" in str(e)
        ref = [torch.empty_like(qd) for _ in range(4)]
        F.fmm_evaluate_tree(tree, qd, 1, *ref)
        F.fmm_evaluate_tree_noalloc(tree, qd, 1, *out)
        torch.cuda.synchronize()
        for u, v in zip(out, ref):
            assert torch.equal(u, v)
    tree.free()
