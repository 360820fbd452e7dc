"""The C-ABI boundary on the GPU: the allocator hook, failures that free
everything they allocated, exact device-memory accounting, and evaluation of
one tree on several streams."""
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


class Counting:
    """Allocator hook over torch's caching allocator that can be told to
    fail from the k-th allocation on, and records what is live."""

    def __init__(self, torch, fail_at=None):
        self.torch = torch
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}
        self.peak = 0

    def alloc(self, n, stream):
        self.calls += 1
        if self.fail_at is not None and self.calls >= self.fail_at:
            return 0
        ptr = int(self.torch.cuda.caching_allocator_alloc(n, self.torch.cuda.current_device(), stream))
        self.live[ptr] = n
        self.peak = max(self.peak, sum(self.live.values()))
        return ptr

    def free(self, ptr, stream):
        self.live.pop(ptr)
        if stream:
            self.torch.cuda.ExternalStream(stream).synchronize()
        else:
            self.torch.cuda.synchronize()
        self.torch.cuda.caching_allocator_delete(ptr)

    def bytes(self):
        return sum(self.live.values())


def _solve(torch, F, X, q, L=3, theta=0.5, p=7, prec=0):
    t = F.fmm_build(*X, L, theta)
    outs = [torch.empty_like(q) for _ in range(4)]
    F.fmm_evaluate_tree(t, q, p, *outs, precision=prec)
    torch.cuda.synchronize()
    return t, [o.cpu().numpy() for o in outs]


def test_null_allocator_gives_enomem_and_no_handle(torch, F):
    say("[boundary] NULL-returning allocator")
    x, y, z, q = W.uniform_cube(3000, seed=1)
    X = [dev(torch, a) for a in (x, y, z)]
    F.fmm_set_allocator(lambda n, s: 0, lambda p, s: None)
    try:
        with pytest.raises(F.FMMError) as e:
            F.fmm_build(*X, 3, 0.5)
        assert e.value.code == F.FMM_ENOMEM
    finally:
        F.fmm_set_allocator()


def test_failure_at_every_allocation_frees_everything(torch, F):
    """An allocator that fails at the k-th request, for every k a build and an
    evaluation make: the call fails with FMM_ENOMEM, every block it got is
    given back, and a tree that was built stays usable and freeable; once the
    allocator works again the result is bitwise the reference."""
    x, y, z, q = W.gaussian_mixture(12000, seed=4)  # one chunked bisection round, split P2P leaves
    X = [dev(torch, a) for a in (x, y, z)]
    qd = dev(torch, q)
    t0, ref = _solve(torch, F, X, qd, L=3, p=6, prec=1)
    t0.free()
    probe = Counting(torch)
    F.fmm_set_allocator(probe.alloc, probe.free)
    try:
        t, _ = _solve(torch, F, X, qd, L=3, p=6, prec=1)
        t.free()
        total = probe.calls
        assert probe.bytes() == 0
        say(f"[boundary] {total} allocations per build + evaluation; failing each in turn")
        failures = 0
        for k in range(1, total + 1):
            c = Counting(torch, fail_at=k)
            F.fmm_set_allocator(c.alloc, c.free)
            tree = None
            try:
                tree = F.fmm_build(*X, 3, 0.5)
            except F.FMMError as e:
                assert e.code == F.FMM_ENOMEM
                failures += 1
            if tree is not None:
                outs = [torch.empty_like(qd) for _ in range(4)]
                with pytest.raises(F.FMMError) as e:
                    F.fmm_evaluate_tree(tree, qd, 6, *outs, precision=1)
                assert e.value.code == F.FMM_ENOMEM
                failures += 1
                # the tree survives a failed evaluation: evaluate again with memory
                c.fail_at = None
                F.fmm_evaluate_tree(tree, qd, 6, *outs, precision=1)
                torch.cuda.synchronize()
                for u, v in zip(outs, ref):
                    assert np.array_equal(u.cpu().numpy(), v)
                tree.free()
            torch.cuda.synchronize()
            assert c.bytes() == 0, f"k={k}: {len(c.live)} blocks left"
        assert failures == total
    finally:
        F.fmm_set_allocator()


def test_tree_bytes_are_exact(torch, F):
    """fmm_tree_bytes: the tree's own bytes equal what the allocator holds
    after the build, and one evaluation's scratch peak is within the stated
    figure, at both precisions and with separate targets."""
    x, y, z, q = W.plummer(20000, seed=3)
    tx, ty, tz, _ = W.uniform_cube(3000, seed=7)
    X = [dev(torch, a) for a in (x, y, z)]
    T = [dev(torch, a) for a in (tx, ty, tz)]
    qd = dev(torch, q)
    c = Counting(torch)
    F.fmm_set_allocator(c.alloc, c.free)
    try:
        tree = F.fmm_build_ex(*X, 3, 0.5, targets=T)
        torch.cuda.synchronize()
        own = c.bytes()
        for p, prec in ((9, 0), (9, 1), (17, 0)):
            tb, eb = F.fmm_tree_bytes(tree, p, prec)
            assert tb == own
            c.peak = own
            outs = [torch.empty_like(qd) for _ in range(4)]
            F.fmm_evaluate_tree(tree, qd, p, *outs, precision=prec)
            touts = [torch.empty(3000, dtype=torch.float64, device="cuda") for _ in range(4)]
            F.fmm_evaluate_targets(tree, qd, p, *touts, precision=prec)
            torch.cuda.synchronize()
            assert c.bytes() == own
            say(f"[boundary] p={p} prec={prec}: tree {tb} B, eval peak {c.peak - own} B, stated {eb} B")
            assert c.peak - own <= eb
            assert c.peak - own >= 0.5 * eb
        tree.free()
        assert c.bytes() == 0
    finally:
        F.fmm_set_allocator()


def test_torch_allocator_budget(torch, F):
    x, y, z, q = W.uniform_cube(20000, seed=2)
    X = [dev(torch, a) for a in (x, y, z)]
    qd = dev(torch, q)
    _, ref = _solve(torch, F, X, qd)
    small = F.TorchAllocator(budget=1 << 16).install()
    try:
        with pytest.raises(F.FMMError) as e:
            _solve(torch, F, X, qd)
        assert e.value.code == F.FMM_ENOMEM
        assert small.in_use == 0
        big = F.TorchAllocator(budget=1 << 30).install()
        t, out = _solve(torch, F, X, qd)
        for u, v in zip(out, ref):
            assert np.array_equal(u, v)
        t.free()
        torch.cuda.synchronize()
        assert big.in_use == 0 and 0 < big.peak < 1 << 30
    finally:
        F.fmm_set_allocator()


def test_build_on_one_stream_evaluate_on_others(torch, F):
    """A tree built on one stream and evaluated right away on two other
    non-blocking streams (no host synchronisation in between), then freed at
    once: every result equals the single-stream one bitwise."""
    x, y, z, q = W.gaussian_mixture(60000, seed=6)
    X = [dev(torch, a) for a in (x, y, z)]
    qd = dev(torch, q)
    t, ref = _solve(torch, F, X, qd, L=4, p=9)
    t.free()
    sb = torch.cuda.Stream()
    s1 = torch.cuda.Stream()
    s2 = torch.cuda.Stream()
    torch.cuda.synchronize()
    outs1 = [torch.empty_like(qd) for _ in range(4)]
    outs2 = [torch.empty_like(qd) for _ in range(4)]
    for rep in range(3):
        tree = F.fmm_build(*X, 4, 0.5, stream=sb)
        F.fmm_evaluate_tree(tree, qd, 9, *outs1, stream=s1)
        F.fmm_evaluate_tree(tree, qd, 9, *outs2, stream=s2)
        tree.free()  # waits on the device for both evaluations
        torch.cuda.synchronize()
        for u, w, v in zip(outs1, outs2, ref):
            assert np.array_equal(u.cpu().numpy(), v)
            assert np.array_equal(w.cpu().numpy(), v)
