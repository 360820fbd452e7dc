"""Pins of the oracle's eta-blended splits (Section 2.1.2) and of its
evaluation at separate targets (the convergence test of Section 3.1 evaluates
at points that are not sources).

Every expected value here comes from numpy or from closed forms, never from
the oracle itself: the split plane of the first bisection from a sort, the
geometric halving at eta = 0, and direct sums at separate points written out
in numpy.
"""
import numpy as np
import pytest

from paper_2002_04894_amd import workloads as W


def direct_at(x, y, z, q, tx, ty, tz):
    """phi and E at separate points, pairs at distance zero skipped (eq. (2.1))."""
    phi = np.zeros(tx.shape[0]); E = np.zeros((3, tx.shape[0]))
    for k in range(tx.shape[0]):
        d = np.stack([tx[k] - x, ty[k] - y, tz[k] - z])
        r2 = (d * d).sum(0)
        ok = r2 > 0
        inv = 1.0 / np.sqrt(r2[ok])
        phi[k] = (q[ok] * inv).sum()
        E[:, k] = (q[ok] * inv ** 3 * d[:, ok]).sum(1)
    return phi, E[0], E[1], E[2]


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --------------------------------------------------------------------------
# eta-blended splits
# --------------------------------------------------------------------------

def test_eta_one_is_the_median_tree(orc):
    x, y, z, _ = W.gaussian_mixture(3000, seed=3)
    a = orc.Tree(x, y, z, 2, 0.5)
    b = orc.Tree(x, y, z, 2, 0.5, eta=1.0)
    assert np.array_equal(a.perm(), b.perm())
    for l in range(3):
        assert np.array_equal(a.geom(l), b.geom(l)) and np.array_equal(a.start(l), b.start(l))


@pytest.mark.parametrize("eta", [0.0, 0.3, 0.75])
def test_eta_first_plane_closed_form(orc, eta):
    """The root's first bisection: axis of the longest extent, plane
    (1 - eta) * midpoint + eta * (midpoint of the two middle coordinates),
    low side = the points strictly below the plane."""
    x, y, z, _ = W.gaussian_mixture(2001, seed=5)
    t = orc.Tree(x, y, z, 1, 0.5, eta=eta)
    P = np.stack([x, y, z])
    lo, hi = P.min(1), P.max(1)
    axis = int(np.argmax(hi - lo))
    c = np.sort(P[axis])
    m = c.shape[0] // 2
    med = 0.5 * (c[m - 1] + c[m])
    plane = (1.0 - eta) * (0.5 * (lo[axis] + hi[axis])) + eta * med
    g, s = t.geom(1), t.start(1)
    # children 0..3 are the low side of the first bisection
    assert np.all(g[0:4, 3 + axis] == plane) and np.all(g[4:8, axis] == plane)
    assert s[4] == np.count_nonzero(P[axis] < plane)


def test_eta_zero_halves_every_cell(orc):
    """eta = 0: every bisection cuts its cell at the midpoint, so each child
    cell is an eighth of its parent (Section 2.1.2: equal-size children)."""
    x, y, z, _ = W.plummer(4000, seed=2)
    L = 3
    t = orc.Tree(x, y, z, L, 0.5, eta=0.0)
    for l in range(1, L + 1):
        g, gp = t.geom(l), t.geom(l - 1)
        w = g[:, 3:6] - g[:, 0:3]
        wp = np.repeat(gp[:, 3:6] - gp[:, 0:3], 8, axis=0)
        # per axis the child extent is the parent's halved k times, k in 0..3
        ratio = w / wp
        ok = np.zeros_like(ratio, dtype=bool)
        for k in range(4):
            ok |= np.isclose(ratio, 0.5 ** k, rtol=1e-12, atol=0)
        assert np.all(ok)
        vol, volp = np.prod(w, 1), np.prod(wp, 1)
        assert np.allclose(vol, volp / 8, rtol=1e-12)


@pytest.mark.parametrize("eta", [0.0, 0.5, 0.9])
@pytest.mark.parametrize("gen", ["uniform", "plummer"])
def test_eta_tree_invariants(orc, eta, gen):
    """Points lie in their closed cells, the permutation is complete and
    every leaf keeps ascending original index (stable partitions)."""
    n, L = 3000, 2
    x, y, z, _ = (W.uniform_cube if gen == "uniform" else W.plummer)(n, seed=9)
    t = orc.Tree(x, y, z, L, 0.5, eta=eta)
    perm = t.perm()
    assert np.array_equal(np.sort(perm), np.arange(n))
    P = np.stack([x, y, z], axis=1)
    for l in range(1, L + 1):
        g, s = t.geom(l), t.start(l)
        assert s[0] == 0 and s[-1] == n and np.all(np.diff(s) >= 0)
        for b in range(g.shape[0]):
            idx = perm[s[b]:s[b + 1]]
            if l == L:
                assert np.all(np.diff(idx) > 0)
            assert np.all(P[idx] >= g[b, 0:3]) and np.all(P[idx] <= g[b, 3:6])


@pytest.mark.parametrize("eta", [0.0, 0.5])
def test_eta_fmm_reduces_to_direct_sum(orc, eta):
    x, y, z, q = W.gaussian_mixture(1200, seed=6)
    d = orc.direct(x, y, z, q)
    for L, theta in ((0, 0.5), (2, 0.0)):
        f = orc.Tree(x, y, z, L, theta, eta=eta).evaluate(q, 4)
        for u, v in zip(f, d):
            assert relerr(u, v) < 1e-13


@pytest.mark.parametrize("eta", [0.0, 0.5])
def test_eta_fmm_accuracy(orc, eta):
    x, y, z, q = W.gaussian_mixture(3000, seed=7)
    d = orc.direct(x, y, z, q)
    f = orc.Tree(x, y, z, 2, 0.5, eta=eta).evaluate(q, 10)
    assert relerr(f[0], d[0]) < 1e-6
    assert relerr(np.concatenate(f[1:]), np.concatenate(d[1:])) < 1e-6


# --------------------------------------------------------------------------
# separate evaluation targets
# --------------------------------------------------------------------------

def test_targets_widen_the_root_cell(orc):
    x, y, z, _ = W.uniform_cube(500, seed=1)
    tx, ty, tz = np.array([-0.5, 0.2]), np.array([0.3, 1.7]), np.array([0.1, 0.4])
    t = orc.Tree(x, y, z, 2, 0.5, targets=(tx, ty, tz))
    g0 = t.geom(0)[0]
    assert np.array_equal(g0[0:3], [min(x.min(), tx.min()), min(y.min(), ty.min()), min(z.min(), tz.min())])
    assert np.array_equal(g0[3:6], [max(x.max(), tx.max()), max(y.max(), ty.max()), max(z.max(), tz.max())])


def test_locate_finds_the_containing_leaf(orc):
    x, y, z, _ = W.gaussian_mixture(4000, seed=2)
    tx, ty, tz, _ = W.uniform_cube(300, seed=3)
    L = 2
    t = orc.Tree(x, y, z, L, 0.5, targets=(tx, ty, tz))
    g = t.geom(L)
    for k in range(300):
        v = np.array([tx[k], ty[k], tz[k]])
        inside = np.nonzero(np.all((v >= g[:, 0:3]) & (v <= g[:, 3:6]), axis=1))[0]
        b = t.locate(*v)
        assert b in inside
        # the first child in order at every level: the smallest containing leaf
        # index among those whose ancestors were also first choices; for a point
        # in the interior of one leaf there is just one
        if inside.shape[0] == 1:
            assert b == inside[0]
    g0 = t.geom(0)[0]
    assert t.locate(g0[3] + 1.0, g0[1], g0[2]) == -1


def test_locate_outside_root_cell(orc):
    x, y, z, _ = W.uniform_cube(200, seed=1)
    t = orc.Tree(x, y, z, 1, 0.5, targets=(np.array([0.5]), np.array([0.5]), np.array([0.5])))
    g0 = t.geom(0)[0]
    for v in ((g0[0] - 1e-9, g0[1], g0[2]), (g0[0], g0[4] + 1e-9, g0[2]), (np.nan, 0.5, 0.5)):
        assert t.locate(*v) == -1
    # the closed root cell's corners are inside
    assert t.locate(g0[0], g0[1], g0[2]) >= 0 and t.locate(g0[3], g0[4], g0[5]) >= 0


def test_targets_equal_to_sources_reproduce_source_evaluation(orc):
    x, y, z, q = W.uniform_cube(3000, seed=4)
    t = orc.Tree(x, y, z, 2, 0.5, targets=(x, y, z))
    a = t.evaluate(q, 6)
    b = t.evaluate_targets(q, 6)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("L,theta", [(0, 0.5), (2, 0.0)])
def test_targets_reduce_to_direct_sum(orc, L, theta):
    x, y, z, q = W.gaussian_mixture(1500, seed=5)
    tx, ty, tz, _ = W.uniform_cube(400, seed=6)
    # a few targets exactly on sources: their own source is skipped
    tx[:5], ty[:5], tz[:5] = x[:5], y[:5], z[:5]
    f = orc.Tree(x, y, z, L, theta, targets=(tx, ty, tz)).evaluate_targets(q, 5)
    d = direct_at(x, y, z, q, tx, ty, tz)
    for u, v in zip(f, d):
        assert relerr(u, v) < 1e-13


def test_targets_convergence_bound(orc):
    """Section 3.1: N = 1000 positive charges at random points, N separate
    random evaluation points; the relative error is bounded by
    C theta^{p+1} / (1 - theta)^2.  C is fitted at p = 1; the bound must hold
    for every larger p until the rounding floor."""
    x, y, z, q = W.uniform_cube(1000, seed=21, charges="pos")
    tx, ty, tz, _ = W.uniform_cube(1000, seed=22)
    phi0 = direct_at(x, y, z, q, tx, ty, tz)[0]
    theta = 0.5
    t = orc.Tree(x, y, z, 2, theta, targets=(tx, ty, tz))
    errs = {}
    for p in range(1, 13):
        errs[p] = np.max(np.abs((phi0 - t.evaluate_targets(q, p)[0]) / phi0))
    C = errs[1] * (1 - theta) ** 2 / theta ** 2
    for p in range(2, 13):
        assert errs[p] <= max(C * theta ** (p + 1) / (1 - theta) ** 2, 1e-14), (p, errs[p])
    assert errs[12] < 1e-6
