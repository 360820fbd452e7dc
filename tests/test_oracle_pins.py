"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test ties one part of the oracle to something other than itself:
closed forms, exact invariants of IEEE arithmetic, hand-worked fixtures,
textbook identities of the expansions, published truncation bounds, and
special cases of the method that reduce to the direct sum (eq. (2.1)).
"""
import json
import os

import numpy as np
import pytest

from paper_2002_04894_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Direct sum, eq. (2.1)
# --------------------------------------------------------------------------

def test_direct_two_points_closed_form(orc):
    x = np.array([0.0, 3.0]); y = np.array([0.0, 4.0]); z = np.array([0.0, 0.0])
    q = np.array([2.0, -5.0])
    phi, ex, ey, ez = orc.direct(x, y, z, q)
    # |x0 - x1| = 5: phi_0 = q_1 / 5, E_0 = q_1 (x0 - x1) / 125
    assert phi[0] == -1.0 and phi[1] == 0.4
    assert np.allclose([ex[0], ey[0], ez[0]], [-5.0 * -3.0 / 125, -5.0 * -4.0 / 125, 0.0], rtol=1e-15, atol=0)
    assert np.allclose([ex[1], ey[1], ez[1]], [2.0 * 3.0 / 125, 2.0 * 4.0 / 125, 0.0], rtol=1e-15, atol=0)


def test_direct_three_points_closed_form(orc):
    # equilateral triangle of side 2 in the plane z = 1, unit charges
    s3 = np.sqrt(3.0)
    x = np.array([0.0, 2.0, 1.0]); y = np.array([0.0, 0.0, s3]); z = np.ones(3)
    q = np.ones(3)
    phi, ex, ey, ez = orc.direct(x, y, z, q)
    assert np.allclose(phi, 1.0, rtol=1e-15)
    # field at vertex 0 points away from the centroid (1, 1/sqrt3), magnitude 2 * cos(30deg) / 4
    mag = 2.0 * (s3 / 2.0) / 4.0
    cx, cy = 1.0, 1.0 / s3
    u = np.array([0.0 - cx, 0.0 - cy]); u /= np.linalg.norm(u)
    assert np.allclose([ex[0], ey[0], ez[0]], [mag * u[0], mag * u[1], 0.0], rtol=1e-14, atol=1e-15)


def test_direct_symmetries_bitwise(orc):
    x, y, z, q = W.uniform_cube(300, seed=11)
    a = orc.direct(x, y, z, q)
    b = orc.direct(x, y, z, -q)           # negating the charges negates everything exactly
    for u, v in zip(a, b):
        assert np.array_equal(u, -v)
    c = orc.direct(2 * x, 2 * y, 2 * z, q)  # scaling by 2: phi/2 and E/4 exactly
    assert np.array_equal(c[0], a[0] / 2)
    for k in (1, 2, 3):
        assert np.array_equal(c[k], a[k] / 4)


def test_direct_coincident_points_skipped(orc):
    x = np.array([0.0, 0.0, 1.0]); y = np.zeros(3); z = np.zeros(3); q = np.array([1.0, 7.0, 3.0])
    phi, ex, _, _ = orc.direct(x, y, z, q)
    assert phi[0] == 3.0 and phi[1] == 3.0 and phi[2] == 8.0
    assert ex[0] == -3.0 and ex[2] == 8.0


def test_direct_targets_subset(orc):
    x, y, z, q = W.uniform_cube(200, seed=5)
    full = orc.direct(x, y, z, q)
    t = np.array([3, 17, 199], dtype=np.int64)
    sub = orc.direct(x, y, z, q, targets=t)
    for u, v in zip(full, sub):
        assert np.array_equal(u[t], v)


# --------------------------------------------------------------------------
# Balanced tree by median splits (Section 2.1.2, eta = 1)
# --------------------------------------------------------------------------

def _closed_form_counts(n, levels):
    """Point counts of every box per level: each bisection gives floor(n/2) to
    the low side (Section 2.1.2: children hold about equal numbers)."""
    out = [[n]]
    cur = [n]
    for _ in range(levels):
        for _ in range(3):
            nxt = []
            for c in cur:
                nxt += [c // 2, c - c // 2]
            cur = nxt
        out.append(cur)
    return out


@pytest.mark.parametrize("n,levels", [(20_000, 3), (3001, 2), (100, 3), (1, 1), (7, 1), (0 + 5, 2)])
def test_tree_counts_closed_form(orc, n, levels):
    x, y, z, _ = W.uniform_cube(n, seed=2)
    t = orc.Tree(x, y, z, levels, 0.5)
    want = _closed_form_counts(n, levels)
    for l in range(levels + 1):
        assert list(np.diff(t.start(l))) == want[l]


def test_tree_uniform20k_leaf_counts(orc):
    x, y, z, _ = W.uniform_cube(20_000, seed=0)
    c = np.diff(orc.Tree(x, y, z, 3, 0.5).start(3))
    vals, cnt = np.unique(c, return_counts=True)
    assert list(vals) == [39, 40] and list(cnt) == [480, 32]


def test_tree_golden_8_points(orc):
    g = json.load(open(os.path.join(GOLDEN, "orb_8pts.json")))
    P = np.array(g["points"])
    t = orc.Tree(P[:, 0], P[:, 1], P[:, 2], g["levels"], 0.5)
    assert list(t.perm()) == g["perm"]
    geom = t.geom(1)
    for c, (lo, hi) in enumerate(g["child_cells"]):
        assert [float(eval(s)) for s in lo] == list(geom[c, 0:3])
        assert [float(eval(s)) for s in hi] == list(geom[c, 3:6])
    # centre and half-diagonal radius of the cells (Section 2.1.1)
    assert np.array_equal(geom[:, 6:9], 0.5 * (geom[:, 0:3] + geom[:, 3:6]))


@pytest.mark.parametrize("gen", ["uniform", "gmix", "plummer"])
def test_tree_invariants(orc, gen):
    n, L = 5000, 2
    if gen == "uniform":
        x, y, z, _ = W.uniform_cube(n, seed=4)
    elif gen == "gmix":
        x, y, z, _ = W.gaussian_mixture(n, seed=4)
    else:
        x, y, z, _ = W.plummer(n, seed=4)
    t = orc.Tree(x, y, z, L, 0.5)
    perm = t.perm()
    assert np.array_equal(np.sort(perm), np.arange(n))
    g0 = t.geom(0)
    assert np.array_equal(g0[0, 0:3], [x.min(), y.min(), z.min()])
    assert np.array_equal(g0[0, 3:6], [x.max(), y.max(), z.max()])
    P = np.stack([x, y, z], axis=1)
    for l in range(1, L + 1):
        g, s = t.geom(l), t.start(l)
        gp = t.geom(l - 1)
        vol = np.prod(g[:, 3:6] - g[:, 0:3], axis=1)
        volp = np.prod(gp[:, 3:6] - gp[:, 0:3], axis=1)
        assert np.allclose(vol.reshape(-1, 8).sum(1), volp, rtol=1e-12)
        for b in range(g.shape[0]):
            idx = perm[s[b]:s[b + 1]]
            if l == L:
                assert np.all(np.diff(idx) > 0)                 # stable: ascending original index in leaves
            assert np.all(P[idx] >= g[b, 0:3]) and np.all(P[idx] <= g[b, 3:6])
            assert np.all(g[b, 0:3] >= gp[b // 8, 0:3]) and np.all(g[b, 3:6] <= gp[b // 8, 3:6])


@pytest.mark.parametrize("n,levels", [(5, 2), (30, 2), (9, 1), (100, 3)])
def test_tree_sparse_points_inside_cells(orc, n, levels):
    """With fewer points than leaves some bisections see one point; every
    point must still lie in the closed cell of its leaf."""
    x, y, z, _ = W.gaussian_mixture(n, seed=n)
    t = orc.Tree(x, y, z, levels, 0.5)
    perm, s, g = t.perm(), t.start(levels), t.geom(levels)
    P = np.stack([x, y, z], axis=1)
    for b in range(8 ** levels):
        idx = perm[s[b]:s[b + 1]]
        assert np.all(P[idx] >= g[b, 0:3]) and np.all(P[idx] <= g[b, 3:6])


def test_tree_power_of_two_scaling(orc):
    x, y, z, _ = W.gaussian_mixture(3000, seed=9)
    a = orc.Tree(x, y, z, 2, 0.5)
    b = orc.Tree(4 * x, 4 * y, 4 * z, 2, 0.5)
    assert np.array_equal(a.perm(), b.perm())
    for l in range(3):
        assert np.array_equal(4 * a.geom(l), b.geom(l))


def test_tree_duplicates_and_negative_zero(orc):
    # all points identical: every split plane is that value, ties go by index
    x = np.full(17, 0.25); y = np.full(17, -0.0); z = np.full(17, 0.0)
    t = orc.Tree(x, y, z, 1, 0.5)
    assert np.array_equal(t.perm(), np.arange(17))
    assert list(np.diff(t.start(1))) == _closed_form_counts(17, 1)[1]
    g = t.geom(1)
    assert np.all(g[:, 9] == 0.0)
    assert not np.signbit(g[:, 0:9]).any()


# --------------------------------------------------------------------------
# theta-criterion lists (eq. (2.2) and the inheritance of Section 2.1.1)
# --------------------------------------------------------------------------

def _lattice_box_index(ix, iy, iz, L):
    b = 0
    for l in range(L):
        sh = L - 1 - l
        b = 8 * b + 4 * ((ix >> sh) & 1) + 2 * ((iy >> sh) & 1) + ((iz >> sh) & 1)
    return b


@pytest.mark.parametrize("theta", ["0.4", "0.5", "0.6"])
def test_lists_lattice_golden(orc, theta):
    """64 points at the integer lattice {0,1,2,3}^3, two levels.  By hand:
    the root cell is [0,3]^3; level-1 cells split every axis at 1.5 and are
    cubes, so each level-1 cell splits x, then y, then z, at 0.5 or 2.5.  Per
    axis the leaf cells are [0,.5], [.5,1.5], [1.5,2.5], [2.5,3] and the
    level-1 cells [0,1.5], [1.5,3].  The criterion of eq. (2.2) is then
    evaluated in 50-digit decimal arithmetic (no pair lies within 1e-20 of
    the boundary) with the inheritance rule of Section 2.1.1."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    k, L = 4, 2
    g = np.arange(k, dtype=np.float64)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    t = orc.Tree(X.ravel(), Y.ravel(), Z.ravel(), L, float(theta))
    th = Decimal(theta)
    cell_lv = {}
    edges = {1: [(0, 1.5), (1.5, 3)], 2: [(0, .5), (.5, 1.5), (1.5, 2.5), (2.5, 3)]}
    for lv in (1, 2):
        kk = 2 ** lv
        cell = {}
        for ix in range(kk):
            for iy in range(kk):
                for iz in range(kk):
                    b = _lattice_box_index(ix, iy, iz, lv)
                    cell[b] = [edges[lv][ix], edges[lv][iy], edges[lv][iz]]
        geom = t.geom(lv)
        for b, c in cell.items():
            assert list(geom[b, 0:3]) == [c[0][0], c[1][0], c[2][0]]
            assert list(geom[b, 3:6]) == [c[0][1], c[1][1], c[2][1]]
        cell_lv[lv] = cell
    def ctr_rad(c):
        ctr = [(Decimal(a) + Decimal(b)) / 2 for a, b in c]
        rad = (sum((Decimal(b) - Decimal(a)) ** 2 for a, b in c)).sqrt() / 2
        return ctr, rad
    strong_prev = {0: {0}}
    for lv in (1, 2):
        s_off, s_idx = t.lists(lv, 0)
        w_off, w_idx = t.lists(lv, 1)
        strong_now = {}
        for i in range(8 ** lv):
            ci, ri = ctr_rad(cell_lv[lv][i])
            exp_s, exp_w = [], []
            for J in sorted(strong_prev[i // 8]):
                for j in range(8 * J, 8 * J + 8):
                    cj, rj = ctr_rad(cell_lv[lv][j])
                    d = sum((a - b) ** 2 for a, b in zip(ci, cj)).sqrt()
                    lhs = max(ri, rj) + th * min(ri, rj)
                    assert i == j or abs(lhs - th * d) > Decimal("1e-20")
                    (exp_w if (i != j and d > 0 and lhs <= th * d) else exp_s).append(j)
            assert list(s_idx[s_off[i]:s_off[i + 1]]) == exp_s
            assert list(w_idx[w_off[i]:w_off[i + 1]]) == exp_w
            strong_now[i] = set(exp_s)
        strong_prev = strong_now


def test_lists_theta_equality_is_weak(orc):
    """Eq. (2.2) uses <=.  Points on the x-axis at 0, 2, 2, 6, 10, 12, 14, 16
    give leaf cells [0,1] (centre .5, radius .5) and [2,4] (centre 3, radius
    1): d = 2.5 and R + theta r = 1.25 = theta d exactly at theta = 1/2."""
    x = np.array([0.0, 2.0, 2.0, 6.0, 10.0, 12.0, 14.0, 16.0])
    t = orc.Tree(x, np.zeros(8), np.zeros(8), 1, 0.5)
    g = t.geom(1)
    assert list(g[0, [0, 3, 6, 9]]) == [0.0, 1.0, 0.5, 0.5]
    assert list(g[2, [0, 3, 6, 9]]) == [2.0, 4.0, 3.0, 1.0]
    w_off, w_idx = t.lists(1, 1)
    assert 2 in w_idx[w_off[0]:w_off[1]] and 0 in w_idx[w_off[2]:w_off[3]]
    s_off, s_idx = t.lists(1, 0)
    assert 1 in s_idx[s_off[0]:s_off[1]]          # adjacent cells stay strong


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.7])
def test_lists_invariants(orc, theta):
    x, y, z, _ = W.gaussian_mixture(4000, seed=6)
    L = 3
    t = orc.Tree(x, y, z, L, theta)
    counts = {l: np.diff(t.start(l)) for l in range(L + 1)}
    for l in range(1, L + 1):
        s_off, s_idx = t.lists(l, 0)
        w_off, w_idx = t.lists(l, 1)
        ps_off, _ = t.lists(l - 1, 0)
        nb = 8 ** l
        S = {(i, j) for i in range(nb) for j in s_idx[s_off[i]:s_off[i + 1]]}
        Wk = {(i, j) for i in range(nb) for j in w_idx[w_off[i]:w_off[i + 1]]}
        assert all((j, i) in S for (i, j) in S)            # symmetric
        assert all((j, i) in Wk for (i, j) in Wk)
        assert not (S & Wk)
        for i in range(nb):                                  # 64x rule of Algorithm 2
            assert (s_off[i + 1] - s_off[i]) + (w_off[i + 1] - w_off[i]) == 8 * (ps_off[i // 8 + 1] - ps_off[i // 8])
            assert (i, i) in S
    # coverage: every source is reached exactly once from every leaf
    n = x.shape[0]
    for leaf in range(0, 8 ** L, 37):
        tot = 0
        b = leaf
        for l in range(L, 0, -1):
            w_off, w_idx = t.lists(l, 1)
            tot += counts[l][w_idx[w_off[b]:w_off[b + 1]]].sum()
            b //= 8
        s_off, s_idx = t.lists(L, 0)
        tot += counts[L][s_idx[s_off[leaf]:s_off[leaf + 1]]].sum()
        assert tot == n


def test_lists_theta_zero_all_strong(orc):
    x, y, z, _ = W.uniform_cube(2000, seed=1)
    t = orc.Tree(x, y, z, 2, 0.0)
    for l in (1, 2):
        assert t.lists(l, 1)[1].size == 0
        assert t.lists(l, 0)[1].size == (8 ** l) ** 2


# --------------------------------------------------------------------------
# Expansions (textbook identities and truncation bounds)
# --------------------------------------------------------------------------

def _cluster(n, c, a, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3)); d /= np.linalg.norm(d, axis=1)[:, None]
    r = a * rng.random(n) ** (1 / 3)
    P = np.asarray(c) + d * r[:, None]
    return P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), rng.uniform(-1, 1, n)


@pytest.mark.parametrize("p", [0, 3, 8, 14])
def test_m2m_exact(orc, p):
    """The multipole of the child shifted to the parent centre equals the
    multipole formed directly about the parent centre (degrees <= p)."""
    x, y, z, q = _cluster(25, [0.3, -0.2, 0.1], 0.15, seed=p)
    cc = np.array([0.32, -0.17, 0.08]); cp = np.array([0.1, 0.05, 0.2])
    Mc = orc.p2m(p, cc, x, y, z, q)
    Mp = orc.p2m(p, cp, x, y, z, q)
    Ms = orc.m2m(p, Mc, cc - cp)
    assert np.abs(Ms - Mp).max() <= 1e-14 * np.abs(Mp).max()


@pytest.mark.parametrize("p", [1, 6, 12])
def test_l2l_exact(orc, p):
    """A local expansion re-centred by L2L gives the same values."""
    x, y, z, q = _cluster(10, [3.0, 1.0, -2.0], 0.5, seed=p)
    c0 = np.array([0.05, 0.0, -0.1]); c1 = c0 + np.array([0.07, -0.04, 0.11])
    L0 = orc.p2l(p, c0, x, y, z, q)
    L1 = orc.l2l(p, L0, c0 - c1)
    rng = np.random.default_rng(p)
    for _ in range(5):
        pt = c1 + 0.1 * rng.standard_normal(3)
        a = orc.l2p(p, L0, c0, pt); b = orc.l2p(p, L1, c1, pt)
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * abs(a[0]))


def test_p2m_m2p_truncation_bound(orc):
    """Multipole truncation bound: |err| <= A/(r-a) (a/r)^{p+1}, A = sum|q|."""
    a = 0.2
    x, y, z, q = _cluster(30, [0, 0, 0], a, seed=3)
    A = np.abs(q).sum()
    pt = np.array([0.5, 0.3, 0.4])
    r = np.linalg.norm(pt)
    exact = orc.direct(np.r_[x, pt[0]], np.r_[y, pt[1]], np.r_[z, pt[2]], np.r_[q, 0.0], targets=[30])[0][0]
    prev = np.inf
    for p in range(0, 16):
        M = orc.p2m(p, [0, 0, 0], x, y, z, q)
        err = abs(orc.m2p(p, M, [0, 0, 0], pt) - exact)
        bound = A / (r - a) * (a / r) ** (p + 1)
        assert err <= bound * (1 + 1e-9) + 1e-15
        prev = err


def test_m2l_l2p_single_source_bound(orc):
    """Point charge -> multipole -> local -> potential and field.  The
    potential error is below the M2L truncation bound (a = source cluster
    radius, b = target region radius, rho = centre distance) and the field
    converges to the exact field of the charges geometrically."""
    xs, ys, zs, qs = _cluster(12, [0, 0, 0], 0.25, seed=1)
    ct = np.array([1.2, -0.5, 0.6])
    M = orc.p2m(20, [0, 0, 0], xs, ys, zs, qs)
    rng = np.random.default_rng(2)
    pts = ct + 0.25 * rng.uniform(-1, 1, (6, 3)) / np.sqrt(3)
    X = np.r_[xs, pts[:, 0]]; Y = np.r_[ys, pts[:, 1]]; Z = np.r_[zs, pts[:, 2]]; Q = np.r_[qs, np.zeros(6)]
    ex = orc.direct(X, Y, Z, Q, targets=np.arange(12, 18))
    A = np.abs(qs).sum(); a = 0.25; b = 0.25; rho = np.linalg.norm(ct)
    errs = []
    for p in (2, 4, 6, 8, 10, 12):
        Lc = orc.m2l(p, M[: (p + 1) ** 2], -ct)
        vals = np.array([orc.l2p(p, Lc, ct, pt) for pt in pts])
        ephi = np.abs(vals[:, 0] - ex[0]).max()
        eE = max(np.abs(vals[:, 1] - ex[1]).max(), np.abs(vals[:, 2] - ex[2]).max(), np.abs(vals[:, 3] - ex[3]).max())
        # M2L error (Greengard-Rokhlin, Theorem 3.3 form with c = rho/(a+b) - 1)
        bound = A / (rho - a - b) * ((a + b) / rho) ** (p + 1) * 2.0
        assert ephi <= bound
        errs.append(eE)
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-6 * np.abs(ex[1]).max()


def test_m2l_matches_direct_local_expansion(orc):
    """The local expansion of the field of point charges (computed directly)
    and M2L of their multipole agree up to the multipole truncation."""
    xs, ys, zs, qs = _cluster(8, [0.1, 0.2, -0.1], 0.1, seed=4)
    cs = np.array([0.1, 0.2, -0.1]); ct = np.array([-0.9, 0.8, 0.5])
    Ld = orc.p2l(10, ct, xs, ys, zs, qs)
    for P, tol in ((30 // 2, 1e-9), (20, 1e-12)):
        M = orc.p2m(P, cs, xs, ys, zs, qs)
        Lm = orc.m2l(P, M, cs - ct)[: 11 * 11]
        assert np.abs(Lm - Ld).max() <= tol * np.abs(Ld).max()


# --------------------------------------------------------------------------
# Whole FMM: special cases and the convergence bound of Section 3.1
# --------------------------------------------------------------------------

def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_fmm_zero_levels_is_direct_sum(orc):
    x, y, z, q = W.uniform_cube(1500, seed=8)
    d = orc.direct(x, y, z, q)
    f = orc.Tree(x, y, z, 0, 0.5).evaluate(q, 6)
    for u, v in zip(f, d):
        assert _relerr(u, v) < 1e-13


def test_fmm_theta_zero_is_direct_sum(orc):
    x, y, z, q = W.gaussian_mixture(1500, seed=8)
    d = orc.direct(x, y, z, q)
    f = orc.Tree(x, y, z, 2, 0.0).evaluate(q, 3)
    for u, v in zip(f, d):
        assert _relerr(u, v) < 1e-13


def test_fmm_near_plus_far_is_total(orc):
    x, y, z, q = W.uniform_cube(1200, seed=3)
    t = orc.Tree(x, y, z, 2, 0.5)
    a = t.evaluate(q, 5, parts=1); b = t.evaluate(q, 5, parts=2); c = t.evaluate(q, 5, parts=3)
    for u, v, w in zip(a, b, c):
        assert np.allclose(u + v, w, rtol=1e-14, atol=1e-14 * np.abs(w).max())


def test_fmm_leaf_subset_matches_full(orc):
    x, y, z, q = W.gaussian_mixture(2500, seed=2)
    t = orc.Tree(x, y, z, 2, 0.5)
    full = t.evaluate(q, 6)
    leaves = np.array([0, 9, 33, 63])
    sub = t.evaluate(q, 6, leaves=leaves)
    s = t.start(2)
    pts = np.concatenate([t.perm()[s[b]:s[b + 1]] for b in leaves])
    for u, v in zip(full, sub):
        assert np.array_equal(u[pts], v[pts])
        assert np.isnan(np.delete(v, pts)).all()


def test_fmm_convergence_bound(orc):
    """Section 3.1: relative error of positive potentials is bounded by
    C theta^{p+1} / (1-theta)^2.  C is fitted at p = 1; the bound must then
    hold for every larger p until the rounding floor."""
    x, y, z, q = W.uniform_cube(1000, seed=21, charges="pos")
    tx, ty, tz, _ = W.uniform_cube(1000, seed=22)
    # evaluation at separate random points: add them as zero-charge sources
    X = np.r_[x, tx]; Y = np.r_[y, ty]; Z = np.r_[z, tz]; Q = np.r_[q, np.zeros(1000)]
    tg = np.arange(1000, 2000)
    phi0 = orc.direct(X, Y, Z, Q, targets=tg)[0]
    theta = 0.5
    t = orc.Tree(X, Y, Z, 2, theta)
    errs = {}
    for p in range(1, 13):
        phi = t.evaluate(Q, p)[0][tg]
        errs[p] = np.max(np.abs((phi0 - phi) / phi0))
    C = errs[1] * (1 - theta) ** 2 / theta ** 2
    for p in range(2, 13):
        assert errs[p] <= max(C * theta ** (p + 1) / (1 - theta) ** 2, 1e-13)
    # and the decay is geometric overall
    assert errs[12] < 1e-4 * errs[2]


def test_fmm_linear_in_charges(orc):
    x, y, z, q1 = W.uniform_cube(1000, seed=13)
    q2 = np.random.default_rng(0).uniform(-1, 1, 1000)
    t = orc.Tree(x, y, z, 2, 0.5)
    a = t.evaluate(q1, 6); b = t.evaluate(q2, 6); c = t.evaluate(q1 + 2 * q2, 6)
    for u, v, w in zip(a, b, c):
        assert np.allclose(u + 2 * v, w, rtol=0, atol=1e-12 * np.abs(w).max())


# --------------------------------------------------------------------------
# Whole FMM at three and four levels: the downward pass (Algorithm 3, L2L)
# --------------------------------------------------------------------------

def _chain_weak(t, levels, leaves):
    """Weak-list entries of the ancestors of `leaves`, per level 1..L."""
    out = {}
    for l in range(1, levels + 1):
        off, _ = t.lists(l, 1)
        anc = np.unique(np.asarray(leaves) // 8 ** (levels - l))
        out[l] = int(sum(off[a + 1] - off[a] for a in anc))
    return out


@pytest.mark.parametrize("gen,n,levels,p,theta", [
    ("cube", 4000, 3, 10, 0.5),
    ("gmix", 4000, 3, 10, 0.5),
    ("cube", 6000, 4, 12, 0.5),
    ("gmix", 6000, 4, 12, 0.5),
    ("gmix", 6000, 4, 10, 0.4),
])
def test_fmm_deep_tree_matches_direct_sum(orc, gen, n, levels, p, theta):
    """With L >= 3 the ancestors of a leaf at levels 2..L-1 hold local
    expansions of their own (weak pairs there), which reach the leaf only
    through L2L.  A wrong L2L (sign of the shift, index, missing term) leaves
    an error far above the truncation error; this is the only whole-method
    check of the downward pass on the CPU.  Every point of 12 sampled leaves
    is compared with the direct sum, eq. (2.1)."""
    make = W.uniform_cube if gen == "cube" else W.gaussian_mixture
    x, y, z, q = make(n, seed=5)
    t = orc.Tree(x, y, z, levels, theta)
    leaves = np.sort(np.random.default_rng(3).choice(8 ** levels, 12, replace=False))
    weak = _chain_weak(t, levels, leaves)
    assert any(weak[l] > 0 for l in range(2, levels)), weak
    f = t.evaluate(q, p, leaves=leaves)
    s, perm = t.start(levels), t.perm()
    pts = np.concatenate([perm[s[b]:s[b + 1]] for b in leaves])
    assert pts.size > 0
    d = orc.direct(x, y, z, q, targets=pts)
    for u, v in zip(f, d):
        assert _relerr(u[pts], v) < 1e-6
    # the far field alone is far from zero at these points: the test sees it
    far = t.evaluate(q, p, parts=2, leaves=leaves)
    assert np.linalg.norm(far[0][pts]) > 1e-2 * np.linalg.norm(d[0])


@pytest.mark.parametrize("levels,p", [(3, 12), (4, 12)])
def test_fmm_deep_tree_separate_targets_match_direct_sum(orc, levels, p):
    """The same at separate evaluation points (Section 3.1 evaluates at
    points that are not sources): L2P + P2P at the target's leaf, whose local
    expansion is built through L2L from levels 2..L-1."""
    x, y, z, q = W.gaussian_mixture(5000, seed=9)
    tx, ty, tz, _ = W.gaussian_mixture(150, seed=10)  # same cloud shape, other points
    t = orc.Tree(x, y, z, levels, 0.5, targets=(tx, ty, tz))
    leaves = np.unique([t.locate(a, b, c) for a, b, c in zip(tx, ty, tz)])
    weak = _chain_weak(t, levels, leaves)
    assert any(weak[l] > 0 for l in range(2, levels)), weak
    f = t.evaluate_targets(q, p)
    # direct sum at the targets: add them as zero-charge sources
    X = np.r_[x, tx]; Y = np.r_[y, ty]; Z = np.r_[z, tz]; Q = np.r_[q, np.zeros(tx.size)]
    d = orc.direct(X, Y, Z, Q, targets=np.arange(x.size, x.size + tx.size))
    for u, v in zip(f, d):
        assert _relerr(u, v) < 1e-6


# --------------------------------------------------------------------------
# The rotational M2L form (Section 2.1.3), threads and the targeted mode
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [0, 1, 2, 3, 7, 12, 15, 16, 20])
def test_m2l_rotational_form_equals_basic_form(orc, p):
    """Two independent derivations of the same operator: the translation
    theorem in its basic O(p^4) form against rotation onto the z-axis,
    z-translation and rotation back.  Directions include the poles (+z, -z),
    the coordinate axes and general ones."""
    rng = np.random.default_rng(100 + p)
    x, y, z = rng.uniform(-0.3, 0.3, (3, 25))
    q = rng.uniform(-1, 1, 25)
    M = orc.p2m(p, (0.0, 0.0, 0.0), x, y, z, q)
    dirs = [(0, 0, 2.5), (0, 0, -2.5), (2.2, 0, 0), (0, -2.2, 0), (1e-12, 0, 3.0), (-1.5, 1.5, 0.0)]
    dirs += [tuple(2.5 * v / np.linalg.norm(v)) for v in rng.normal(size=(6, 3))]
    for d in dirs:
        a = orc.m2l(p, M, d)
        b = orc.m2l_rot(p, M, d)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), d


def test_fmm_rotational_form_same_result(orc):
    x, y, z, q = W.gaussian_mixture(6000, seed=12)
    t = orc.Tree(x, y, z, 3, 0.5)
    leaves = np.arange(0, 512, 9)
    a = t.evaluate(q, 9, leaves=leaves)
    orc.set_m2l_form(True)
    try:
        b = t.evaluate(q, 9, leaves=leaves)
    finally:
        orc.set_m2l_form(False)
    s, perm = t.start(3), t.perm()
    pts = np.concatenate([perm[s[k]:s[k + 1]] for k in leaves])
    for u, v in zip(a, b):
        assert _relerr(v[pts], u[pts]) < 1e-13


def test_oracle_threads_do_not_change_results(orc):
    """Threads share out boxes, leaves and targets; each sum keeps its order,
    so the results are bitwise those of one thread."""
    x, y, z, q = W.plummer(9000, seed=4, charges="pm1")
    tx, ty, tz, _ = W.uniform_cube(300, seed=5)
    old = orc.set_threads(0)
    try:
        outs = []
        for nt in (1, 4):
            orc.set_threads(nt)
            t = orc.Tree(x, y, z, 3, 0.5, targets=(tx, ty, tz))
            outs.append((t.perm(), t.lists(3, 1), t.evaluate(q, 7), t.evaluate_targets(q, 7),
                         orc.direct(x, y, z, q, targets=np.arange(0, 9000, 7))))
        (pa, la, ea, ta, da), (pb, lb, eb, tb, db) = outs
        assert np.array_equal(pa, pb)
        assert np.array_equal(la[0], lb[0]) and np.array_equal(la[1], lb[1])
        for u, v in zip(ea + ta + da, eb + tb + db):
            assert np.array_equal(u, v)
    finally:
        orc.set_threads(old)


def test_targeted_mode_equals_the_full_tree(orc):
    """Targeted mode (lists only along the chains of chosen leaves): the rows
    of the chain boxes equal the full tree's, every other row is empty, the
    evaluation at the chosen leaves is bitwise the full one, and other leaves
    are refused."""
    x, y, z, q = W.plummer(30000, seed=8, charges="pm1")
    leaves = np.array([0, 77, 300, 511])
    full = orc.Tree(x, y, z, 3, 0.5)
    tg = orc.Tree(x, y, z, 3, 0.5, leaves=leaves)
    assert np.array_equal(full.perm(), tg.perm())
    for l in range(1, 4):
        anc = set((leaves // 8 ** (3 - l)).tolist())
        for kind in (0, 1):
            fo, fi = full.lists(l, kind)
            to, ti = tg.lists(l, kind)
            for b in range(8 ** l):
                row_t = ti[to[b]:to[b + 1]]
                if b in anc:
                    assert np.array_equal(row_t, fi[fo[b]:fo[b + 1]])
                else:
                    assert row_t.size == 0
    a = full.evaluate(q, 8, leaves=leaves)
    b = tg.evaluate(q, 8, leaves=leaves)
    for u, v in zip(a, b):
        assert np.array_equal(u, v, equal_nan=True)
    with pytest.raises(ValueError):
        tg.evaluate(q, 8, leaves=np.array([1]))
    with pytest.raises(ValueError):
        tg.evaluate(q, 8)
